"""Textbook reference pieces of the solver (Sec. 7), for pinning the GPU
multigrid and preconditioner building blocks.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

* lumped inverse-viscosity pressure mass of eq:pmass (row sums, one-point rule);
* velocity transfer operators P (x) I3 and P^T built from the oracle's own
  prolongation matrix;
* the Chebyshev iteration on D^{-1} A in Saad's three-term recurrence form
  (Iterative Methods for Sparse Linear Systems, Sec. 12.3), as the paper's
  smoother "second-degree Chebyshev polynomial" reads.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .stokes import QC, StokesOracle, ref_basis, wedge_geometry


def lumped_pressure_mass(orc: StokesOracle, eta_wedge: np.ndarray) -> np.ndarray:
    """m = row sums of P^T M_f P with (M_f)_ij = sum_e (V_e / eta_e) N_i(q_c) N_j(q_c).

    Since P 1 = 1 the row sums are P^T (M_f 1)."""
    m = orc.mesh
    wn = m.wedge_nodes()
    N, _ = ref_basis(*QC)
    _, V, _ = wedge_geometry(m.node_xyz()[wn])
    mf1 = np.zeros(m.n_nodes)
    # (M_f 1)_i = sum_e (V/eta) N_i sum_j N_j
    np.add.at(mf1, wn, (V / eta_wedge)[:, None] * N[None, :] * N.sum())
    return orc.P.T @ mf1


def velocity_prolongation(orc: StokesOracle) -> sp.csr_matrix:
    """P (x) I3 in node-major / component-fastest DoF order."""
    return sp.kron(orc.P, sp.identity(3), format="csr")


def restrict_velocity(orc: StokesOracle, f: np.ndarray, coarse_boundary: np.ndarray) -> np.ndarray:
    """c = P^T f with the coarse Dirichlet rows set to zero.  f: [n_fine, 3]."""
    c = (velocity_prolongation(orc).T @ f.ravel()).reshape(-1, 3)
    c[coarse_boundary] = 0.0
    return c


def chebyshev(A: sp.spmatrix, diag: np.ndarray, b: np.ndarray, x: np.ndarray, degree: int, steps: int,
              lmin: float, lmax: float) -> np.ndarray:
    """`steps` applications of the degree-`degree` Chebyshev polynomial smoother
    for D^{-1} A x = D^{-1} b with eigenvalues assumed in [lmin, lmax]."""
    x = np.array(x, dtype=np.float64)
    theta = 0.5 * (lmax + lmin)
    delta = 0.5 * (lmax - lmin)
    sigma = theta / delta
    dinv = 1.0 / diag
    for _ in range(steps):
        r = b - A @ x
        d = dinv * r / theta
        rho = 1.0 / sigma
        x = x + d
        for _k in range(1, degree):
            r = b - A @ x
            rho_new = 1.0 / (2.0 * sigma - rho)
            d = rho_new * rho * d + (2.0 * rho_new / delta) * dinv * r
            x = x + d
            rho = rho_new
    return x
