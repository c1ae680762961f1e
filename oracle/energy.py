"""Oracle energy operator (Sec. 1 eq:energy, Boussinesq form with unit
diffusivity; Sec. 6 scheme list: SUPG-stabilised Galerkin) with the
one-point rule of Sec. 4, assembled explicitly.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Backward Euler:  (M_L / dt + K + C(u) + S(u)) T^{n+1} = M_L (T^n / dt + H),
with per wedge, at q_c:  M_L lumped (V/6 per vertex), K_ij = V grad phi_i .
grad phi_j, C_ij = V N_i(q_c) ubar . grad phi_j, S_ij = V tau (ubar . grad
phi_i)(ubar . grad phi_j); ubar = mean of the six nodal velocities; the
standard streamline-upwind parameter tau = h / (2 |ubar|) (coth Pe - 1/Pe),
Pe = |ubar| h / 2, h = V^(1/3).  Temperature Dirichlet rows on both spheres
are identity rows; their columns are kept (the boundary values enter the
interior equations).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .mesh import ShellMesh
from .stokes import QC, ref_basis, wedge_geometry


def supg_tau(unorm: np.ndarray, h: np.ndarray) -> np.ndarray:
    """tau = h/(2|u|) (coth Pe - 1/Pe), Pe = |u| h / 2; the Pe -> 0 limit h^2/12."""
    unorm = np.asarray(unorm, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    pe = 0.5 * unorm * h
    out = np.empty_like(pe)
    small = pe < 1e-3
    out[small] = h[small] ** 2 / 12.0 * (1.0 - pe[small] ** 2 / 15.0)
    p = pe[~small]
    out[~small] = h[~small] / (2.0 * unorm[~small]) * (1.0 / np.tanh(p) - 1.0 / p)
    return out


class EnergyOracle:
    def __init__(self, mesh: ShellMesh, u_nodes: np.ndarray, dt: float):
        self.mesh = m = mesh
        wn = m.wedge_nodes()
        xw = m.node_xyz()[wn]
        N, _ = ref_basis(*QC)
        _, V, g = wedge_geometry(xw)                        # g: [w, 6, 3]
        ub = u_nodes[wn].mean(axis=1)                      # [w, 3]
        un = np.linalg.norm(ub, axis=1)
        tau = supg_tau(un, np.cbrt(V))
        ug = np.einsum("wa,wja->wj", ub, g)                # ubar . grad phi_j
        K = np.einsum("wia,wja->wij", g, g)
        C = N[None, :, None] * ug[:, None, :]
        S = tau[:, None, None] * ug[:, :, None] * ug[:, None, :]
        rows = np.repeat(wn, 6, axis=1).ravel()
        cols = np.tile(wn, (1, 6)).ravel()

        def assemble(Ee):
            return sp.csr_matrix(((V[:, None, None] * Ee).ravel(), (rows, cols)), shape=(m.n_nodes, m.n_nodes))

        # the three parts separately (diffusion, advection, streamline diffusion),
        # without Dirichlet rows, and their sum
        self.K, self.C, self.S = assemble(K), assemble(C), assemble(S)
        A = assemble(K + C + S)
        ml = np.zeros(m.n_nodes)
        np.add.at(ml, wn, V[:, None] * N[None, :])
        self.mass = ml
        self.A_noD = (A + sp.diags(ml / dt)).tocsr()
        bnd = m.boundary_nodes()
        keep = sp.diags((~bnd).astype(np.float64))
        self.E = (keep @ self.A_noD + sp.diags(bnd.astype(np.float64))).tocsr()
        self.dt = dt
        self.bnd = bnd

    def apply(self, T):
        return self.E @ T

    def rhs(self, Tn, H=None, T_inner=1.0, T_outer=0.0):
        b = self.mass * (Tn / self.dt + (0.0 if H is None else H))
        k = np.tile(np.arange(self.mesh.nr + 1), self.mesh.n_lat)
        b[k == 0] = T_inner
        b[k == self.mesh.nr] = T_outer
        return b

    def step(self, Tn, H=None, T_inner=1.0, T_outer=0.0):
        return spla.spsolve(self.E.tocsc(), self.rhs(Tn, H, T_inner, T_outer))
