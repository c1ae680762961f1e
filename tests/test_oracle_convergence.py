"""Manufactured-solution convergence of the oracle (Sec. 4: the one-point
discretisation converges at the optimal rate on the assembled shell).

The paper shows the orders only in a figure, so the pin is the textbook
second order of W1 velocity in the discrete L2 norm: halving h must divide
the error by about four.  A wrong element scale, a wrong B/A ratio or a
wrong sign of B leaves an O(1) error and fails the ratio.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import sympy as s

from oracle.mesh import ShellMesh
from oracle.stokes import QC, StokesOracle, ref_basis, wedge_geometry

R_IN, R_OUT = 0.55, 1.0
X = s.symbols("x y z")


def _fields(stokes: bool):
    x, y, z = X
    r = s.sqrt(x ** 2 + y ** 2 + z ** 2)
    eta = 1 + s.Rational(1, 2) * x * z
    if stokes:
        phi = ((r - R_IN) * (R_OUT - r)) ** 2
        psi = [phi * y * z, phi * s.sin(x), phi * (x + z ** 2)]
        u = [s.diff(psi[2], y) - s.diff(psi[1], z), s.diff(psi[0], z) - s.diff(psi[2], x),
             s.diff(psi[1], x) - s.diff(psi[0], y)]           # divergence-free, zero on both spheres
        p = x * y + z ** 3
    else:
        phi = (r - R_IN) * (R_OUT - r)
        u = [phi * (s.sin(2 * y) + z), phi * s.cos(x), phi * x * y]
        p = s.Integer(0)
    L = [[s.diff(u[c], X[a]) for a in range(3)] for c in range(3)]
    div = sum(L[i][i] for i in range(3))
    tau = [[eta * (L[c][a] + L[a][c]) - s.Rational(2, 3) * eta * div * (1 if a == c else 0) for a in range(3)]
           for c in range(3)]                                      # eq:stress
    f = [-sum(s.diff(tau[c][a], X[a]) for a in range(3)) + s.diff(p, X[c]) for c in range(3)]
    lam = lambda e: s.lambdify(X, e, "numpy")
    return lam(u), lam(f), lam(eta), lam(p)


def _discrete(mt, fu, ff, fe, hg_alpha=0.0, quad="one"):
    m = ShellMesh(mt, mt, R_IN, R_OUT)
    xyz = m.node_xyz()
    wn = m.wedge_nodes()
    xw = xyz[wn]
    N, _ = ref_basis(*QC)
    xq = np.einsum("j,wja->wa", N, xw)                   # x(q_c) of each wedge
    o = StokesOracle(mt, mt, fe(*xq.T), R_IN, R_OUT, hg_alpha=hg_alpha, quad=quad)
    _, V, _ = wedge_geometry(xw)
    fq = np.array(ff(*xq.T)).T
    F = np.zeros((m.n_nodes, 3))
    np.add.at(F, wn, V[:, None, None] * N[None, :, None] * fq[:, None, :])
    F[m.boundary_nodes()] = 0.0
    ue = np.array(fu(*xyz.T)).T
    return m, o, F, ue


@pytest.mark.slow
@pytest.mark.parametrize("hg_alpha,quad", [(0.0, "one"), (0.05, "one"), (0.0, "two")])
def test_viscous_block_second_order(hg_alpha, quad):
    """Also with hourglass control (eq:hgstab) and with the two-radial-point rule: the
    error keeps the optimal order."""
    fu, ff, fe, _ = _fields(stokes=False)
    errs = []
    for mt in (4, 8):
        m, o, F, ue = _discrete(mt, fu, ff, fe, hg_alpha, quad)
        uh = spla.spsolve(o.A_D.tocsc(), F.ravel()).reshape(-1, 3)
        errs.append(np.sqrt(np.mean((uh - ue) ** 2)))
    assert errs[0] / errs[1] > 3.4, errs


@pytest.mark.slow
@pytest.mark.parametrize("hg_alpha", [0.0, 0.05])
def test_stokes_second_order_velocity_and_pressure(hg_alpha):
    fu, ff, fe, fp = _fields(stokes=True)
    eu, ep = [], []
    for mt in (4, 8):
        m, o, F, ue = _discrete(mt, fu, ff, fe, hg_alpha)
        uh, ph = o.solve(F)
        pc = fp(*ShellMesh(mt // 2, mt // 2, R_IN, R_OUT).node_xyz().T)
        pc = pc - pc.mean()
        eu.append(np.sqrt(np.mean((uh - ue) ** 2)))
        ep.append(np.sqrt(np.mean((ph - pc) ** 2)))
    assert eu[0] / eu[1] > 3.4, eu
    assert ep[0] / ep[1] > 3.0, ep
    assert ep[1] < 0.02                  # |p| is O(1)
