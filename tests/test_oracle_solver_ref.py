"""Pins of the oracle's solver reference pieces (Sec. 7)."""
import numpy as np
import scipy.sparse as sp

from oracle.mesh import ShellMesh
from oracle.solver_ref import chebyshev, lumped_pressure_mass, restrict_velocity, velocity_prolongation
from oracle.stokes import QC, StokesOracle, ref_basis, wedge_geometry


def test_lumped_mass_total_volume_and_brute_force():
    """With eta = 1 the lumped masses add up to the one-point volume of the
    shell (partition of unity of the pressure basis); with random eta they are
    the row sums of the explicitly assembled P^T M_f P."""
    m = ShellMesh(4, 4)
    orc = StokesOracle(4, 4, np.ones(m.n_wedges))
    _, V, _ = wedge_geometry(m.node_xyz()[m.wedge_nodes()])
    assert np.isclose(lumped_pressure_mass(orc, np.ones(m.n_wedges)).sum(), V.sum(), rtol=1e-13)
    eta = 10 ** np.random.default_rng(0).uniform(-1, 1, m.n_wedges)
    wn = m.wedge_nodes()
    N, _ = ref_basis(*QC)
    rows = np.repeat(wn, 6, axis=1).ravel()
    cols = np.tile(wn, (1, 6)).ravel()
    vals = ((V / eta)[:, None, None] * N[None, :, None] * N[None, None, :]).ravel()
    Mf = sp.csr_matrix((vals, (rows, cols)), shape=(m.n_nodes, m.n_nodes))
    M = (orc.P.T @ Mf @ orc.P).toarray()
    assert np.allclose(lumped_pressure_mass(orc, eta), M.sum(axis=1), rtol=1e-13)
    assert np.all(lumped_pressure_mass(orc, eta) > 0)


def test_chebyshev_matches_closed_form_polynomial():
    """On A = diag(lambda) with D = I and b = 0 one step of degree k maps x to
    T_k((theta - lambda)/delta) / T_k(theta/delta) x (Chebyshev polynomials)."""
    lam = np.linspace(0.05, 2.0, 40)
    A = sp.diags(lam)
    x0 = np.random.default_rng(1).standard_normal(40)
    lmin, lmax = 0.2, 2.2
    th, de = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)

    def T(k, z):
        return np.cosh(k * np.arccosh(z)) if np.all(np.abs(z) >= 1) and z.ndim == 0 else \
            np.where(np.abs(z) <= 1, np.cos(k * np.arccos(np.clip(z, -1, 1))),
                     np.cosh(k * np.arccosh(np.abs(z))) * np.sign(z) ** k)

    for k in (1, 2, 3):
        x = chebyshev(A, np.ones(40), np.zeros(40), x0, k, 1, lmin, lmax)
        p = T(k, (th - lam) / de) / T(k, np.array(th / de))
        assert np.allclose(x, p * x0, rtol=1e-12, atol=1e-14), k


def test_velocity_transfer_is_transpose_pair():
    m = ShellMesh(4, 4)
    orc = StokesOracle(4, 4, np.ones(m.n_wedges))
    Pv = velocity_prolongation(orc)
    assert Pv.shape == (3 * m.n_nodes, 3 * orc.n_p)
    rng = np.random.default_rng(2)
    f = rng.standard_normal((m.n_nodes, 3))
    c = rng.standard_normal((orc.n_p, 3))
    mc = ShellMesh(2, 2)
    cb = mc.boundary_nodes()
    c[cb] = 0.0
    lhs = np.sum(restrict_velocity(orc, f, cb) * c)
    rhs = np.sum(f.ravel() * (Pv @ c.ravel()))
    assert np.isclose(lhs, rhs, rtol=1e-12)
