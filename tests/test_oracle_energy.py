"""Pins of the oracle energy operator."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synthetic
from oracle.energy import EnergyOracle, supg_tau
from oracle.mesh import ShellMesh
from oracle.stokes import wedge_geometry


def test_tau_limits():
    h = np.array([0.1, 0.1, 0.1])
    u = np.array([1e-9, 1e3, 1e6])
    t = supg_tau(u, h)
    assert t[0] == pytest.approx(h[0] ** 2 / 12, rel=1e-9)        # diffusive limit
    assert t[2] == pytest.approx(h[2] / (2 * u[2]), rel=1e-4)      # advective limit
    # continuity across the series / closed-form switch
    pe = np.array([0.999e-3, 1.001e-3])
    uu = 2 * pe / 0.1
    tt = supg_tau(uu, np.full(2, 0.1))
    assert abs(tt[0] - tt[1]) / tt[0] < 1e-6


def test_constants_lumped_mass_and_total_volume():
    m = ShellMesh(4, 4)
    rng = np.random.default_rng(0)
    u = rng.standard_normal((m.n_nodes, 3))
    eo = EnergyOracle(m, u, dt=0.3)
    _, V, _ = wedge_geometry(m.node_xyz()[m.wedge_nodes()])
    assert eo.mass.sum() == pytest.approx(V.sum(), rel=1e-13)
    # diffusion, advection and SUPG annihilate constants
    r = eo.A_noD @ np.ones(m.n_nodes) - eo.mass / 0.3
    assert np.abs(r).max() < 1e-12


def test_steady_conduction_converges_to_analytic_profile():
    """u = 0, dt -> infinity: K T = 0 with T = 1 inside, 0 outside converges
    at second order to the spherical conduction profile."""
    errs = []
    for mt in (4, 8):
        m = ShellMesh(mt, mt)
        eo = EnergyOracle(m, np.zeros((m.n_nodes, 3)), dt=1e30)
        T = eo.step(np.zeros(m.n_nodes))
        r = np.tile(m.r, m.n_lat)
        errs.append(np.sqrt(np.mean((T - synthetic.conductive_profile(r, 0.55, 1.0)) ** 2)))
    assert errs[0] / errs[1] > 3.5, errs


def test_dirichlet_rows_and_step_solution():
    m = ShellMesh(4, 4)
    rng = np.random.default_rng(1)
    eo = EnergyOracle(m, rng.standard_normal((m.n_nodes, 3)), dt=0.05)
    Tn = rng.uniform(0, 1, m.n_nodes)
    T1 = eo.step(Tn, H=np.full(m.n_nodes, 2.0))
    k = np.tile(np.arange(m.nr + 1), m.n_lat)
    assert np.allclose(T1[k == 0], 1.0) and np.allclose(T1[k == m.nr], 0.0)
    assert np.abs(eo.apply(T1) - eo.rhs(Tn, np.full(m.n_nodes, 2.0))).max() < 1e-12


def test_advection_of_a_linear_field_is_exact():
    """Constant velocity ubar and T = a . x: the isoparametric W1 interpolant
    reproduces T exactly, so grad T_h = a at q_c and every row of the advection
    matrix is (C T)_i = sum_e V_e N_i(q_c) ubar . a = m_i (ubar . a), with m the
    lumped mass, at every node.  The transposed matrix (a plausible slip of the
    test/trial roles) does not satisfy this."""
    m = ShellMesh(4, 4)
    ub = np.array([0.3, -0.7, 0.4])
    a = np.array([1.0, 2.0, -0.5])
    eo = EnergyOracle(m, np.tile(ub, (m.n_nodes, 1)), dt=1.0)
    T = m.node_xyz() @ a
    want = (ub @ a) * eo.mass
    assert np.abs(eo.C @ T - want).max() < 1e-14 * np.abs(want).max()
    assert np.abs(eo.C.T @ T - want).max() > 1e-2 * np.abs(want).max()


def test_supg_term_is_symmetric_psd_and_blind_across_the_flow():
    """S_ij = sum_e V_e tau_e (ubar . grad phi_i)(ubar . grad phi_j) is a
    streamline diffusion: symmetric, positive semi-definite, zero on constants
    and on every linear field whose gradient is orthogonal to a constant flow."""
    m = ShellMesh(2, 2)
    ub = np.array([0.5, 0.2, -0.4])
    eo = EnergyOracle(m, np.tile(ub, (m.n_nodes, 1)), dt=1.0)
    S = eo.S.toarray()
    assert np.abs(S - S.T).max() < 1e-15 * np.abs(S).max()
    assert np.linalg.eigvalsh(S).min() > -1e-13 * np.abs(S).max()
    a = np.cross(ub, [1.0, 0.0, 0.0])                       # a . ubar = 0
    x = m.node_xyz()
    assert np.abs(S @ (x @ a)).max() < 1e-14 * np.abs(S).max()
    assert np.abs(S @ np.ones(m.n_nodes)).max() < 1e-14 * np.abs(S).max()
    assert np.abs(S @ (x @ ub)).max() > 1e-3 * np.abs(S).max()


def _mms_error(mt, transpose_advection=False):
    """Steady advection-diffusion -lap T + u . grad T = F in the shell with a
    rigid-rotation flow u = 3 w x x (divergence free) and the manufactured
    solution T* = x^2 - y z + sin z (so grad T* = (2x, -z, cos z - y) and
    lap T* = 2 - sin z); Dirichlet T = T* on both spheres; lumped load."""
    import scipy.sparse as sp
    w = np.array([0.3, -0.5, 1.0])
    m = ShellMesh(mt, mt)
    x = m.node_xyz()
    u = 3.0 * np.cross(np.tile(w, (m.n_nodes, 1)), x)
    eo = EnergyOracle(m, u, dt=1e30)
    Ts = x[:, 0] ** 2 - x[:, 1] * x[:, 2] + np.sin(x[:, 2])
    gT = np.stack([2 * x[:, 0], -x[:, 2], np.cos(x[:, 2]) - x[:, 1]], axis=1)
    F = -(2.0 - np.sin(x[:, 2])) + np.einsum("na,na->n", u, gT)
    b = eo.mass * F
    bnd = m.boundary_nodes()
    b[bnd] = Ts[bnd]
    if transpose_advection:
        A = eo.K + eo.C.T + eo.S
        E = sp.diags((~bnd).astype(float)) @ A + sp.diags(bnd.astype(float))
    else:
        E = eo.E
    T = spla.spsolve(E.tocsc(), b)
    return np.sqrt(np.mean((T - Ts) ** 2))


def test_steady_advection_diffusion_converges_at_second_order():
    e4, e8 = _mms_error(4), _mms_error(8)
    assert e4 / e8 > 3.4, (e4, e8)
    # with the advection matrix transposed the error does not fall
    m4, m8 = _mms_error(4, True), _mms_error(8, True)
    assert m8 > 10 * e8 and m4 / m8 < 1.5, (m4, m8)
