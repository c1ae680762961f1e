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
