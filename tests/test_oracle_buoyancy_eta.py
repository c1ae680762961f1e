"""Pins of the oracle's buoyancy right-hand side and temperature-viscosity law
against things other than themselves.

* Buoyancy (eq:stokes right-hand side, Boussinesq form, one-point rule of
  Sec. 4): brute force on the coarsest shell (the isoparametric map and its
  Jacobian evaluated from a hand-written wedge basis by central differences,
  which are exact for the map's quadratic terms), and the hydrostatic special
  case: a purely radial temperature makes Ra T rhat the gradient of
  Phi(r) = Ra int T dr, so the exact Stokes solution is u = 0, p = Phi + const;
  the discrete solution approaches it at second order in the pressure.
* Viscosity law (the Frank-Kamenetskii family of Sec. 8 with a depth factor,
  eta at q_c per Sec. 4): values computed by hand from the formula.

Each pin is also run on planted mistakes (copies of the oracle function with
one plausible error) to show that it rejects them.
"""
import numpy as np
import pytest

import synthetic
from oracle.mesh import ShellMesh
from oracle.saddle import SchurSolver
from oracle.stokes import QC, StokesOracle, buoyancy_rhs, eta_from_temperature, ref_basis, wedge_geometry


# ---- hand-written wedge basis and brute-force buoyancy ----------------------

def _basis(xi, et, ze):
    lat = (1.0 - xi - et, xi, et)
    rad = (0.5 * (1.0 - ze), 0.5 * (1.0 + ze))
    return np.array([lat[j % 3] * rad[j // 3] for j in range(6)])


def _brute_force_buoyancy(mesh, T, Ra):
    """f_j = sum_e V_e N_j(q_c) Ra T(q_c) x(q_c)/|x(q_c)|, every quantity from the
    wedge's own map x(xi, eta, zeta) = sum_j N_j x_j and plain loops."""
    wn = mesh.wedge_nodes()
    xyz = mesh.node_xyz()
    f = np.zeros((mesh.n_nodes, 3))
    q = np.array([1.0 / 3.0, 1.0 / 3.0, 0.0])
    hstep = 1e-3
    for w in range(len(wn)):
        xs = xyz[wn[w]]

        def x_of(pt):
            return _basis(*pt) @ xs

        J = np.empty((3, 3))
        for m in range(3):
            e = np.zeros(3)
            e[m] = hstep
            J[:, m] = (x_of(q + e) - x_of(q - e)) / (2 * hstep)
        V = abs(np.linalg.det(J))
        N = _basis(*q)
        xq = x_of(q)
        Tq = N @ T[wn[w]]
        for j in range(6):
            f[wn[w][j]] += V * N[j] * Ra * Tq * xq / np.linalg.norm(xq)
    return f


def _mutant_rhat_at_node(mesh, T, Ra):
    wn = mesh.wedge_nodes()
    xw = mesh.node_xyz()[wn]
    N, _ = ref_basis(*QC)
    _, V, _ = wedge_geometry(xw)
    Tq = np.einsum("j,wj->w", N, T[wn])
    rhat = xw / np.linalg.norm(xw, axis=2)[:, :, None]         # planted: direction of the node
    f = np.zeros((mesh.n_nodes, 3))
    np.add.at(f, wn, (V * Tq * Ra)[:, None, None] * N[None, :, None] * rhat)
    return f


def _mutant_no_basis_weight(mesh, T, Ra):
    return 6.0 * buoyancy_rhs(mesh, T, Ra)                       # planted: N_j(q_c) = 1/6 dropped


def _mutant_nodal_T(mesh, T, Ra):
    wn = mesh.wedge_nodes()
    xw = mesh.node_xyz()[wn]
    N, _ = ref_basis(*QC)
    _, V, _ = wedge_geometry(xw)
    xq = np.einsum("j,wja->wa", N, xw)
    rhat = xq / np.linalg.norm(xq, axis=1)[:, None]
    f = np.zeros((mesh.n_nodes, 3))
    contrib = (V * Ra)[:, None, None] * (N[None, :] * T[wn])[:, :, None] * rhat[:, None, :]   # planted: T_j, not T(q_c)
    np.add.at(f, wn, contrib)
    return f


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("mt,nr", [(1, 1), (2, 1)])
def test_buoyancy_equals_brute_force(mt, nr):
    m = ShellMesh(mt, nr)
    T = np.random.default_rng(5).uniform(0.0, 1.0, m.n_nodes)
    want = _brute_force_buoyancy(m, T, 3.0)
    assert _rel(buoyancy_rhs(m, T, 3.0), want) < 1e-12
    for mutant in (_mutant_rhat_at_node, _mutant_no_basis_weight, _mutant_nodal_T):
        assert _rel(mutant(m, T, 3.0), want) > 1e-4, mutant.__name__


def _hydrostatic(mt, T_of_r, rhs=buoyancy_rhs):
    """Solve with eta = 1 and f = rhs(T(r)); returns (rms |u|, rms |u| of the same
    problem with a lateral temperature perturbation, relative pressure error
    against Phi(r) - mean)."""
    om = ShellMesh(mt, mt)
    r = np.tile(om.r, om.n_lat)
    T = T_of_r(r)
    eta = np.ones(om.n_wedges)
    orc = StokesOracle(mt, mt, eta, hierarchy=om.h)
    sol = SchurSolver(orc, eta)
    f = rhs(om, T, 1.0)
    f[om.boundary_nodes()] = 0.0
    u, p, _ = sol.solve(f)
    f2 = rhs(om, T + 0.1 * np.repeat(om.s[:, 0], mt + 1), 1.0)
    f2[om.boundary_nodes()] = 0.0
    u2, _, _ = sol.solve(f2)
    return u, u2, p, om


@pytest.mark.parametrize("case", ["uniform", "conductive"])
def test_radial_temperature_gives_hydrostatic_pressure(case):
    rin, rout = 0.55, 1.0
    if case == "uniform":
        T_of_r = np.ones_like
        Phi = lambda r: r                                                        # noqa: E731
    else:
        T_of_r = lambda r: synthetic.conductive_profile(r, rin, rout)            # noqa: E731
        Phi = lambda r: rin / (rout - rin) * (rout * np.log(r) - r)             # noqa: E731
    out = []
    for mt in (4, 8):
        u, u2, p, om = _hydrostatic(mt, T_of_r)
        omp = ShellMesh(mt // 2, mt // 2, hierarchy=om.h)
        phi = Phi(np.tile(omp.r, omp.n_lat))
        phi -= phi.mean()
        rms = np.sqrt(om.n_nodes)
        out.append((np.linalg.norm(u) / rms, np.linalg.norm(u2) / rms, np.linalg.norm(p - phi) / np.linalg.norm(phi)))
    (u4, v4, e4), (u8, v8, e8) = out
    # the gradient force drives (nearly) no flow: an order of magnitude below the
    # flow of a lateral perturbation, and falling with the mesh size
    assert u8 < 0.1 * v8 and u8 < 0.6 * u4, out
    # p -> Phi - mean at second order
    assert e8 < 0.02 and e4 / e8 > 3.4, out


def test_hydrostatic_pin_rejects_a_dropped_basis_weight():
    u, u2, p, om = _hydrostatic(4, np.ones_like, rhs=_mutant_no_basis_weight)
    omp = ShellMesh(2, 2, hierarchy=om.h)
    phi = np.tile(omp.r, omp.n_lat)
    phi -= phi.mean()
    assert np.linalg.norm(p - phi) / np.linalg.norm(phi) > 1.0


# ---- viscosity law -------------------------------------------------------------

def _mutant_eta_mean_of_three(mesh, T, E, F=0.0):
    wn = mesh.wedge_nodes()
    Tbar = T[wn[:, :3]].mean(axis=1)                          # planted: bottom triangle only
    k = np.tile(np.arange(mesh.nr), len(mesh.tris))
    rm = 0.5 * (mesh.r[k] + mesh.r[k + 1])
    return np.exp(-E * Tbar + F * (1.0 - rm))


def test_eta_law_hand_values():
    """eta = exp(-E Tbar + F (1 - r_m)) with E = ln 1e3, F = ln 10 on [0.55, 1]:
    * one layer, T = 0 inside, 1 outside: Tbar = 1/2, r_m = 0.775, so every wedge
      has eta = 10^(-3/2 + 0.225) = 10^-1.275;
    * two layers, T = (r - 0.55)/0.45: layer 0 Tbar = 1/4, r_m = 0.6625 -> 10^-0.4125,
      layer 1 Tbar = 3/4, r_m = 0.8875 -> 10^-2.1375."""
    E, F = np.log(1e3), np.log(10.0)
    m = ShellMesh(2, 1)
    T = np.tile([0.0, 1.0], m.n_lat)
    assert np.allclose(eta_from_temperature(m, T, E, F), 10.0 ** -1.275, rtol=1e-14, atol=0)
    assert not np.allclose(_mutant_eta_mean_of_three(m, T, E, F), 10.0 ** -1.275, rtol=1e-6)
    m2 = ShellMesh(2, 2)
    T2 = np.tile([0.0, 0.5, 1.0], m2.n_lat)
    eta = eta_from_temperature(m2, T2, E, F).reshape(-1, 2)     # [triangle, layer]
    assert np.allclose(eta[:, 0], 10.0 ** -0.4125, rtol=1e-14, atol=0)
    assert np.allclose(eta[:, 1], 10.0 ** -2.1375, rtol=1e-14, atol=0)
    assert not np.allclose(_mutant_eta_mean_of_three(m2, T2, E, F).reshape(-1, 2)[:, 0], 10.0 ** -0.4125, rtol=1e-6)


def test_eta_law_lateral_mean_over_the_wedge_nodes():
    """A temperature equal to the height z of the node: Tbar_e is the mean of z
    over the wedge's six nodes, checked against the nodes found by position
    (the wedge's six corner positions average to x(q_c), the map at the
    barycentre), so eta_e = exp(-E z(q_c)) exactly for F = 0."""
    m = ShellMesh(4, 2)
    x = m.node_xyz()
    T = x[:, 2]
    wn = m.wedge_nodes()
    N, _ = ref_basis(*QC)
    xq = np.einsum("j,wja->wa", N, x[wn])          # x(q_c) = mean of the six corners
    assert np.allclose(eta_from_temperature(m, T, 2.0), np.exp(-2.0 * xq[:, 2]), rtol=1e-13, atol=0)
