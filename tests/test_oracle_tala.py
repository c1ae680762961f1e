"""Pins of the oracle's compressible (TALA) terms, Sec. 1: the mass balance
div(rhobar u) = 0 (eq:mass), the buoyancy rhobar alphabar T' rhat of eq:stokes
and the split T = Tbar(r) + T' of eq:tsplit.

Reading (also the library's): the mass rows are -(psi, div(rhobar u)) with
rhobar u interpolated nodally, B_rho = B R, R = diag(rhobar(r_j)).
* A constant reference density scales B.
* The discrete compatibility 1^T B_rho = 0 (the divergence of a velocity that
  vanishes on the spheres sums to zero over the pressure nodes) holds exactly;
  the product form rhobar div u + u . grad rhobar at q_c (a plausible
  alternative) violates it, which would leave the saddle point inconsistent.
* A mass flux rhobar u that is a rigid rotation is divergence-free: B_rho u = 0.
* With free slip the mass rows are B R P: a velocity normal to the spheres carries no
  mass through them (it does without the projection), a tangential one enters unchanged.
* Manufactured anelastic solution u = curl(psi) / rhobar: second order.
* The TALA buoyancy reduces to the Boussinesq one for rhobar alphabar = 1, Tbar = 0,
  and vanishes for T = Tbar.
"""
import numpy as np
import pytest
import sympy as s

from oracle.mesh import ShellMesh
from oracle.saddle import SchurSolver
from oracle.stokes import QC, StokesOracle, buoyancy_rhs, buoyancy_rhs_tala, ref_basis, wedge_geometry

R_IN, R_OUT = 0.55, 1.0
LAM = np.log(1.6)          # density rises by 60 % from the surface to the inner sphere


def rho_of(r):
    return np.exp(LAM * (R_OUT - r) / (R_OUT - R_IN))


@pytest.fixture(scope="module")
def shell():
    om = ShellMesh(4, 4)
    eta = 10.0 ** np.random.default_rng(5).uniform(-1.0, 1.0, om.n_wedges)
    return om, eta


def test_constant_density_scales_B(shell):
    om, eta = shell
    o = StokesOracle(4, 4, eta, hierarchy=om.h, rho_nodes=np.full(5, 2.5))
    assert abs(o.B_mass - 2.5 * o.B_D).max() <= 1e-15 * abs(o.B_D).max()


def test_compatibility_and_divergence_free_flux(shell):
    om, eta = shell
    rho = rho_of(om.r)
    o = StokesOracle(4, 4, eta, hierarchy=om.h, rho_nodes=rho)
    ones = np.ones(o.n_p)
    assert np.abs(ones @ o.B_mass).max() <= 1e-15 * abs(o.B_mass).max() * o.n_p
    # rhobar u = w x x (a rigid rotation, zero velocity on the spheres masked by the BC)
    x = om.node_xyz()
    k = np.tile(np.arange(om.nr + 1), om.n_lat)
    v = np.cross(np.tile([0.3, -0.2, 0.9], (om.n_nodes, 1)), x)
    u = v / rho[k][:, None]
    o_fs = StokesOracle(4, 4, eta, hierarchy=om.h, rho_nodes=rho, bc=("freeslip", "freeslip"))
    assert np.abs(o_fs.B_mass @ u.ravel()).max() < 1e-15 * abs(o_fs.B_mass).max() * np.abs(v).max() * 20
    # planted alternative: -(psi, rhobar(q_c) div u + rhobar'(q_c) u(q_c) . rhat(q_c)) on a
    # field vanishing on the spheres does not sum to zero over the pressure nodes
    wn = om.wedge_nodes()
    xw = x[wn]
    N, _ = ref_basis(*QC)
    _, V, g = wedge_geometry(xw)
    kw = np.tile(np.arange(om.nr), len(om.tris))
    h = om.r[1] - om.r[0]
    rm, drho = 0.5 * (rho[kw] + rho[kw + 1]), (rho[kw + 1] - rho[kw]) / h
    uu = np.random.default_rng(6).standard_normal((om.n_nodes, 3))
    uu[om.boundary_nodes()] = 0.0
    div = np.einsum("wja,wja->w", g, uu[wn])
    uq = np.einsum("j,wja->wa", N, uu[wn])
    xq = np.einsum("j,wja->wa", N, xw)
    ur = np.einsum("wa,wa->w", uq, xq / np.linalg.norm(xq, axis=1)[:, None])
    total_product_form = -(V * (rm * div + drho * ur)).sum()
    total_nodal_form = ones @ (o.B_mass @ uu.ravel())
    assert abs(total_nodal_form) < 1e-14 * np.abs(o.B_mass @ uu.ravel()).sum()
    assert abs(total_product_form) > 1e-6 * np.abs(o.B_mass @ uu.ravel()).sum()


def test_freeslip_mass_rows_take_the_tangential_sphere_velocity(shell):
    """With free slip the mass rows are B R P: a velocity normal to the spheres (at their
    nodes only) carries no mass through them, while without the projection it does; a
    tangential sphere velocity enters unchanged."""
    om, eta = shell
    rho = rho_of(om.r)
    o_fs = StokesOracle(4, 4, eta, hierarchy=om.h, rho_nodes=rho, bc=("freeslip", "freeslip"))
    o_no = StokesOracle(4, 4, eta, hierarchy=om.h, rho_nodes=rho, bc=("none", "none"))
    x = om.node_xyz()
    rhat = x / np.linalg.norm(x, axis=1)[:, None]
    k = np.tile(np.arange(om.nr + 1), om.n_lat)
    interior = (k != 0) & (k != om.nr)
    rng = np.random.default_rng(8)
    un = rhat * rng.standard_normal(om.n_nodes)[:, None]
    un[interior] = 0.0
    scale = abs(o_no.B_mass).max() * np.abs(un).max()
    assert np.abs(o_fs.B_mass @ un.ravel()).max() <= 1e-14 * scale
    assert np.abs(o_no.B_mass @ un.ravel()).max() > 1e-2 * scale
    w = rng.standard_normal((om.n_nodes, 3))
    ut = w - rhat * np.sum(w * rhat, 1)[:, None]
    ut[interior] = w[interior]
    assert np.abs(o_fs.B_mass @ ut.ravel() - o_no.B_mass @ ut.ravel()).max() <= 1e-14 * abs(o_no.B_mass).max() * 4


def test_tala_buoyancy_special_cases(shell):
    om, _ = shell
    rng = np.random.default_rng(8)
    T = rng.uniform(0.0, 1.0, om.n_nodes)
    f0 = buoyancy_rhs_tala(om, T, 3.0, np.zeros(om.nr + 1), np.ones(om.nr + 1))
    assert np.abs(f0 - buoyancy_rhs(om, T, 3.0)).max() <= 1e-15 * np.abs(f0).max()
    Tbar = np.linspace(1.0, 0.0, om.nr + 1)
    k = np.tile(np.arange(om.nr + 1), om.n_lat)
    assert np.abs(buoyancy_rhs_tala(om, Tbar[k], 3.0, Tbar, rho_of(om.r))).max() < 1e-15
    # a layer-constant factor scales the result of its layer's wedges; for a constant
    # factor everything
    f2 = buoyancy_rhs_tala(om, T, 3.0, Tbar, np.full(om.nr + 1, 2.0))
    f1 = buoyancy_rhs_tala(om, T, 3.0, Tbar, np.ones(om.nr + 1))
    assert np.abs(f2 - 2.0 * f1).max() <= 1e-15 * np.abs(f1).max() * 4


@pytest.mark.slow
def test_anelastic_manufactured_solution_second_order():
    X = s.symbols("x y z")
    x, y, z = X
    r = s.sqrt(x ** 2 + y ** 2 + z ** 2)
    rho = s.exp(LAM * (R_OUT - r) / (R_OUT - R_IN))
    eta = 1 + s.Rational(1, 2) * x * z
    phi = ((r - R_IN) * (R_OUT - r)) ** 2
    psi = [phi * y * z, phi * s.sin(x), phi * (x + z ** 2)]
    curl = [s.diff(psi[2], y) - s.diff(psi[1], z), s.diff(psi[0], z) - s.diff(psi[2], x),
            s.diff(psi[1], x) - s.diff(psi[0], y)]
    u = [c / rho for c in curl]                                    # div(rho u) = 0
    p = x * y + z ** 3
    L = [[s.diff(u[c], X[a]) for a in range(3)] for c in range(3)]
    div = sum(L[i][i] for i in range(3))
    tau = [[eta * (L[c][a] + L[a][c]) - s.Rational(2, 3) * eta * div * (1 if a == c else 0) for a in range(3)]
           for c in range(3)]
    f = [-sum(s.diff(tau[c][a], X[a]) for a in range(3)) + s.diff(p, X[c]) for c in range(3)]
    lam = lambda e: s.lambdify(X, e, "numpy")                     # noqa: E731
    fu, ff, fe, fp = lam(u), lam(f), lam(eta), lam(p)
    eu, ep = [], []
    for mt in (4, 8):
        m = ShellMesh(mt, mt, R_IN, R_OUT)
        xyz = m.node_xyz()
        wn = m.wedge_nodes()
        xw = xyz[wn]
        N, _ = ref_basis(*QC)
        xq = np.einsum("j,wja->wa", N, xw)
        etaw = fe(*xq.T)
        o = StokesOracle(mt, mt, etaw, R_IN, R_OUT, rho_nodes=rho_of(m.r))
        _, V, _ = wedge_geometry(xw)
        fq = np.array(ff(*xq.T)).T
        F = np.zeros((m.n_nodes, 3))
        np.add.at(F, wn, V[:, None, None] * N[None, :, None] * fq[:, None, :])
        F[m.boundary_nodes()] = 0.0
        uh, ph, info = SchurSolver(o, etaw).solve(F, rtol=1e-12)
        assert info["rel_res"] < 1e-10
        ue = np.array(fu(*xyz.T)).T
        pc = fp(*ShellMesh(mt // 2, mt // 2, R_IN, R_OUT).node_xyz().T)
        pc = pc - pc.mean()
        eu.append(np.sqrt(np.mean((uh - ue) ** 2)))
        ep.append(np.sqrt(np.mean((ph - pc) ** 2)))
    assert eu[0] / eu[1] > 3.4, eu
    assert ep[0] / ep[1] > 3.0, ep
