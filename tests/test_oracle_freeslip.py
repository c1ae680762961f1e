"""Pins of the oracle's free-slip boundary condition (the setup of the paper's
verification runs, Sec. 8: zero normal velocity and zero tangential traction
on the spheres, imposed by rotating a boundary node's velocity to the frame
(rhat, two tangents) and making the normal component a Dirichlet DoF).

* With free slip on both spheres the rigid rotations u = w x x are tangential
  and strain-free, so they span the null space of the viscous block exactly
  (three zero eigenvalues, the rest positive); they are divergence-free, so
  B annihilates them too.
* With no slip on either sphere there is no null space (positive definite).
* In the rotated frame the normal row is an identity row and the normal input
  does not enter any other row.
Each property is also checked to reject a planted mistake.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle.mesh import ShellMesh
from oracle.stokes import StokesOracle, boundary_projections

MT = NR = 4


@pytest.fixture(scope="module")
def shell():
    om = ShellMesh(MT, NR)
    eta = 10.0 ** np.random.default_rng(3).uniform(-1.0, 1.0, om.n_wedges)
    return om, eta


def _rotations(om):
    x = om.node_xyz()
    return np.stack([np.cross(np.tile(w, (om.n_nodes, 1)), x).ravel() for w in np.eye(3)], axis=1)


def test_noslip_projection_is_the_dirichlet_operator(shell):
    om, eta = shell
    o = StokesOracle(MT, NR, eta, hierarchy=om.h)
    d = (~np.repeat(om.boundary_nodes(), 3)).astype(float)
    A_D = sp.diags(d) @ o.A @ sp.diags(d) + sp.diags(1.0 - d)
    assert abs(o.A_D - A_D).max() == 0.0
    assert abs(o.BT_D - sp.diags(d) @ o.B.T).max() == 0.0


def test_freeslip_rotations_span_the_null_space(shell):
    om, eta = shell
    o = StokesOracle(MT, NR, eta, hierarchy=om.h, bc=("freeslip", "freeslip"))
    A = o.A_D.toarray()
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    R = _rotations(om)
    assert np.abs(o.P_bc @ R - R).max() < 1e-15            # tangential on both spheres
    assert np.abs(A @ R).max() < 1e-12 * np.abs(A).max()
    assert np.abs(o.B_D @ R).max() < 1e-12 * np.abs(o.B_D).max()
    lam = np.linalg.eigvalsh(A)
    top = lam.max()
    assert np.all(lam > -1e-12 * top)
    assert np.sum(lam < 1e-10 * top) == 3
    assert lam[3] > 1e-6 * top
    # planted mistake: the normal identity rows left out (P A P alone) adds a zero
    # eigenvalue for every boundary node's normal direction
    lam_bad = np.linalg.eigvalsh((o.P_bc @ o.A @ o.P_bc).toarray())
    assert np.sum(lam_bad < 1e-10 * top) > 3


def test_noslip_inner_freeslip_outer_is_positive_definite(shell):
    om, eta = shell
    o = StokesOracle(MT, NR, eta, hierarchy=om.h, bc=("noslip", "freeslip"))
    lam = np.linalg.eigvalsh(o.A_D.toarray())
    assert lam.min() > 1e-6 * lam.max()
    # a rigid rotation is no longer admissible on the no-slip sphere: it has energy
    R = _rotations(om)
    assert np.linalg.norm(o.A_D @ R) > 1e-3 * np.linalg.norm(R)


def test_freeslip_normal_rows_are_identity_rows(shell):
    """rhat . (K x)_i = rhat . u_i at every free-slip node, and changing the normal
    input component of a boundary node changes no other row; the operator stays
    symmetric.  A one-sided projection (A P + N, a plausible slip) is not."""
    om, eta = shell
    o = StokesOracle(MT, NR, eta, hierarchy=om.h, bc=("freeslip", "freeslip"))
    rng = np.random.default_rng(4)
    u = rng.standard_normal((om.n_nodes, 3))
    p = rng.standard_normal(o.n_p)
    yu, yp = o.apply(u, p)
    bnd = om.boundary_nodes()
    x = om.node_xyz()
    rhat = x / np.linalg.norm(x, axis=1)[:, None]
    assert np.allclose((yu * rhat).sum(1)[bnd], (u * rhat).sum(1)[bnd], rtol=0, atol=1e-13)
    u2 = u.copy()
    u2[bnd] += 0.7 * rhat[bnd]                                # normal components only
    yu2, yp2 = o.apply(u2, p)
    change = yu2 - yu
    assert np.allclose(change[~bnd], 0.0, atol=1e-13) and np.allclose(yp2, yp, atol=1e-13)
    assert np.allclose(change[bnd], 0.7 * rhat[bnd], atol=1e-13)
    K = o.K
    assert abs(K - K.T).max() <= 1e-14 * abs(K).max()
    one_sided = (o.A @ o.P_bc + o.N_bc).tocsr()
    assert abs(one_sided - one_sided.T).max() > 1e-6 * abs(o.A).max()


def test_boundary_projections_reject_unknown_kinds():
    om = ShellMesh(2, 2)
    with pytest.raises(ValueError):
        boundary_projections(om, ("slip", "noslip"))


# ---- the gauged direct solve (pressure mean fixed by a multiplier) ----------------------

def _layers(om):
    k = np.tile(np.arange(NR + 1), om.n_lat)
    return k == 0, k == NR


def _rhs(om, bc, seed):
    """Random body force, zero on no-slip rows; on free-slip rows the normal part
    is the prescribed normal velocity."""
    f = np.random.default_rng(seed).standard_normal((om.n_nodes, 3))
    inner, outer = _layers(om)
    if bc[0] == "noslip":
        f[inner] = 0.0
    if bc[1] == "noslip":
        f[outer] = 0.0
    return f


def test_gauged_solve_is_the_pinned_solve_with_no_slip(shell):
    om, eta = shell
    o = StokesOracle(MT, NR, eta, hierarchy=om.h)
    f = _rhs(om, ("noslip", "noslip"), 11)
    u1, p1 = o.solve(f)
    u2, p2, c = o.solve_gauged(f)
    assert np.linalg.norm(u2 - u1) < 1e-10 * np.linalg.norm(u1)
    assert np.linalg.norm(p2 - p1) < 1e-10 * np.linalg.norm(p1)
    assert abs(c) < 1e-12 * np.abs(p1).max()


def test_freeslip_keeps_the_constant_pressure_null_space_only_to_h2(shell):
    """B_D^T 1 vanishes with no slip, not with free slip (node normals against the
    chordal boundary facets), and shrinks like h^2 under refinement."""
    om, eta = shell
    one = lambda o: np.ones(o.n_p)
    o_ns = StokesOracle(MT, NR, eta, hierarchy=om.h)
    assert np.linalg.norm(o_ns.BT_D @ one(o_ns)) < 1e-13 * abs(o_ns.BT_D).max()
    res = []
    for mt in (4, 8):
        m = ShellMesh(mt, mt)
        o = StokesOracle(mt, mt, np.ones(m.n_wedges), hierarchy=m.h, bc=("noslip", "freeslip"))
        r = np.linalg.norm(o.BT_D @ one(o))
        assert np.linalg.norm(one(o) @ o.B_D) == pytest.approx(r, rel=1e-10)   # symmetric
        res.append(r)
    assert res[0] > 1e-3 and 3.0 < res[0] / res[1] < 6.0


@pytest.mark.parametrize("bc", [("noslip", "freeslip"), ("freeslip", "noslip")])
def test_gauged_freeslip_solve_satisfies_its_equations(shell, bc):
    om, eta = shell
    o = StokesOracle(MT, NR, eta, hierarchy=om.h, bc=bc)
    f = _rhs(om, bc, 12)
    u, p, c = o.solve_gauged(f)
    fn = np.linalg.norm(f)
    assert np.linalg.norm(o.A_D @ u.ravel() + o.BT_D @ p - f.ravel()) < 1e-10 * fn
    assert np.linalg.norm(o.B_D @ u.ravel() - c) < 1e-10 * np.linalg.norm(u)
    assert abs(p.mean()) < 1e-12 * np.abs(p).max()
    assert abs(c) > 1e-8                                 # the multiplier is needed here
    # normal velocity on the free-slip sphere = the normal part of f
    inner, outer = _layers(om)
    fsn = inner if bc[0] == "freeslip" else outer
    rhat = om.node_xyz()[fsn]
    rhat /= np.linalg.norm(rhat, axis=1)[:, None]
    assert np.allclose(np.sum(u[fsn] * rhat, 1), np.sum(f[fsn] * rhat, 1), rtol=0, atol=1e-12 * fn)
    # planted contrast: the pinned solve of the no-slip case, taken as it is, leaves a
    # momentum residual of the size of c B_D^T 1
    u1, p1 = o.solve(f)
    assert np.linalg.norm(o.A_D @ u1.ravel() + o.BT_D @ p1 - f.ravel()) > 1e-6 * fn


def test_gauged_solve_with_free_slip_on_both_spheres(shell):
    """Both spheres free: the rotations are a null space, the solve takes u
    orthogonal to them; for a body force orthogonal to them the rotation
    multipliers vanish and every equation holds.  A buoyancy-type force (radial
    at the wedge centroid, one-point rule) is orthogonal to them exactly."""
    om, eta = shell
    bc = ("freeslip", "freeslip")
    o = StokesOracle(MT, NR, eta, hierarchy=om.h, bc=bc)
    R = o.rotations()
    f = _rhs(om, bc, 14).ravel()
    f -= R @ np.linalg.solve(R.T @ R, R.T @ f)
    u, p, c = o.solve_gauged(f.reshape(-1, 3))
    fn = np.linalg.norm(f)
    assert np.linalg.norm(o.last_rotation_multipliers) < 1e-10 * fn
    assert np.linalg.norm(o.A_D @ u.ravel() + o.BT_D @ p - f) < 1e-10 * fn
    assert np.linalg.norm(o.B_D @ u.ravel() - c) < 1e-10 * np.linalg.norm(u)
    assert np.linalg.norm(R.T @ u.ravel()) < 1e-10 * np.linalg.norm(u) * np.linalg.norm(R)
    # adding a rotation to u changes no equation (the null space)
    assert np.linalg.norm(o.A_D @ R[:, 0]) < 1e-12 * np.linalg.norm(R[:, 0])
    # the body force Ra T rhat(q_c) of the one-point rule is orthogonal to the rotations
    from oracle.stokes import buoyancy_rhs
    T = np.random.default_rng(15).uniform(0.0, 1.0, om.n_nodes)
    fb = buoyancy_rhs(om, T, 1e5).ravel()
    assert np.linalg.norm(R.T @ fb) < 1e-12 * np.linalg.norm(fb) * np.linalg.norm(R)
