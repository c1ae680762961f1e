"""Pins of the oracle's modified method of characteristics (Sec. 6,
eq:characteristic, eq:departure, eq:mmoc)."""
import numpy as np
import pytest

from oracle.energy import EnergyOracle
from oracle.mesh import ShellMesh
from oracle.mmoc import departure_points, interpolate, locate, mmoc_step


@pytest.fixture(scope="module")
def mesh():
    return ShellMesh(4, 4)


def _random_points(mesh, n, seed):
    """Points inside the chordal shell (the flat triangles lie inside the unit sphere, so
    near the outer sphere a point of radius < r_out can still be outside the mesh)."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    r = rng.uniform(mesh.r_in, 0.9 * mesh.r_out, n)
    return d * r[:, None]


def test_location_reproduces_the_point(mesh):
    """The found wedge coordinates map back to the point through the wedge's own
    isoparametric map, and lie in the reference wedge."""
    pts = _random_points(mesh, 400, 1)
    tri, xi, eta, k, zeta = locate(mesh, pts)
    S = mesh.s[mesh.tris[tri]]
    s = (1 - xi - eta)[:, None] * S[:, 0] + xi[:, None] * S[:, 1] + eta[:, None] * S[:, 2]
    r = 0.5 * (1 - zeta) * mesh.r[k] + 0.5 * (1 + zeta) * mesh.r[k + 1]
    assert np.abs(r[:, None] * s - pts).max() < 1e-13
    tol = 1e-12
    assert (xi > -tol).all() and (eta > -tol).all() and (xi + eta < 1 + tol).all()
    assert (np.abs(zeta) <= 1 + tol).all()


def test_interpolation_reproduces_linear_fields(mesh):
    """The W1 interpolant of T = a . x + c is exact everywhere (isoparametric map)."""
    a, c = np.array([0.3, -1.2, 0.7]), 0.4
    T = mesh.node_xyz() @ a + c
    pts = _random_points(mesh, 500, 2)
    assert np.abs(interpolate(mesh, T, pts) - (pts @ a + c)).max() < 1e-13
    # nodes interpolate their own values
    assert np.abs(interpolate(mesh, T, mesh.node_xyz()) - T).max() < 1e-13


def test_departure_points_of_a_rigid_rotation(mesh):
    """u = w x x is reproduced exactly by W1, so the departure point is the explicit
    midpoint rule's: x - dt w x x + dt^2/2 w x (w x x), third-order close to the exact
    rotation by -|w| dt (the local error falls by 8 when dt halves)."""
    w = np.array([0.2, -0.5, 1.1])
    x = mesh.node_xyz()
    u = np.cross(np.tile(w, (len(x), 1)), x)
    wn = np.linalg.norm(w)
    axis = w / wn

    def rotate(v, ang):
        return (v * np.cos(ang) + np.cross(np.tile(axis, (len(v), 1)), v) * np.sin(ang)
                + axis * (v @ axis)[:, None] * (1 - np.cos(ang)))

    errs = []
    for dt in (0.04, 0.02):
        xh = departure_points(mesh, u, dt)
        want = x - dt * np.cross(np.tile(w, (len(x), 1)), x - 0.5 * dt * u)
        inside = (np.linalg.norm(want, axis=1) < mesh.r_out - 1e-12)   # clamping aside
        assert np.abs(xh - want)[inside].max() < 1e-13
        errs.append(np.abs(xh - rotate(x, -wn * dt))[inside].max())
    assert 7.0 < errs[0] / errs[1] < 9.0, errs


def test_still_flow_is_implicit_diffusion(mesh):
    """u = 0: the departure points are the nodes, That = T^n, and the step is the
    backward-Euler conduction step of the energy operator without flow."""
    rng = np.random.default_rng(3)
    T = rng.uniform(0, 1, mesh.n_nodes)
    H = rng.uniform(0, 2, mesh.n_nodes)
    That, T1 = mmoc_step(mesh, T, np.zeros((mesh.n_nodes, 3)), 0.01, H)
    assert np.abs(That - T).max() < 1e-14
    assert np.abs(T1 - EnergyOracle(mesh, np.zeros((mesh.n_nodes, 3)), 0.01).step(T, H)).max() < 1e-12


def test_linear_field_advected_by_rotation(mesh):
    """A linear temperature carried by a rigid rotation: That_i = a . xhat_i exactly
    (interior nodes: a node on a sphere rotates to just outside the chordal shell, whose
    outer faces are flat, and is brought back onto it)."""
    w = np.array([0.0, 0.0, 2.0])
    x = mesh.node_xyz()
    u = np.cross(np.tile(w, (len(x), 1)), x)
    a = np.array([1.0, -0.5, 0.25])
    xh = departure_points(mesh, u, 0.05)
    That = interpolate(mesh, x @ a, xh)
    inner = ~mesh.boundary_nodes()
    assert np.abs(That - xh @ a)[inner].max() < 1e-13
