"""Oracle of the modified method of characteristics for the temperature
(Sec. 6: eq:characteristic, eq:departure, eq:mmoc).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

One time step of the energy equation with unit diffusivity (Boussinesq form):

1. departure points (eq:departure): every node x_i is traced back along the
   (steady, per step) velocity field over dt with the explicit midpoint rule,
   a two-stage explicit Runge-Kutta method:
       x_mid = x_i - dt/2 u(x_i),    xhat_i = x_i - dt u(x_mid);
2. the old temperature at the departure points, That_i = T^n(xhat_i), by the
   W1 interpolant of the wedge containing xhat_i ("linear interpolation");
3. the implicit diffusion step of eq:mmoc with the lumped mass of the W1
   energy operator (Sec. 6) and Dirichlet temperatures on the spheres:
       (M_L / dt + K) T^{n+1} = M_L (That / dt + H).

Readings: the velocity u is the nodal W1 field of the Stokes solve of the step,
interpolated like the temperature; a departure point that leaves the shell
is brought back radially onto it (its radius clamped to [r_in, r_out]).

Point location is by brute force: each wedge is the set {lam s : s in the flat
(chordal) triangle of its three lateral nodes, lam in [r_k, r_k+1]} (the
isoparametric map x = r(zeta) s(xi, eta)), so x = a s0 + b s1 + c s2 with
(a, b, c) from Cramer's rule gives lam = a + b + c and the barycentric
coordinates (xi, eta) = (b, c) / lam; the triangle is the one with
min(a, b, c) largest (all >= 0 inside), found by testing every triangle.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .energy import EnergyOracle
from .mesh import ShellMesh


def locate(mesh: ShellMesh, pts: np.ndarray, chunk: int = 256):
    """(tri, xi, eta, k, zeta) of every point [P, 3] (radius clamped to the shell)."""
    pts = np.asarray(pts, np.float64)
    S = mesh.s[mesh.tris]                          # [T, 3 corners, 3]
    s0, s1, s2 = S[:, 0], S[:, 1], S[:, 2]
    det = np.einsum("ta,ta->t", s0, np.cross(s1, s2))
    tri = np.empty(len(pts), np.int64)
    coef = np.empty((len(pts), 3))
    for a0 in range(0, len(pts), chunk):
        x = pts[a0:a0 + chunk]                     # [P, 3]
        a = np.einsum("pa,ta->pt", x, np.cross(s1, s2)) / det
        b = np.einsum("pa,ta->pt", x, np.cross(s2, s0)) / det
        c = np.einsum("pa,ta->pt", x, np.cross(s0, s1)) / det
        score = np.minimum(np.minimum(a, b), c)
        best = np.argmax(score, axis=1)
        rows = np.arange(len(x))
        tri[a0:a0 + chunk] = best
        coef[a0:a0 + chunk] = np.stack([a[rows, best], b[rows, best], c[rows, best]], axis=1)
    lam = coef.sum(axis=1)
    xi, eta = coef[:, 1] / lam, coef[:, 2] / lam
    lam = np.clip(lam, mesh.r_in, mesh.r_out)
    dr = (mesh.r_out - mesh.r_in) / mesh.nr
    k = np.clip(np.floor((lam - mesh.r_in) / dr).astype(np.int64), 0, mesh.nr - 1)
    zeta = 2.0 * (lam - mesh.r[k]) / dr - 1.0
    return tri, xi, eta, k, zeta


def interpolate(mesh: ShellMesh, field: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """W1 interpolant of a node field ([n_nodes] or [n_nodes, C]) at the points."""
    tri, xi, eta, k, zeta = locate(mesh, pts)
    lat = np.stack([1.0 - xi - eta, xi, eta], axis=1)                 # [P, 3]
    rad = np.stack([0.5 * (1.0 - zeta), 0.5 * (1.0 + zeta)], axis=1)  # [P, 2]
    corners = mesh.tris[tri]                                          # [P, 3]
    f = np.asarray(field, np.float64)
    out = 0.0
    for a in range(3):
        for b in range(2):
            node = corners[:, a] * (mesh.nr + 1) + k + b
            w = lat[:, a] * rad[:, b]
            out = out + (w[:, None] * f[node] if f.ndim == 2 else w * f[node])
    return out


def departure_points(mesh: ShellMesh, u_nodes: np.ndarray, dt: float) -> np.ndarray:
    """Explicit midpoint rule backwards along the nodal velocity field (eq:departure)."""
    x = mesh.node_xyz()
    u = np.asarray(u_nodes, np.float64)
    x_mid = x - 0.5 * dt * u
    return x - dt * interpolate(mesh, u, x_mid)


def mmoc_step(mesh: ShellMesh, T_n: np.ndarray, u_nodes: np.ndarray, dt: float, H=None,
              T_inner: float = 1.0, T_outer: float = 0.0):
    """One MMOC step (eq:mmoc): returns (That, T^{n+1})."""
    That = interpolate(mesh, T_n, departure_points(mesh, u_nodes, dt))
    diff = EnergyOracle(mesh, np.zeros((mesh.n_nodes, 3)), dt)       # M_L / dt + K, Dirichlet rows
    b = diff.rhs(That, H, T_inner, T_outer)
    return That, spla.spsolve(diff.E.tocsc(), b)
