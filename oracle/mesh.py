"""Oracle shell mesh (Sec. 2 "Grid and Parallelization", Table 1, Sec. 3 eq:wedgebasis).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper builds the shell from an icosahedron with 12 vertices whose 20
spherical triangles are paired into 10 diamonds, refines the triangles by
recursive midpoint refinement, extrudes the surface mesh radially and splits
each extruded hexahedron into two wedges.  This oracle builds the same set of
wedges WITHOUT any diamond index space: it refines the 20 triangles directly,
one into four per level, so the only thing it shares with the library is the
geometry, and the two are matched by node coordinates.

Readings of passages that the paper leaves open (same reading on both sides):
* orientation: poles on the z axis, upper ring at z = 1/sqrt(5) with longitudes
  2 pi k / 5, lower ring at z = -1/sqrt(5) with longitudes 2 pi k / 5 + pi / 5;
* "midpoint refinement": the new node of an edge (a, b) is (a + b) / |a + b|,
  the midpoint of the great-circle arc, applied recursively level by level;
* radial layers are uniform, r_k = r_in + k (r_out - r_in) / nr.

One-into-four refinement of a triangle (a, b, c) gives the corner triangles
(a, ab, ca), (ab, b, bc), (ca, bc, c) and the centre triangle (ab, bc, ca).  In
a diamond's (i, j) index space these are exactly the two triangles of each quad
split along the diagonal parallel to the diamond's shared diagonal, which is
what makes fine wedges nest inside coarse wedges.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def icosahedron():
    """The 12 vertices and 20 faces of the base icosahedron (Sec. 2, Fig. diamonds).

    Returns (verts[12, 3], tris[20, 3]).  Vertex ids: 0 = north pole, 1..5 =
    upper ring U_0..U_4, 6..10 = lower ring L_0..L_4, 11 = south pole.
    """
    z = 1.0 / np.sqrt(5.0)
    rho = 2.0 / np.sqrt(5.0)
    verts = [np.array([0.0, 0.0, 1.0])]
    for k in range(5):
        a = 2.0 * np.pi * k / 5.0
        verts.append(np.array([rho * np.cos(a), rho * np.sin(a), z]))
    for k in range(5):
        a = 2.0 * np.pi * k / 5.0 + np.pi / 5.0
        verts.append(np.array([rho * np.cos(a), rho * np.sin(a), -z]))
    verts.append(np.array([0.0, 0.0, -1.0]))
    N, S = 0, 11

    def U(k):
        return 1 + (k % 5)

    def L(k):
        return 6 + (k % 5)

    tris = []
    for k in range(5):
        tris.append((N, U(k), U(k + 1)))          # polar cap of north diamond k
        tris.append((U(k), L(k), U(k + 1)))       # equatorial half of north diamond k
        tris.append((U(k + 1), L(k), L(k + 1)))   # equatorial half of south diamond k
        tris.append((L(k), S, L(k + 1)))          # polar cap of south diamond k
    return np.array(verts), np.array(tris, dtype=np.int64)


def refine_once(verts: np.ndarray, tris: np.ndarray):
    """One level of recursive geodesic midpoint refinement (Sec. 2).

    Returns (new_verts, new_tris, parents) where the first len(verts) vertices
    are the old ones unchanged and ``parents[n - len(verts)]`` are the two old
    vertices whose arc midpoint is new vertex n.
    """
    nv = len(verts)
    mid = {}
    new_pts = []
    parents = []

    def midpoint(a, b):
        key = (a, b) if a < b else (b, a)
        m = mid.get(key)
        if m is None:
            s = verts[a] + verts[b]
            new_pts.append(s / np.sqrt(s @ s))
            parents.append(key)
            m = nv + len(new_pts) - 1
            mid[key] = m
        return m

    out = []
    for a, b, c in tris:
        ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
        out.append((a, ab, ca))
        out.append((ab, b, bc))
        out.append((ca, bc, c))
        out.append((ab, bc, ca))
    new_verts = np.vstack([verts, np.array(new_pts)]) if new_pts else verts.copy()
    return new_verts, np.array(out, dtype=np.int64), np.array(parents, dtype=np.int64).reshape(-1, 2)


def level_of(mt: int) -> int:
    L = int(round(np.log2(mt)))
    if mt < 1 or 2 ** L != mt:
        raise ValueError("mt must be a power of two")
    return L


class SphereHierarchy:
    """Surface triangulations of every level 0..L (mt = 2**level intervals per diamond edge)."""

    def __init__(self, mt: int):
        self.L = level_of(mt)
        v, t = icosahedron()
        self.verts = [v]
        self.tris = [t]
        self.parents = [None]
        for _ in range(self.L):
            v, t, par = refine_once(v, t)
            self.verts.append(v)
            self.tris.append(t)
            self.parents.append(par)

    def n_nodes(self, level: int) -> int:
        return len(self.verts[level])


class ShellMesh:
    """Extruded shell at lateral level log2(mt) with nr uniform radial intervals.

    Node numbering: node = lat * (nr + 1) + k.  Wedge numbering: w = tri * nr + k,
    with local nodes 0..2 = the triangle's vertices at r_k and 3..5 = at r_{k+1}
    (eq:wedgebasis: nodes 0-2 bottom face, 3-5 top face).
    """

    def __init__(self, mt: int, nr: int, r_in: float = 0.55, r_out: float = 1.0,
                 hierarchy: SphereHierarchy | None = None):
        self.mt, self.nr, self.r_in, self.r_out = mt, nr, float(r_in), float(r_out)
        self.L = level_of(mt)
        self.h = hierarchy if hierarchy is not None and hierarchy.L >= self.L else SphereHierarchy(mt)
        self.s = self.h.verts[self.L]                 # unit vectors of lateral nodes
        self.tris = self.h.tris[self.L]
        self.r = r_in + (r_out - r_in) * np.arange(nr + 1) / nr
        self.n_lat = len(self.s)
        self.n_nodes = self.n_lat * (nr + 1)
        self.n_wedges = len(self.tris) * nr

    def node(self, lat, k):
        return np.asarray(lat) * (self.nr + 1) + np.asarray(k)

    def wedge_nodes(self) -> np.ndarray:
        """[n_wedges, 6] global node ids, wedge w = tri * nr + k."""
        nr = self.nr
        k = np.arange(nr)
        t = self.tris
        bot = t[:, None, :] * (nr + 1) + k[None, :, None]
        top = bot + 1
        return np.concatenate([bot, top], axis=2).reshape(-1, 6)

    def node_xyz(self) -> np.ndarray:
        """[n_nodes, 3] physical coordinates r_k * s_lat."""
        return (self.s[:, None, :] * self.r[None, :, None]).reshape(-1, 3)

    def boundary_nodes(self) -> np.ndarray:
        """Boolean [n_nodes]: node lies on the inner or outer sphere."""
        k = np.tile(np.arange(self.nr + 1), self.n_lat)
        return (k == 0) | (k == self.nr)


def prolongation(h: SphereHierarchy, fine_level: int, nr_fine: int) -> sp.csr_matrix:
    """W1 interpolation from (level-1, nr/2) to (level, nr) in index space.

    Pressure lives on the coarse grid (Sec. 3: W1-iso-W2 / W1 pair).  Its values
    inside the fine wedges are the fine-W1 interpolant of the coarse nodal
    values: a fine node that is a coarse node copies it, a node created on a
    coarse edge takes the mean of the edge's two end nodes, and the same rule
    applies radially (odd layers are the mean of the two coarse layers).
    Rows = fine nodes (lat * (nr+1) + k), columns = coarse nodes.
    """
    if nr_fine % 2:
        raise ValueError("nr must be even")
    nrc = nr_fine // 2
    n_c = h.n_nodes(fine_level - 1)
    n_f = h.n_nodes(fine_level)
    par = h.parents[fine_level]
    # lateral interpolation, n_f x n_c
    rows = list(range(n_c))
    cols = list(range(n_c))
    vals = [1.0] * n_c
    for m, (a, b) in enumerate(par):
        rows += [n_c + m, n_c + m]
        cols += [int(a), int(b)]
        vals += [0.5, 0.5]
    Plat = sp.csr_matrix((vals, (rows, cols)), shape=(n_f, n_c))
    # radial interpolation, (nr+1) x (nrc+1)
    rr, rc, rv = [], [], []
    for k in range(nr_fine + 1):
        if k % 2 == 0:
            rr.append(k); rc.append(k // 2); rv.append(1.0)
        else:
            rr += [k, k]; rc += [(k - 1) // 2, (k + 1) // 2]; rv += [0.5, 0.5]
    Prad = sp.csr_matrix((rv, (rr, rc)), shape=(nr_fine + 1, nrc + 1))
    # node = lat * (nr+1) + k  ->  Kronecker product lat (x) rad
    return sp.kron(Plat, Prad, format="csr")


def match_points(a: np.ndarray, b: np.ndarray, tol: float = 1e-9) -> np.ndarray:
    """For each row of ``a`` the index of the row of ``b`` at the same position.

    Raises if any point of ``a`` has no partner in ``b`` within ``tol``.  Used
    to match the library's duplicated-diamond layout to the oracle's unique
    nodes by coordinates only (no shared index conventions).
    """
    from scipy.spatial import cKDTree
    d, idx = cKDTree(b).query(a, k=1)
    if np.max(d, initial=0.0) > tol:
        raise ValueError(f"unmatched points: max distance {np.max(d):.3e}")
    return idx
