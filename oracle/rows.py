"""Selected rows of the oracle Stokes operator, one row at a time.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

At full size (e.g. the (128,128) shell, 66 M unknowns) the assembled matrix of
``StokesOracle`` does not fit a test, but every row of K_D is still a short
sum over the wedges around one node, and that sum is evaluated here with the
same element matrices (eq:elemmat, one point q_c, ``element_matrices`` /
``element_divergence``) and the same readings as ``StokesOracle``:

* velocity row (node f, component c), f interior:
      y = sum_{e ∋ f} [A_e (D u)_e + B_{f,e}^T (P p)_e]_{(f, c)}
  and y = u_(f, c) on the Dirichlet spheres (identity rows of K_D);
* pressure row (coarse node q):
      y = sum_f P_{f q} sum_{e ∋ f} [B_{f,e} (D u)_e]_f,
  i.e. B = P^T B_f with P the W1 index-space interpolation from the coarse
  pressure grid (level - 1, nr / 2), D the Dirichlet column mask.

Each row also returns the sum of the magnitudes of its terms, the natural
scale for a rounding-error bound on any other evaluation order.
"""
from __future__ import annotations

import numpy as np

from .mesh import ShellMesh
from .stokes import element_divergence, element_matrices_hg


class StokesRows:
    """Row evaluator of K_D on ``mesh`` (velocity level) with pressure on level - 1."""

    def __init__(self, mesh: ShellMesh, hg_alpha: float = 0.0):
        self.mesh = m = mesh
        self.hg_alpha = hg_alpha
        if m.nr % 2:
            raise ValueError("nr must be even")
        self.nrc = m.nr // 2
        # lateral vertex -> triangles containing it
        tri = m.tris
        order = np.argsort(tri.ravel(), kind="stable")
        self._tri_of = (order // 3).astype(np.int64)
        counts = np.bincount(tri.ravel(), minlength=m.n_lat)
        self._tri_ptr = np.concatenate([[0], np.cumsum(counts)])
        # lateral W1 interpolation: fine vertex -> (coarse vertices, weights)
        n_c = m.h.n_nodes(m.L - 1)
        self.n_c = n_c
        par = np.asarray(m.h.parents[m.L])            # parents of fine vertices n_c ..
        self._par = par
        # coarse vertex -> fine vertices interpolating from it (itself + edge midpoints)
        mids = np.concatenate([par[:, 0], par[:, 1]])
        mid_ids = np.concatenate([np.arange(len(par)), np.arange(len(par))]) + n_c
        o = np.argsort(mids, kind="stable")
        self._mid_of = mid_ids[o]
        cnt = np.bincount(mids, minlength=n_c)
        self._mid_ptr = np.concatenate([[0], np.cumsum(cnt)])
        self._xyz_r = m.r

    # -- topology ------------------------------------------------------------
    def wedges_of(self, lat: int, k: int) -> np.ndarray:
        """Wedges w = tri * nr + kk containing node (lat, k)."""
        m = self.mesh
        tris = self._tri_of[self._tri_ptr[lat]:self._tri_ptr[lat + 1]]
        ks = [kk for kk in (k - 1, k) if 0 <= kk < m.nr]
        return (tris[:, None] * m.nr + np.asarray(ks)[None, :]).ravel()

    def wedge_nodes(self, w: np.ndarray) -> np.ndarray:
        """[len(w), 6] node ids (0-2 at r_k, 3-5 at r_{k+1})."""
        m = self.mesh
        tri, k = np.divmod(np.asarray(w), m.nr)
        bot = m.tris[tri] * (m.nr + 1) + k[:, None]
        return np.concatenate([bot, bot + 1], axis=1)

    def node_xyz(self, nodes: np.ndarray) -> np.ndarray:
        m = self.mesh
        lat, k = np.divmod(np.asarray(nodes), m.nr + 1)
        return m.s[lat] * m.r[k][..., None]

    def boundary(self, nodes: np.ndarray) -> np.ndarray:
        k = np.asarray(nodes) % (self.mesh.nr + 1)
        return (k == 0) | (k == self.mesh.nr)

    # -- pressure interpolation ------------------------------------------------
    def lat_weights(self, lat: int):
        """Coarse vertices and weights of the fine lateral vertex ``lat``."""
        if lat < self.n_c:
            return [lat], [1.0]
        a, b = self._par[lat - self.n_c]
        return [int(a), int(b)], [0.5, 0.5]

    def rad_weights(self, k: int):
        if k % 2 == 0:
            return [k // 2], [1.0]
        return [(k - 1) // 2, (k + 1) // 2], [0.5, 0.5]

    def interp_p(self, nodes: np.ndarray, p: np.ndarray) -> np.ndarray:
        """(P p) at fine nodes; p indexed latc * (nrc + 1) + kc."""
        out = np.empty(len(nodes))
        for t, nd in enumerate(np.asarray(nodes).ravel()):
            lat, k = divmod(int(nd), self.mesh.nr + 1)
            v = 0.0
            for lc, wl in zip(*self.lat_weights(lat)):
                for kc, wr in zip(*self.rad_weights(k)):
                    v += wl * wr * p[lc * (self.nrc + 1) + kc]
            out[t] = v
        return out

    def fine_of_coarse(self, q: int):
        """Fine nodes f with P[f, q] != 0 and their weights."""
        latc, kc = divmod(int(q), self.nrc + 1)
        lats = [latc] + list(self._mid_of[self._mid_ptr[latc]:self._mid_ptr[latc + 1]])
        wl = [1.0] + [0.5] * (len(lats) - 1)
        ks = [2 * kc] + [k for k in (2 * kc - 1, 2 * kc + 1) if 0 <= k <= self.mesh.nr]
        wr = [1.0] + [0.5] * (len(ks) - 1)
        nodes, wts = [], []
        for la, a in zip(lats, wl):
            for k, b in zip(ks, wr):
                nodes.append(int(la) * (self.mesh.nr + 1) + k)
                wts.append(a * b)
        return nodes, wts

    # -- rows -----------------------------------------------------------------
    def _element_terms(self, lat: int, k: int, eta_of):
        w = self.wedges_of(lat, k)
        wn = self.wedge_nodes(w)
        xw = self.node_xyz(wn)
        f = lat * (self.mesh.nr + 1) + k
        loc = np.argmax(wn == f, axis=1)               # local index of f in each wedge
        return w, wn, xw, loc

    def velocity_row(self, node: int, eta_of, u: np.ndarray, p: np.ndarray):
        """(y[3], scale[3]) of K_D at node; u [n_nodes, 3], p coarse nodal values."""
        if self.boundary(np.array([node]))[0]:
            return u[node].astype(np.float64).copy(), np.abs(u[node]).astype(np.float64)
        lat, k = divmod(int(node), self.mesh.nr + 1)
        w, wn, xw, loc = self._element_terms(lat, k, eta_of)
        A = element_matrices_hg(xw, eta_of(w), self.hg_alpha)  # [n, 18, 18]
        Bf = element_divergence(xw)                           # [n, 6, 18]
        ue = u[wn].astype(np.float64)                          # [n, 6, 3]
        ue[self.boundary(wn)] = 0.0                            # Dirichlet columns
        ue = ue.reshape(len(w), 18)
        pe = self.interp_p(wn.ravel(), p).reshape(wn.shape)    # (P p) at the wedge nodes
        y = np.zeros(3)
        s = np.zeros(3)
        for e in range(len(w)):
            rows = 3 * loc[e] + np.arange(3)
            ta = A[e, rows, :] * ue[e][None, :]                # [3, 18]
            tb = Bf[e][:, rows].T * pe[e][None, :]             # [3, 6]: B_f^T (P p)
            y += ta.sum(axis=1) + tb.sum(axis=1)
            s += np.abs(ta).sum(axis=1) + np.abs(tb).sum(axis=1)
        return y, s

    def pressure_row(self, q: int, eta_of, u: np.ndarray):
        """(y, scale) of the row q of B D."""
        y = 0.0
        s = 0.0
        for f, wt in zip(*self.fine_of_coarse(q)):
            lat, k = divmod(int(f), self.mesh.nr + 1)
            w, wn, xw, loc = self._element_terms(lat, k, eta_of)
            Bf = element_divergence(xw)
            ue = u[wn].astype(np.float64)
            ue[self.boundary(wn)] = 0.0
            ue = ue.reshape(len(w), 18)
            for e in range(len(w)):
                t = wt * Bf[e, loc[e], :] * ue[e]
                y += t.sum()
                s += np.abs(t).sum()
        return y, s


def eta_law(mesh: ShellMesh, T_node: np.ndarray, wedges: np.ndarray, E: float, F: float = 0.0):
    """eta_e = exp(-E Tbar_e + F (1 - r_m,e)) for the given wedges only (the law of
    ``stokes.eta_from_temperature``: Tbar_e the mean of the six nodal values)."""
    nr = mesh.nr
    tri, k = np.divmod(np.asarray(wedges), nr)
    bot = mesh.tris[tri] * (nr + 1) + k[:, None]
    wn = np.concatenate([bot, bot + 1], axis=1)
    Tbar = T_node[wn].mean(axis=1)
    rm = 0.5 * (mesh.r[k] + mesh.r[k + 1])
    return np.exp(-E * Tbar + F * (1.0 - rm))
