"""Test-side glue between the library's duplicated-diamond layout and the
oracle's unique numbering.  The two are matched by coordinates only."""
from __future__ import annotations

import numpy as np

from oracle.mesh import ShellMesh, match_points


class LayoutMap:
    """Maps fields of one library level onto an oracle ShellMesh of the same (m, n)."""

    def __init__(self, lib_unit_xyz: np.ndarray, lib_r: np.ndarray, om: ShellMesh):
        self.om = om
        m1 = lib_unit_xyz.shape[1]
        self.m = m1 - 1
        self.n = len(lib_r) - 1
        assert np.allclose(lib_r, om.r, rtol=0, atol=1e-14)
        self.slot2lat = match_points(lib_unit_xyz.reshape(-1, 3), om.s, tol=1e-12)
        # every oracle node is reached by some slot
        assert len(np.unique(self.slot2lat)) == om.n_lat
        self.shape = (10, m1, m1, self.n + 1)
        n1 = self.n + 1
        self.slot_node = (self.slot2lat[:, None] * n1 + np.arange(n1)[None, :]).reshape(self.shape)
        # first slot of every oracle lateral node
        first = np.full(om.n_lat, -1)
        for s_, l_ in enumerate(self.slot2lat):
            if first[l_] < 0:
                first[l_] = s_
        self.first_slot = first

    # node fields ---------------------------------------------------------
    def to_lib(self, field_nodes: np.ndarray) -> np.ndarray:
        """[n_nodes, C] or [n_nodes] oracle field -> [C, 10, m+1, m+1, n+1] (or without C)."""
        f = np.asarray(field_nodes)
        if f.ndim == 1:
            return f[self.slot_node]
        return np.moveaxis(f[self.slot_node], -1, 0)

    def from_lib(self, field_lib: np.ndarray, check_dups: float | None = None) -> np.ndarray:
        """Library field -> oracle order, reading the first copy of every node."""
        f = np.asarray(field_lib)
        lead = f.shape[:-4]
        flat = f.reshape(lead + (-1, self.n + 1))
        out = flat[..., self.first_slot, :]                      # [..., n_lat, n+1]
        if check_dups is not None:
            full = flat                                          # every copy equals its first copy
            ref = out[..., self.slot2lat, :]
            scale = max(np.abs(ref).max(), 1e-300)
            assert np.abs(full - ref).max() <= check_dups * scale, "duplicate copies disagree"
        out = out.reshape(lead + (-1,))
        return np.moveaxis(out, 0, -1) if lead else out

    # wedge fields --------------------------------------------------------
    def wedge_index(self) -> np.ndarray:
        """Oracle wedge id of every library wedge [10, m, m, n, 2]."""
        m, n = self.m, self.n
        s2l = self.slot2lat.reshape(10, m + 1, m + 1)
        tri_id = {tuple(sorted(t)): q for q, t in enumerate(self.om.tris)}
        out = np.empty((10, m, m, n, 2), dtype=np.int64)
        for d in range(10):
            for i in range(m):
                for j in range(m):
                    ta = tuple(sorted((s2l[d, i, j], s2l[d, i + 1, j], s2l[d, i, j + 1])))
                    tb = tuple(sorted((s2l[d, i + 1, j + 1], s2l[d, i, j + 1], s2l[d, i + 1, j])))
                    out[d, i, j, :, 0] = tri_id[ta] * n + np.arange(n)
                    out[d, i, j, :, 1] = tri_id[tb] * n + np.arange(n)
        return out
