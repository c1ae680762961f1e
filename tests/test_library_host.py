"""CPU-side checks of the C-ABI library: it loads, exports every declared
symbol, validates arguments, and its host mesh equals the oracle mesh."""
import glob
import os
import re

import numpy as np
import pytest

from oracle.mesh import ShellMesh, SphereHierarchy
from tests._support import LayoutMap

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    import paper_2609_21633_amd as tng
    return tng


def test_library_exports_every_declared_symbol():
    tng = _lib()
    L = tng.lib()
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(tng_[a-z0-9_]+)\s*\(", src))
    assert names, "no declarations found"
    missing = [n for n in sorted(names) if not hasattr(L, n)]
    assert not missing, missing


def test_argument_validation_without_gpu():
    import ctypes as C
    tng = _lib()
    L = tng.lib()
    h = C.c_void_p()
    assert L.tng_mesh_create(None, 3, 4, 0.55, 1.0, 1, C.byref(h)) == -1
    assert b"power of two" in L.tng_last_error()
    assert L.tng_mesh_create(None, 8, 8, 1.0, 0.5, 1, C.byref(h)) == -1
    assert L.tng_mesh_create(None, 8, 6, 0.55, 1.0, 3, C.byref(h)) == -1
    assert L.tng_ctx_set_apply_bands(None, 0) == -1
    # 32-bit field offsets: (1024, 512) has 10 * 1025^2 * 513 > 2^31 node slots
    assert L.tng_mesh_create(None, 1024, 512, 0.55, 1.0, 1, C.byref(h)) == -1
    assert b"too large" in L.tng_last_error()
    # a host-only mesh is rejected by device calls
    m = tng.Mesh(None, 4, 4, levels=2)
    y = (C.c_void_p * 3)(1, 2, 3)
    rc = L.tng_stokes_apply(None, m.h, 0, 0, 1, 0.0, C.c_void_p(1), y, None, y, None)
    assert rc == -1
    assert L.tng_stokes_apply(C.c_void_p(0), m.h, 5, 0, 1, 0.0, None, y, None, y, None) == -1
    # hourglass-control scale must be finite and non-negative
    assert L.tng_stokes_apply(None, m.h, 0, 0, 1, -0.5, C.c_void_p(1), y, None, y, None) == -1
    assert b"hg_alpha" in L.tng_last_error()


@pytest.mark.parametrize("mt,nr", [(2, 2), (4, 4), (8, 4), (16, 16)])
def test_host_mesh_matches_oracle(mt, nr):
    """Counts, coordinates (matched by position), duplicate groups of size
    2 (edges), 3 (ring vertices) and 5 (poles), wedges = oracle wedges."""
    tng = _lib()
    m = tng.Mesh(None, mt, nr, levels=2 if mt > 1 else 1)
    c = m.counts(0)
    assert c["lat_unique"] == 10 * mt * mt + 2
    assert c["lat_slots"] == 10 * (mt + 1) ** 2
    assert c["cells"] == 10 * mt * mt * nr and c["wedges"] == 2 * c["cells"]
    xyz, r = m.coords(0)
    assert np.allclose(np.linalg.norm(xyz, axis=-1), 1.0, atol=1e-15)
    om = ShellMesh(mt, nr)
    lm = LayoutMap(xyz, r, om)
    # coordinates agree to rounding, not just within the matching tolerance
    assert np.abs(xyz.reshape(-1, 3) - om.s[lm.slot2lat]).max() < 1e-15
    uid = m.unique_ids(0).ravel()
    # same unique id <=> same oracle node
    assert len(np.unique(uid)) == om.n_lat
    pairs = np.unique(np.stack([uid, lm.slot2lat], 1), axis=0)
    assert len(pairs) == om.n_lat
    sizes = np.bincount(np.bincount(uid))
    assert sizes[2] == 20 * (mt - 1) and sizes[3] == 10 and sizes[5] == 2
    assert 10 * (mt + 1) ** 2 - (10 * mt * mt + 2) == 20 * mt + 8
    # every oracle wedge appears exactly once
    wi = lm.wedge_index()
    assert np.array_equal(np.sort(wi.ravel()), np.arange(om.n_wedges))


def test_pressure_level_nests():
    """Level 1 nodes are the even-index nodes of level 0 (pressure on the coarser grid)."""
    tng = _lib()
    m = tng.Mesh(None, 8, 8, levels=3)
    x0, r0 = m.coords(0)
    x1, r1 = m.coords(1)
    assert np.array_equal(x0[:, ::2, ::2], x1)
    assert np.array_equal(r0[::2], r1)


def test_binding_refuses_bad_tensors_before_any_call():
    """The binding checks device, dtype, contiguity and size of every field before
    it reaches the library (which sees only raw pointers)."""
    import torch
    tng = _lib()
    mesh = tng.Mesh(None, 4, 4, levels=2)

    class Ctx:                      # stands in for a context on device 0; never reaches the library
        device = 0
        h = None

    shp = (3,) + mesh.shape(0)
    eta = torch.ones(mesh.wedge_shape(0), dtype=torch.float64)
    u = torch.zeros(shp, dtype=torch.float64)
    y = torch.zeros(shp, dtype=torch.float64)
    with pytest.raises(TypeError, match="cuda:0"):
        tng.stokes_apply(Ctx, mesh, 0, tng.OP_A, eta, u, None, y, None)
    # the remaining checks, on tensors that claim to be on the device
    class Fake:
        def __init__(self, t, is_cuda=True):
            self.t, self.is_cuda = t, is_cuda
            self.device = torch.device("cuda", 0)
            self.dtype, self.shape = t.dtype, t.shape

        def is_contiguous(self):
            return self.t.is_contiguous()

        def numel(self):
            return self.t.numel()

        def __getitem__(self, i):
            return Fake(self.t[i])

        def __len__(self):
            return len(self.t)

    with pytest.raises(TypeError, match="dtype"):
        tng.stokes_apply(Ctx, mesh, 0, tng.OP_A, Fake(eta.float()), Fake(u), None, Fake(y), None)
    with pytest.raises(ValueError, match="values"):
        tng.stokes_apply(Ctx, mesh, 0, tng.OP_A, Fake(eta.reshape(-1)[:10].clone()), Fake(u), None, Fake(y), None)
    with pytest.raises(ValueError, match="contiguous"):
        tng.stokes_apply(Ctx, mesh, 0, tng.OP_A, Fake(eta), Fake(u.transpose(1, 2)), None, Fake(y), None)


def test_binding_structs_mirror_the_header(tmp_path):
    """The ctypes mirrors of the option and result structs have the C header's size
    and field offsets (a field added to one side only shifts every later one)."""
    import ctypes
    import shutil
    import subprocess
    from paper_2609_21633_amd import binding as b
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"tng_solver_opts": b.SolverOpts, "tng_solve_info": b.SolveInfo,
               "tng_step_opts": b.StepOpts, "tng_step_info": b.StepInfo}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "tng.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in filter(None, out):
        cname, field, val = line.split()
        got[(cname, field)] = int(val)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
    # the same field names in the same order (a field added in the padding of the last
    # one keeps the size)
    hdr = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "tng.h")).read(), flags=re.S)
    for cname, py in structs.items():
        body = re.search(r"typedef struct\s*\{([^{}]*)\}\s*" + cname + r"\s*;", hdr).group(1)
        names = []
        for decl in filter(None, (d.strip() for d in body.split(";"))):
            for part in decl.split(","):
                names.append(re.findall(r"[A-Za-z_][A-Za-z0-9_]*", part.split("[")[0])[-1])
        assert names == [f for f, _ in py._fields_], (cname, names)
