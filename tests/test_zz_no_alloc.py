"""The no-allocation smoother (tng_smooth_noalloc) against tng_smooth.

Both run the same Chebyshev kernels; the no-allocation entry point draws its
work vectors from the library's fixed device scratch array instead of
allocating them.  Two calls in a row, the second on a smaller level, so the
second call starts from whatever the first left in the array.  The (8,8)
results are also checked against the oracle's textbook Chebyshev iteration
(relative 1e-12 FP64, 1e-5 FP32).
"""
import numpy as np
import pytest

import synthetic
from oracle.mesh import ShellMesh
from oracle.solver_ref import chebyshev
from oracle.stokes import StokesOracle
from tests._support import LayoutMap

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tng():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_21633_amd as t
    return t


@pytest.fixture(scope="module")
def ctx(tng):
    return tng.Context(0)


def _case(tng, ctx, mt, seed):
    import torch
    mesh = tng.Mesh(ctx, mt, mt, levels=1)
    om = ShellMesh(mt, mt)
    lm = LayoutMap(*mesh.coords(0), om)
    rng = np.random.default_rng(seed)
    eta = 10.0 ** rng.uniform(-1, 1, om.n_wedges)
    b = rng.standard_normal((om.n_nodes, 3))
    x = rng.standard_normal((om.n_nodes, 3))
    bnd = om.boundary_nodes()
    b[bnd] = 0.0
    x[bnd] = 0.0
    dev = torch.device("cuda", 0)
    t = dict(eta=torch.tensor(eta[lm.wedge_index()], device=dev),
             b=torch.tensor(lm.to_lib(b), device=dev).contiguous(),
             x=torch.tensor(lm.to_lib(x), device=dev).contiguous())
    return mesh, om, lm, eta, b, x, t


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("dtype,tol", [("float64", 1e-12), ("float32", 1e-5)])
def test_noalloc_smoother_matches_smooth(tng, ctx, dtype, tol):
    import torch
    dt = getattr(torch, dtype)
    for call, mt in enumerate((16, 8)):          # the second call is the smaller level
        mesh, om, lm, eta, b, x, t = _case(tng, ctx, mt, 11 + call)
        eta_t = t["eta"].to(dt)
        d = torch.empty((3,) + mesh.shape(0), dtype=dt, device="cuda")
        tng.diag_A(ctx, mesh, 0, eta_t, d)
        x_ref = t["x"].to(dt).clone()
        x_na = t["x"].to(dt).clone()
        tng.smooth(ctx, mesh, 0, eta_t, d, t["b"].to(dt), x_ref, 2, 2, 0.3, 3.3)
        tng.smooth_noalloc(ctx, mesh, 0, eta_t, d, t["b"].to(dt), x_na, 2, 2, 0.3, 3.3)
        torch.cuda.synchronize()
        got = lm.from_lib(x_na.double().cpu().numpy(), check_dups=1e-6)
        ref = lm.from_lib(x_ref.double().cpu().numpy())
        e_lib = _rel(got, ref)
        print(f"no-alloc smoother {dtype} ({mt},{mt}) call {call + 1}: rel diff to tng_smooth {e_lib:.2e}", flush=True)
        assert e_lib <= (1e-13 if dtype == "float64" else 1e-6)
        if mt == 8:
            orc = StokesOracle(mt, mt, eta, hierarchy=om.h)
            want = chebyshev(orc.A_D, orc.diag_A().ravel(), b.ravel(), x.ravel(), 2, 2, 0.3, 3.3).reshape(-1, 3)
            e_orc = _rel(got, want)
            print(f"  vs oracle Chebyshev: {e_orc:.2e}", flush=True)
            assert e_orc < tol


def test_noalloc_smoother_rejects_oversized_level(tng, ctx):
    """(64,64) needs more than the 48 MiB scratch array: refused before any launch."""
    import torch
    mesh = tng.Mesh(ctx, 64, 64, levels=1)
    shp = (3,) + mesh.shape(0)
    eta = torch.ones(mesh.wedge_shape(0), dtype=torch.float64, device="cuda")
    d = torch.ones(shp, dtype=torch.float64, device="cuda")
    b = torch.zeros(shp, dtype=torch.float64, device="cuda")
    x = torch.zeros(shp, dtype=torch.float64, device="cuda")
    with pytest.raises(tng.TngError) as ei:
        tng.smooth_noalloc(ctx, mesh, 0, eta, d, b, x, 2, 2, 0.3, 3.3)
    assert ei.value.code == -1 and "scratch" in str(ei.value)
