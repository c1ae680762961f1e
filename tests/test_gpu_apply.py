"""Parity of the HIP Stokes apply with the assembled FP64 oracle.

Tolerances (relative 2-norm per block over unique DoFs): 1e-12 for FP64,
1e-5 for FP32 (the FP32 path is fed the FP64 inputs rounded to FP32 and is
compared with the FP64 oracle on the original inputs).
"""
import numpy as np
import pytest

import synthetic
from oracle.mesh import ShellMesh
from oracle.stokes import StokesOracle
from tests._support import LayoutMap

pytestmark = pytest.mark.gpu

OPS_ALL = 1 | 2 | 4 | 8


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


_cache = {}


def setup_case(tng, ctx, mt, nr, seed=0):
    key = (mt, nr, seed)
    if key in _cache:
        return _cache[key]
    import torch
    mesh = tng.Mesh(ctx, mt, nr, levels=2)
    om = ShellMesh(mt, nr)
    omp = ShellMesh(mt // 2, nr // 2, hierarchy=om.h)
    lm = LayoutMap(*mesh.coords(0), om)
    lmp = LayoutMap(*mesh.coords(1), omp)
    eta, u, p = synthetic.uniform_operator_inputs(om.n_wedges, om.n_nodes, omp.n_nodes, seed)
    u[om.boundary_nodes()] = 0.0
    orc = StokesOracle(mt, nr, eta, hierarchy=om.h)
    dev = torch.device("cuda", 0)
    t = dict(
        eta=torch.tensor(eta[lm.wedge_index()], device=dev),
        u=torch.tensor(lm.to_lib(u), device=dev).contiguous(),
        p=torch.tensor(lmp.to_lib(p), device=dev).contiguous(),
    )
    _cache[key] = (mesh, om, lm, lmp, eta, u, p, orc, t)
    return _cache[key]


def run_apply(tng, ctx, mesh, t, flags, dtype):
    import torch
    eta, u, p = (t[k].to(dtype) for k in ("eta", "u", "p"))
    yu = torch.full_like(u, float("nan"))
    yp = torch.full_like(p, float("nan"))
    tng.stokes_apply(ctx, mesh, 0, flags, eta, u, p, yu, yp)
    torch.cuda.synchronize()
    return yu.double().cpu().numpy(), yp.double().cpu().numpy()


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("mt,nr", [(8, 8), (16, 16), (8, 6), (16, 10), (4, 2)])
def test_full_operator_fp64(tng, ctx, mt, nr):
    mesh, om, lm, lmp, eta, u, p, orc, t = setup_case(tng, ctx, mt, nr)
    import torch
    yu, yp = run_apply(tng, ctx, mesh, t, OPS_ALL, torch.float64)
    ru, rp = orc.apply(u, p)
    gu = lm.from_lib(yu, check_dups=1e-13)
    gp = lmp.from_lib(yp, check_dups=1e-13)
    print(f"fp64 ({mt},{nr}) rel u {rel(gu, ru):.2e} p {rel(gp, rp):.2e}")
    assert rel(gu, ru) < 1e-12
    assert rel(gp, rp) < 1e-12


@pytest.mark.parametrize("mt,nr", [(8, 8), (16, 16), (16, 10)])
def test_full_operator_fp32(tng, ctx, mt, nr):
    mesh, om, lm, lmp, eta, u, p, orc, t = setup_case(tng, ctx, mt, nr)
    import torch
    yu, yp = run_apply(tng, ctx, mesh, t, OPS_ALL, torch.float32)
    ru, rp = orc.apply(u, p)
    gu = lm.from_lib(yu, check_dups=1e-6)
    gp = lmp.from_lib(yp, check_dups=1e-6)
    print(f"fp32 ({mt},{nr}) rel u {rel(gu, ru):.2e} p {rel(gp, rp):.2e}")
    assert rel(gu, ru) < 1e-5
    assert rel(gp, rp) < 1e-5


def test_blocks_separately(tng, ctx):
    """A alone without Dirichlet, B^T alone and B alone with Dirichlet."""
    import torch
    mesh, om, lm, lmp, eta, u, p, orc, t = setup_case(tng, ctx, 8, 8)
    rng = np.random.default_rng(7)
    uf = rng.uniform(-1, 1, u.shape)                      # nonzero on the boundary
    tt = dict(t, u=torch.tensor(lm.to_lib(uf), device="cuda").contiguous())
    yu, _ = run_apply(tng, ctx, mesh, tt, 1, torch.float64)
    assert rel(lm.from_lib(yu), (orc.A @ uf.ravel()).reshape(-1, 3)) < 1e-12
    yu, _ = run_apply(tng, ctx, mesh, tt, 2 | 8, torch.float64)
    assert rel(lm.from_lib(yu), (orc.BT_D @ p).reshape(-1, 3)) < 1e-12
    _, yp = run_apply(tng, ctx, mesh, tt, 4 | 8, torch.float64)
    assert rel(lmp.from_lib(yp), orc.B_D @ uf.ravel()) < 1e-12
    yu, _ = run_apply(tng, ctx, mesh, tt, 1 | 8, torch.float64)
    assert rel(lm.from_lib(yu), (orc.A_D @ uf.ravel()).reshape(-1, 3)) < 1e-12


def test_unit_columns(tng, ctx):
    """Matrix-free == assembled (eq:matfree): columns of K for unit inputs."""
    import torch
    mesh, om, lm, lmp, eta, u, p, orc, t = setup_case(tng, ctx, 4, 4)
    K = orc.K.tocsc()
    rng = np.random.default_rng(3)
    interior = np.where(~orc.dirichlet)[0]
    for col in list(rng.choice(interior, 4, replace=False)) + list(orc.n_u + rng.choice(orc.n_p, 2)):
        x = np.zeros(orc.n_u + orc.n_p)
        x[col] = 1.0
        uu, pp = x[:orc.n_u].reshape(-1, 3), x[orc.n_u:]
        tt = dict(t, u=torch.tensor(lm.to_lib(uu), device="cuda").contiguous(),
                  p=torch.tensor(lmp.to_lib(pp), device="cuda").contiguous())
        yu, yp = run_apply(tng, ctx, mesh, tt, OPS_ALL, torch.float64)
        got = np.concatenate([lm.from_lib(yu).ravel(), lmp.from_lib(yp)])
        want = K[:, col].toarray().ravel()
        assert np.abs(got - want).max() < 1e-13 * np.abs(want).max(), col


# ---- hourglass control (eq:hgstab) ---------------------------------------------------

HG = 0.05


@pytest.mark.parametrize("mt,nr,prec", [(8, 8, "f64"), (16, 10, "f64"), (8, 6, "f32"), (16, 16, "f32")])
def test_hourglass_controlled_operator(tng, ctx, mt, nr, prec):
    """K with the stabilised viscous block against the oracle assembled with the
    same alpha: full operator with Dirichlet rows and A alone without them."""
    import torch
    from oracle.stokes import StokesOracle
    mesh, om, lm, lmp, eta, u, p, orc, t = setup_case(tng, ctx, mt, nr)
    orh = StokesOracle(mt, nr, eta, hierarchy=om.h, hg_alpha=HG)
    dt, tol = (torch.float64, 1e-12) if prec == "f64" else (torch.float32, 1e-5)
    e, uu, pp = (t[k].to(dt) for k in ("eta", "u", "p"))
    yu, yp = torch.full_like(uu, float("nan")), torch.full_like(pp, float("nan"))
    tng.stokes_apply(ctx, mesh, 0, OPS_ALL, e, uu, pp, yu, yp, hg_alpha=HG)
    ru, rp = orh.apply(u, p)
    gu, gp = lm.from_lib(yu.double().cpu().numpy()), lmp.from_lib(yp.double().cpu().numpy())
    print(f"hg {prec} ({mt},{nr}) rel u {rel(gu, ru):.2e} p {rel(gp, rp):.2e}")
    assert rel(gu, ru) < tol and rel(gp, rp) < tol
    # the stabilisation changes the result (it is not a no-op on random inputs)
    assert rel(ru, orc.apply(u, p)[0]) > 1e-3
    rng = np.random.default_rng(5)
    uf = rng.uniform(-1, 1, u.shape)
    ut = torch.tensor(lm.to_lib(uf), device="cuda").to(dt).contiguous()
    tng.stokes_apply(ctx, mesh, 0, 1, e, ut, None, yu, None, hg_alpha=HG)
    assert rel(lm.from_lib(yu.double().cpu().numpy()), (orh.A @ uf.ravel()).reshape(-1, 3)) < tol


# ---- radial split: a column handled by 2 or 4 waves of one workgroup -----------------

@pytest.mark.parametrize("mt,nr,prec", [(4, 96, "f64"), (4, 160, "f64"), (4, 320, "f64"),
                                         (4, 160, "f32"), (4, 288, "f32")])
def test_radial_split_columns(tng, ctx, mt, nr, prec):
    """Radial sizes that split a column among the waves of a workgroup, with a
    partly filled last stretch, empty stretches (FP64 nr 160 and 320, FP32 nr 288)
    and workgroup ranges with seams; every block with Dirichlet rows."""
    import torch
    mesh, om, lm, lmp, eta, u, p, orc, t = setup_case(tng, ctx, mt, nr)
    dt, tol = (torch.float64, 1e-12) if prec == "f64" else (torch.float32, 1e-5)
    yu, yp = run_apply(tng, ctx, mesh, t, OPS_ALL, dt)
    ru, rp = orc.apply(u, p)
    gu = lm.from_lib(yu, check_dups=1e-6)
    gp = lmp.from_lib(yp, check_dups=1e-6)
    print(f"split {prec} ({mt},{nr}) rel u {rel(gu, ru):.2e} p {rel(gp, rp):.2e}")
    assert rel(gu, ru) < tol and rel(gp, rp) < tol


# ---- band partition: bands of unequal length (forced through the context) -------------

@pytest.mark.parametrize("mt,nr,bands,prec", [(16, 16, 3, "f64"), (16, 10, 5, "f64"), (32, 8, 7, "f32"),
                                               (16, 16, 8, "f32"), (8, 8, 1, "f64")])
def test_forced_band_counts(tng, ctx, mt, nr, bands, prec):
    """Bands of 4-6, 2-4 and 4-6 rows (counts that do not divide the rows), eight
    two-row bands and a single band: the result does not depend on the partition."""
    import torch
    mesh, om, lm, lmp, eta, u, p, orc, t = setup_case(tng, ctx, mt, nr)
    dt, tol = (torch.float64, 1e-12) if prec == "f64" else (torch.float32, 1e-5)
    ctx.set_apply_bands(bands)
    try:
        yu, yp = run_apply(tng, ctx, mesh, t, OPS_ALL, dt)
    finally:
        ctx.set_apply_bands(0)
    ru, rp = orc.apply(u, p)
    gu = lm.from_lib(yu, check_dups=1e-6)
    gp = lmp.from_lib(yp, check_dups=1e-6)
    print(f"bands {bands} {prec} ({mt},{nr}) rel u {rel(gu, ru):.2e} p {rel(gp, rp):.2e}")
    assert rel(gu, ru) < tol and rel(gp, rp) < tol
