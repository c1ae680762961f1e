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


def check_rows(got, want, M, x, tol, what):
    """Element-wise bound |y - y_ref| <= tol * s per row, s = (|M| |x|)_row the
    sum of the magnitudes of the row's terms (a localised error at a few seam
    nodes cannot hide in a global norm)."""
    s = (abs(M) @ np.abs(np.asarray(x).ravel())).reshape(np.shape(want))
    # rows whose terms cancel exactly (a component on a symmetry plane) hold only the
    # rounding residue of the assembled entries: floor at 1e-15 of the largest row scale
    s = s + 1e-15 * s.max()
    err = np.abs(np.asarray(got) - np.asarray(want))
    ratio = err / np.maximum(s, 1e-300)
    worst = float(ratio.max()) if ratio.size else 0.0
    assert worst <= tol, f"{what}: worst error / row scale {worst:.2e} > {tol:.0e} " \
                         f"({int((ratio > tol).sum())} rows)"
    return worst


def check_K(orc, gu, gp, u, p, tol, what, K=None):
    K = orc.K if K is None else K
    x = np.concatenate([np.asarray(u).ravel(), np.asarray(p)])
    want = K @ x
    got = np.concatenate([np.asarray(gu).ravel(), np.asarray(gp)])
    return check_rows(got, want, K, x, tol, what)


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
    check_K(orc, gu, gp, u, p, 1e-12, f"fp64 ({mt},{nr})")


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
    check_K(orc, gu, gp, u, p, 1e-5, f"fp32 ({mt},{nr})")


def test_blocks_separately(tng, ctx):
    """A alone without Dirichlet, B^T alone and B alone with Dirichlet."""
    import torch
    mesh, om, lm, lmp, eta, u, p, orc, t = setup_case(tng, ctx, 8, 8)
    rng = np.random.default_rng(7)
    uf = rng.uniform(-1, 1, u.shape)                      # nonzero on the boundary
    tt = dict(t, u=torch.tensor(lm.to_lib(uf), device="cuda").contiguous())
    yu, _ = run_apply(tng, ctx, mesh, tt, 1, torch.float64)
    assert rel(lm.from_lib(yu), (orc.A @ uf.ravel()).reshape(-1, 3)) < 1e-12
    check_rows(lm.from_lib(yu).ravel(), orc.A @ uf.ravel(), orc.A, uf, 1e-12, "A")
    yu, _ = run_apply(tng, ctx, mesh, tt, 2 | 8, torch.float64)
    assert rel(lm.from_lib(yu), (orc.BT_D @ p).reshape(-1, 3)) < 1e-12
    check_rows(lm.from_lib(yu).ravel(), orc.BT_D @ p, orc.BT_D, p, 1e-12, "B^T_D")
    _, yp = run_apply(tng, ctx, mesh, tt, 4 | 8, torch.float64)
    assert rel(lmp.from_lib(yp), orc.B_D @ uf.ravel()) < 1e-12
    check_rows(lmp.from_lib(yp), orc.B_D @ uf.ravel(), orc.B_D, uf, 1e-12, "B_D")
    yu, _ = run_apply(tng, ctx, mesh, tt, 1 | 8, torch.float64)
    assert rel(lm.from_lib(yu), (orc.A_D @ uf.ravel()).reshape(-1, 3)) < 1e-12
    check_rows(lm.from_lib(yu).ravel(), orc.A_D @ uf.ravel(), orc.A_D, uf, 1e-12, "A_D")


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
    check_K(orh, gu, gp, u, p, tol, f"hg {prec} ({mt},{nr})")
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
    check_K(orc, gu, gp, u, p, tol, f"split {prec} ({mt},{nr})")


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
    check_K(orc, gu, gp, u, p, tol, f"bands {bands} {prec} ({mt},{nr})")


@pytest.mark.parametrize("prec,bands", [("f32", 0), ("f32", 8), ("f64", 0), ("f64", 6)])
def test_apply_is_bitwise_reproducible(tng, ctx, prec, bands):
    """Repeated applies of the full operator on the (32,32) shell, with the band
    count chosen per launch or forced, agree bit for bit: every node sums its
    partials in an order that does not depend on timing (coarse rows belong to one
    band each, tile seams take two atomic partials)."""
    import torch
    mesh = tng.Mesh(ctx, 32, 32, levels=2)
    dt = torch.float64 if prec == "f64" else torch.float32
    g = torch.Generator(device="cpu").manual_seed(21)
    t = {"u": torch.rand((3,) + mesh.shape(0), generator=g, dtype=torch.float64).cuda() * 2 - 1,
         "p": torch.rand(mesh.shape(1), generator=g, dtype=torch.float64).cuda() * 2 - 1,
         "eta": 10.0 ** (torch.rand(mesh.wedge_shape(0), generator=g, dtype=torch.float64).cuda() * 2 - 1)}
    tng.interface_sum(ctx, mesh, 0, [t["u"][0], t["u"][1], t["u"][2]], mode=1)
    tng.interface_sum(ctx, mesh, 1, [t["p"]], mode=1)
    ctx.set_apply_bands(bands)
    try:
        runs = [run_apply(tng, ctx, mesh, t, OPS_ALL, dt) for _ in range(4)]
    finally:
        ctx.set_apply_bands(0)
    for yu, yp in runs[1:]:
        assert np.array_equal(yu, runs[0][0]) and np.array_equal(yp, runs[0][1])


# ---- argument checks of the C entry points and the bandwidth probe --------------------

def test_device_pointer_checks(tng, ctx):
    """The check every entry point applies to its device pointers: host and pinned-host
    memory are refused, device memory is accepted only up to its allocation's end.
    (tng_check_device_buffer launches nothing, whatever it is given.)"""
    import torch
    a = np.zeros(1000)
    with pytest.raises(tng.TngError, match="device memory"):
        tng.check_device_buffer(ctx, a.ctypes.data, a.nbytes)
    pinned = torch.zeros(1000, dtype=torch.float64, pin_memory=True)
    with pytest.raises(tng.TngError, match="device memory"):
        tng.check_device_buffer(ctx, pinned.data_ptr(), 8000)
    t = torch.zeros(1000, dtype=torch.float64, device="cuda")
    tng.check_device_buffer(ctx, t.data_ptr(), 8000)
    with pytest.raises(tng.TngError, match="too small"):
        tng.check_device_buffer(ctx, t.data_ptr(), 64 << 20)


def test_stream_copy(tng, ctx):
    import torch
    for n in (1 << 22, 4 * 12345 + 4):                # whole trips, and a ragged tail
        x = torch.randn(n, dtype=torch.float32, device="cuda")
        y = torch.full_like(x, float("nan"))
        tng.stream_copy(ctx, x, y)
        torch.cuda.synchronize()
        assert torch.equal(x, y)


# ---- free slip (Sec. 8 setup): rotated normal constraint on one or both spheres ---------

FS_IN, FS_OUT = 16, 32


@pytest.mark.parametrize("mt,nr,bc,prec", [
    (8, 8, ("freeslip", "freeslip"), "f64"), (16, 10, ("noslip", "freeslip"), "f64"),
    (8, 6, ("freeslip", "noslip"), "f64"), (16, 16, ("freeslip", "freeslip"), "f32"),
    (4, 160, ("freeslip", "freeslip"), "f64"), (4, 288, ("noslip", "freeslip"), "f32")])
def test_freeslip_operator(tng, ctx, mt, nr, bc, prec):
    """K with free slip (y_u = P (A P u + B^T p) + N u on the free-slip spheres, y_p = B P u)
    against the oracle assembled with the same conditions, element-wise, including radial
    splits (nr 160, 288); then A, B^T and B alone."""
    import torch
    mesh, om, lm, lmp, eta, u, p, orc, t = setup_case(tng, ctx, mt, nr)
    orf = StokesOracle(mt, nr, eta, hierarchy=om.h, bc=bc)
    rng = np.random.default_rng(9)
    uf = rng.uniform(-1, 1, u.shape)                     # nonzero on both spheres
    flags = OPS_ALL | (FS_IN if bc[0] == "freeslip" else 0) | (FS_OUT if bc[1] == "freeslip" else 0)
    dt, tol = (torch.float64, 1e-12) if prec == "f64" else (torch.float32, 1e-5)
    e = t["eta"].to(dt)
    ut = torch.tensor(lm.to_lib(uf), device="cuda").to(dt).contiguous()
    pt = t["p"].to(dt)
    yu, yp = torch.full_like(ut, float("nan")), torch.full_like(pt, float("nan"))
    tng.stokes_apply(ctx, mesh, 0, flags, e, ut, pt, yu, yp)
    gu = lm.from_lib(yu.double().cpu().numpy(), check_dups=1e-6)
    gp = lmp.from_lib(yp.double().cpu().numpy(), check_dups=1e-6)
    ru, rp = orf.apply(uf, p)
    print(f"freeslip {bc} {prec} ({mt},{nr}) rel u {rel(gu, ru):.2e} p {rel(gp, rp):.2e}", flush=True)
    assert rel(gu, ru) < tol and rel(gp, rp) < tol
    check_K(orf, gu, gp, uf, p, tol, f"freeslip {bc} {prec} ({mt},{nr})")
    # the condition changes the result (not the no-slip operator)
    assert rel(ru, orc.apply(uf, p)[0]) > 1e-3
    fsb = flags & (FS_IN | FS_OUT)
    # row scales from the magnitudes of the terms before they cancel: the projection
    # y - rhat (rhat . y) has terms |y_c| and |rhat_c| (|rhat| . |y|) (a node whose rhat lies
    # on a coordinate axis has a zero row of P, where the oracle's P holds rounding residue),
    # and B = P_iso^T B_f
    Pa = abs(orf.P_bc) + abs(orf.N_bc)
    Na = abs(orf.N_bc)
    Bf, Pi = abs(orf.Bf), abs(orf.P)
    scales = {1 | 8: lambda x: Pa @ (abs(orf.A) @ (Pa @ np.abs(x))) + Na @ np.abs(x),
              2 | 8: lambda x: Pa @ (Bf.T @ (Pi @ np.abs(x))),
              4 | 8: lambda x: Pi.T @ (Bf @ (Pa @ np.abs(x)))}
    for blk, M, x in ((1 | 8, orf.A_D, uf), (2 | 8, orf.BT_D, p), (4 | 8, orf.B_D, uf)):
        yu.fill_(float("nan"))
        yp.fill_(float("nan"))
        tng.stokes_apply(ctx, mesh, 0, blk | fsb, e, ut if blk != (2 | 8) else None,
                         pt if blk == (2 | 8) else None, yu if blk != (4 | 8) else None, yp if blk == (4 | 8) else None)
        if blk == (4 | 8):
            got = lmp.from_lib(yp.double().cpu().numpy())
        else:
            got = lm.from_lib(yu.double().cpu().numpy()).ravel()
        want = M @ np.asarray(x).ravel()
        assert rel(got, want) < tol, blk
        sc = scales[blk](np.asarray(x).ravel())
        sc = sc + 1e-15 * sc.max()
        ratio = np.abs(got - want) / np.maximum(sc, 1e-300)
        worst = float(ratio.max())
        if worst > tol:
            bad = np.flatnonzero(ratio > tol)
            nodes = bad // 3 if blk != (4 | 8) else bad
            n1 = (nr + 1) if blk != (4 | 8) else (nr // 2 + 1)
            lat = lm.slot2lat if blk != (4 | 8) else lmp.slot2lat
            mult = np.bincount(lat)
            print("bad rows (row, lateral node, k, copies, got, want, scale):", flush=True)
            for b_, nd in list(zip(bad, nodes))[:12]:
                print(int(b_), int(nd // n1), int(nd % n1), int(mult[nd // n1]), got[b_], want[b_], sc[b_], flush=True)
        assert worst <= tol, f"freeslip block {blk}: worst error / row scale {worst:.2e}"


# ---- compressible (TALA) terms: div(rhobar u) rows and the rhobar alphabar T' buoyancy ----------

TALA = 64


def _rho(r):
    return np.exp(np.log(1.6) * (1.0 - r) / 0.45)


@pytest.mark.parametrize("mt,nr,prec,bands", [(8, 8, "f64", 0), (16, 10, "f64", 3), (16, 16, "f32", 0),
                                               (4, 160, "f64", 0), (4, 288, "f32", 0), (32, 8, "f32", 7)])
def test_tala_operator(tng, ctx, mt, nr, prec, bands):
    """K and B alone with the reference density against the oracle (B_rho = B R), element-wise;
    including radial splits and forced band counts."""
    import torch
    mesh, om, lm, lmp, eta, u, p, orc, t = setup_case(tng, ctx, mt, nr)
    rho = _rho(om.r)
    mesh.set_density(rho)
    ort = StokesOracle(mt, nr, eta, hierarchy=om.h, rho_nodes=rho)
    dt, tol = (torch.float64, 1e-12) if prec == "f64" else (torch.float32, 1e-5)
    e, uu, pp = (t[k].to(dt) for k in ("eta", "u", "p"))
    ctx.set_apply_bands(bands)
    try:
        yu, yp = torch.full_like(uu, float("nan")), torch.full_like(pp, float("nan"))
        tng.stokes_apply(ctx, mesh, 0, OPS_ALL | TALA, e, uu, pp, yu, yp)
        yb = torch.full_like(pp, float("nan"))
        tng.stokes_apply(ctx, mesh, 0, 4 | 8 | TALA, None, uu, None, None, yb)
    finally:
        ctx.set_apply_bands(0)
    gu, gp = lm.from_lib(yu.double().cpu().numpy(), check_dups=1e-6), lmp.from_lib(yp.double().cpu().numpy())
    ru, rp = ort.apply(u, p)
    print(f"tala {prec} ({mt},{nr}) bands {bands}: rel u {rel(gu, ru):.2e} p {rel(gp, rp):.2e}", flush=True)
    assert rel(gu, ru) < tol and rel(gp, rp) < tol
    check_K(ort, gu, gp, u, p, tol, f"tala {prec} ({mt},{nr})")
    assert rel(rp, orc.apply(u, p)[1]) > 1e-3                    # the density matters
    gb = lmp.from_lib(yb.double().cpu().numpy(), check_dups=1e-6)
    check_rows(gb, ort.B_mass @ u.ravel(), ort.B_mass, u, tol, "B_rho")


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_tala_buoyancy(tng, ctx, prec):
    import torch
    from oracle.stokes import buoyancy_rhs_tala
    mesh, om, lm, lmp, eta, u, p, orc, t = setup_case(tng, ctx, 16, 10)
    rng = np.random.default_rng(12)
    T = rng.uniform(0.0, 1.0, om.n_nodes)
    Tbar = np.linspace(1.0, 0.0, om.nr + 1) ** 1.5
    ra = _rho(om.r) * np.exp(-np.log(3.0) * (1.0 - om.r) / 0.45)
    dt, tol = (torch.float64, 1e-12) if prec == "f64" else (torch.float32, 1e-5)
    Tt = torch.tensor(lm.to_lib(T), device="cuda").to(dt)
    f = torch.full((3,) + mesh.shape(0), float("nan"), dtype=dt, device="cuda")
    tng.rhs_buoyancy_tala(ctx, mesh, 0, Tt, 1e5, Tbar, ra, f)
    got = lm.from_lib(f.double().cpu().numpy(), check_dups=1e-6)
    want = buoyancy_rhs_tala(om, T, 1e5, Tbar, ra)
    want[om.boundary_nodes()] = 0.0
    print(f"tala buoyancy {prec}: rel {rel(got, want):.2e}", flush=True)
    assert rel(got, want) < tol


# ---- two-radial-point rule for the viscous block (Sec. 4) --------------------------------

TWOPT = 128


@pytest.mark.parametrize("mt,nr,prec", [(8, 8, "f64"), (16, 10, "f64"), (16, 16, "f32"), (4, 160, "f64"),
                                         (4, 288, "f32")])
def test_two_point_operator(tng, ctx, mt, nr, prec):
    """K and A with the viscous block on two radial points against the oracle assembled
    with the same rule, element-wise, including radial splits."""
    import torch
    mesh, om, lm, lmp, eta, u, p, orc, t = setup_case(tng, ctx, mt, nr)
    or2 = StokesOracle(mt, nr, eta, hierarchy=om.h, quad="two")
    dt, tol = (torch.float64, 1e-12) if prec == "f64" else (torch.float32, 1e-5)
    e, uu, pp = (t[k].to(dt) for k in ("eta", "u", "p"))
    yu, yp = torch.full_like(uu, float("nan")), torch.full_like(pp, float("nan"))
    tng.stokes_apply(ctx, mesh, 0, OPS_ALL | TWOPT, e, uu, pp, yu, yp)
    gu, gp = lm.from_lib(yu.double().cpu().numpy(), check_dups=1e-6), lmp.from_lib(yp.double().cpu().numpy())
    ru, rp = or2.apply(u, p)
    print(f"two-point {prec} ({mt},{nr}): rel u {rel(gu, ru):.2e} p {rel(gp, rp):.2e}", flush=True)
    assert rel(gu, ru) < tol and rel(gp, rp) < tol
    check_K(or2, gu, gp, u, p, tol, f"two-point {prec} ({mt},{nr})")
    # the rule changes the operator (by O(dr^2): little on thin layers)
    assert rel(ru, orc.apply(u, p)[0]) > (1e-3 if nr <= 16 else 1e-6)
    rng = np.random.default_rng(13)
    uf = rng.uniform(-1, 1, u.shape)
    ut = torch.tensor(lm.to_lib(uf), device="cuda").to(dt).contiguous()
    tng.stokes_apply(ctx, mesh, 0, 1 | TWOPT, e, ut, None, yu, None)
    got = lm.from_lib(yu.double().cpu().numpy()).ravel()
    check_rows(got, or2.A @ uf.ravel(), or2.A, uf, tol, f"two-point A {prec} ({mt},{nr})")


@pytest.mark.parametrize("mt,nr,prec,bc", [(8, 8, "f64", ("noslip", "freeslip")), (16, 10, "f64", ("freeslip", "freeslip")),
                                            (16, 16, "f32", ("freeslip", "noslip")), (4, 160, "f64", ("noslip", "freeslip"))])
def test_tala_with_free_slip(tng, ctx, mt, nr, prec, bc):
    """The compressible mass rows with free-slip spheres: y_p = B R P u and the full
    operator against the oracle with both (B_mass = B R P), element-wise."""
    import torch
    mesh, om, lm, lmp, eta, u, p, orc, t = setup_case(tng, ctx, mt, nr)
    rho = _rho(om.r)
    mesh.set_density(rho)
    ort = StokesOracle(mt, nr, eta, hierarchy=om.h, rho_nodes=rho, bc=bc)
    fsb = (FS_IN if bc[0] == "freeslip" else 0) | (FS_OUT if bc[1] == "freeslip" else 0)
    dt, tol = (torch.float64, 1e-12) if prec == "f64" else (torch.float32, 1e-5)
    # nonzero on both spheres: a zero sphere velocity leaves the rows of the nodes whose
    # rhat lies on a coordinate axis (a zero row of P, N u = 0) with only rounding residue
    uf = np.random.default_rng(11).uniform(-1, 1, u.shape)
    e, pp = (t[k].to(dt) for k in ("eta", "p"))
    uu = torch.tensor(lm.to_lib(uf), device="cuda").to(dt).contiguous()
    yu, yp = torch.full_like(uu, float("nan")), torch.full_like(pp, float("nan"))
    tng.stokes_apply(ctx, mesh, 0, OPS_ALL | TALA | fsb, e, uu, pp, yu, yp)
    yb = torch.full_like(pp, float("nan"))
    tng.stokes_apply(ctx, mesh, 0, 4 | 8 | TALA | fsb, None, uu, None, None, yb)
    gu, gp = lm.from_lib(yu.double().cpu().numpy(), check_dups=1e-6), lmp.from_lib(yp.double().cpu().numpy())
    check_K(ort, gu, gp, uf, p, tol, f"tala+fs {prec} ({mt},{nr}) {bc}")
    gb = lmp.from_lib(yb.double().cpu().numpy(), check_dups=1e-6)
    check_rows(gb, ort.B_mass @ uf.ravel(), ort.B_mass, uf, tol, "B_rho P")
    # both options matter: not the free-slip operator without density, nor TALA with no slip
    orf = StokesOracle(mt, nr, eta, hierarchy=om.h, bc=bc)
    assert rel(gp, orf.apply(uf, p)[1]) > 1e-3
    assert rel(gp, StokesOracle(mt, nr, eta, hierarchy=om.h, rho_nodes=rho).apply(uf, p)[1]) > 1e-6
