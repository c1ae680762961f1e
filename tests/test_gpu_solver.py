"""GPU parity of the multigrid pieces and of the Stokes solve (Sec. 7) with
the FP64 oracle: operator diagonal, lumped pressure mass, transfers,
Chebyshev smoother, V-cycle symmetry, and the solution of K_D x = b compared
with the oracle's sparse direct solve."""
import numpy as np
import pytest

import synthetic
from oracle.mesh import ShellMesh
from oracle.solver_ref import chebyshev, lumped_pressure_mass, restrict_velocity, velocity_prolongation
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


_cache = {}


def case(tng, ctx, mt, seed=0):
    if (mt, seed) in _cache:
        return _cache[(mt, seed)]
    import torch
    levels = int(np.log2(mt))           # down to (2, 2)
    mesh = tng.Mesh(ctx, mt, mt, levels=levels)
    om = ShellMesh(mt, mt)
    omp = ShellMesh(mt // 2, mt // 2, hierarchy=om.h)
    lm = LayoutMap(*mesh.coords(0), om)
    lmp = LayoutMap(*mesh.coords(1), omp)
    eta, _, _ = synthetic.uniform_operator_inputs(om.n_wedges, om.n_nodes, omp.n_nodes, seed)
    orc = StokesOracle(mt, mt, eta, hierarchy=om.h)
    eta_t = torch.tensor(eta[lm.wedge_index()], device="cuda")
    _cache[(mt, seed)] = (mesh, om, omp, lm, lmp, eta, orc, eta_t)
    return _cache[(mt, seed)]


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def vel(lm, arr):
    import torch
    return torch.tensor(lm.to_lib(arr), device="cuda").contiguous()


@pytest.mark.parametrize("mt", [8, 16])
def test_diag_and_pressure_mass(tng, ctx, mt):
    import torch
    mesh, om, omp, lm, lmp, eta, orc, eta_t = case(tng, ctx, mt)
    d = torch.empty((3,) + mesh.shape(0), dtype=torch.float64, device="cuda")
    tng.diag_A(ctx, mesh, 0, eta_t, d)
    pm = torch.empty(mesh.shape(1), dtype=torch.float64, device="cuda")
    tng.pressure_mass(ctx, mesh, 0, eta_t, pm)
    torch.cuda.synchronize()
    assert rel(lm.from_lib(d.cpu().numpy(), check_dups=1e-13), orc.diag_A()) < 1e-12
    assert rel(lmp.from_lib(pm.cpu().numpy(), check_dups=1e-13), lumped_pressure_mass(orc, eta)) < 1e-12


def test_transfers(tng, ctx):
    import torch
    mesh, om, omp, lm, lmp, eta, orc, eta_t = case(tng, ctx, 8)
    lmc = LayoutMap(*mesh.coords(1), omp)
    rng = np.random.default_rng(3)
    f = rng.standard_normal((om.n_nodes, 3))
    f[om.boundary_nodes()] = 0.0
    c = torch.empty((3,) + mesh.shape(1), dtype=torch.float64, device="cuda")
    tng.restrict(ctx, mesh, 0, vel(lm, f), c)
    cc = rng.standard_normal((omp.n_nodes, 3))
    cc[omp.boundary_nodes()] = 0.0
    fo = torch.empty((3,) + mesh.shape(0), dtype=torch.float64, device="cuda")
    tng.prolong(ctx, mesh, 0, vel(lmc, cc), fo)
    torch.cuda.synchronize()
    want_c = restrict_velocity(orc, f, omp.boundary_nodes())
    assert rel(lmc.from_lib(c.cpu().numpy(), check_dups=1e-13), want_c) < 1e-13
    want_f = (velocity_prolongation(orc) @ cc.ravel()).reshape(-1, 3)
    assert rel(lm.from_lib(fo.cpu().numpy(), check_dups=1e-13), want_f) < 1e-13


@pytest.mark.parametrize("mt", [8, 16])
@pytest.mark.parametrize("dtype,tol", [("float64", 1e-12), ("float32", 1e-5)])
def test_chebyshev_smoother(tng, ctx, dtype, tol, mt):
    """Two Chebyshev steps of degree 2 against the textbook iteration on the assembled
    operator: the smoother's two-term recurrence with the apply's closing pass fused
    into the update, on one tile per diamond row (8,8) and with tile seams (16,16)."""
    import torch
    dt = getattr(torch, dtype)
    mesh, om, omp, lm, lmp, eta, orc, eta_t = case(tng, ctx, mt)
    rng = np.random.default_rng(4)
    b = rng.standard_normal((om.n_nodes, 3))
    x = rng.standard_normal((om.n_nodes, 3))
    bnd = om.boundary_nodes()
    b[bnd] = 0.0
    x[bnd] = 0.0
    d = torch.empty((3,) + mesh.shape(0), dtype=dt, device="cuda")
    tng.diag_A(ctx, mesh, 0, eta_t.to(dt), d)
    xt = vel(lm, x).to(dt)
    tng.smooth(ctx, mesh, 0, eta_t.to(dt), d, vel(lm, b).to(dt), xt, 2, 2, 0.3, 3.3)
    want = chebyshev(orc.A_D, orc.diag_A().ravel(), b.ravel(), x.ravel(), 2, 2, 0.3, 3.3).reshape(-1, 3)
    got = lm.from_lib(xt.double().cpu().numpy(), check_dups=tol)
    print(f"chebyshev ({mt},{mt}) {dtype}: rel {rel(got, want):.2e}", flush=True)
    assert rel(got, want) < tol


@pytest.mark.parametrize("mixed", [0, 1])
def test_vcycle_is_symmetric(tng, ctx, mixed):
    """Symmetric smoothing and R = P^T make the V-cycle a symmetric operator."""
    import torch
    mesh, om, omp, lm, lmp, eta, orc, eta_t = case(tng, ctx, 16)
    s = tng.StokesSolver(ctx, mesh, mixed=mixed)
    s.setup(eta_t)
    dt = torch.float32 if mixed else torch.float64
    rng = np.random.default_rng(5)
    bnd = om.boundary_nodes()
    vs = []
    for _ in range(2):
        v = rng.standard_normal((om.n_nodes, 3))
        v[bnd] = 0.0
        vs.append(v)
    out = []
    for v in vs:
        x = torch.empty((3,) + mesh.shape(0), dtype=dt, device="cuda")
        s.vcycle(vel(lm, v).to(dt), x)
        torch.cuda.synchronize()
        out.append(lm.from_lib(x.double().cpu().numpy(), check_dups=1e-5 if mixed else 1e-12))
    a, b = np.sum(vs[0] * out[1]), np.sum(vs[1] * out[0])
    assert abs(a - b) / max(abs(a), abs(b)) < (1e-5 if mixed else 1e-11)
    # a useful preconditioner: positive on the interior
    assert np.sum(vs[0] * out[0]) > 0


@pytest.mark.parametrize("mt,mixed", [(8, 0), (8, 1)])
def test_solve_matches_direct_solve(tng, ctx, mt, mixed):
    """Solution of K_D [u; p] = [f; 0] vs the oracle's sparse direct solve."""
    import torch
    mesh, om, omp, lm, lmp, eta, orc, eta_t = case(tng, ctx, mt)
    rng = np.random.default_rng(6)
    f = rng.standard_normal((om.n_nodes, 3))
    f[om.boundary_nodes()] = 0.0
    s = tng.StokesSolver(ctx, mesh, mixed=mixed, rtol=1e-10, max_iters=400)
    u = torch.empty((3,) + mesh.shape(0), dtype=torch.float64, device="cuda")
    p = torch.empty(mesh.shape(1), dtype=torch.float64, device="cuda")
    info = s.solve(vel(lm, f), None, u, p, eta=eta_t)
    uo, po = orc.solve(f)
    gu = lm.from_lib(u.cpu().numpy(), check_dups=1e-12)
    gp = lmp.from_lib(p.cpu().numpy(), check_dups=1e-12)
    eu, ep = rel(gu, uo), rel(gp, po)
    print(f"solve ({mt},{mt}) mixed={mixed}: its {info['inner_its']} outer {info['outer_its']} "
          f"res {info['rel_res']:.2e} err u {eu:.2e} p {ep:.2e} t {info['seconds']:.3f}s")
    assert info["rel_res"] <= 1e-10
    assert eu < 1e-7 and ep < 1e-7


def test_mixed_matches_fp64_solve_16(tng, ctx):
    """(16,16): the sparse direct oracle solve is too slow here, so the mixed
    solve is compared with the FP64 GPU solve (both to 1e-10), which the
    (8,8) case ties to the oracle."""
    import torch
    mesh, om, omp, lm, lmp, eta, orc, eta_t = case(tng, ctx, 16)
    rng = np.random.default_rng(7)
    f = rng.standard_normal((om.n_nodes, 3))
    f[om.boundary_nodes()] = 0.0
    res = []
    for mixed in (0, 1):
        s = tng.StokesSolver(ctx, mesh, mixed=mixed, rtol=1e-10, max_iters=600)
        u = torch.empty((3,) + mesh.shape(0), dtype=torch.float64, device="cuda")
        p = torch.empty(mesh.shape(1), dtype=torch.float64, device="cuda")
        info = s.solve(vel(lm, f), None, u, p, eta=eta_t)
        print(f"solve (16,16) mixed={mixed}: its {info['inner_its']} outer {info['outer_its']} "
              f"res {info['rel_res']:.2e} t {info['seconds']:.3f}s")
        res.append((lm.from_lib(u.cpu().numpy()), lmp.from_lib(p.cpu().numpy())))
    assert rel(res[1][0], res[0][0]) < 1e-7
    assert rel(res[1][1], res[0][1]) < 1e-7


# ---- hourglass control (eq:hgstab) ---------------------------------------------------

HG = 0.05


def test_diag_with_hourglass_control(tng, ctx):
    import torch
    from oracle.stokes import StokesOracle
    mesh, om, omp, lm, lmp, eta, orc, eta_t = case(tng, ctx, 8)
    orh = StokesOracle(8, 8, eta, hierarchy=om.h, hg_alpha=HG)
    d = torch.empty((3,) + mesh.shape(0), dtype=torch.float64, device="cuda")
    tng.diag_A(ctx, mesh, 0, eta_t, d, hg_alpha=HG)
    assert rel(lm.from_lib(d.cpu().numpy(), check_dups=1e-13), orh.diag_A()) < 1e-12


@pytest.mark.parametrize("mixed", [0, 1])
def test_hourglass_controlled_solve_matches_direct_solve(tng, ctx, mixed):
    """With hg_alpha the solver solves the stabilised system on every level;
    its solution matches the oracle's direct solve of that system."""
    import torch
    from oracle.stokes import StokesOracle
    mesh, om, omp, lm, lmp, eta, orc, eta_t = case(tng, ctx, 8)
    orh = StokesOracle(8, 8, eta, hierarchy=om.h, hg_alpha=HG)
    rng = np.random.default_rng(6)
    f = rng.standard_normal((om.n_nodes, 3))
    f[om.boundary_nodes()] = 0.0
    s = tng.StokesSolver(ctx, mesh, mixed=mixed, rtol=1e-10, max_iters=400, hg_alpha=HG)
    u = torch.empty((3,) + mesh.shape(0), dtype=torch.float64, device="cuda")
    p = torch.empty(mesh.shape(1), dtype=torch.float64, device="cuda")
    info = s.solve(vel(lm, f), None, u, p, eta=eta_t)
    uo, po = orh.solve(f)
    eu = rel(lm.from_lib(u.cpu().numpy(), check_dups=1e-12), uo)
    ep = rel(lmp.from_lib(p.cpu().numpy(), check_dups=1e-12), po)
    print(f"hg solve (8,8) mixed={mixed}: its {info['inner_its']} res {info['rel_res']:.2e} "
          f"err u {eu:.2e} p {ep:.2e}")
    assert info["rel_res"] <= 1e-10
    assert eu < 1e-7 and ep < 1e-7


@pytest.mark.parametrize("mt,mixed", [(8, 0), (16, 0), (8, 1)])
def test_graph_preconditioner_equals_eager(tng, ctx, mt, mixed):
    """The preconditioner replayed as captured HIP graphs (one per Krylov
    index, with the FGMRES kernels and host read-backs between replays) gives
    exactly the solves of launching every kernel from the host, also after the
    same solver is set up again for another viscosity (graphs reused): every
    node of the operator apply sums its partials in an order that does not
    depend on timing (at most two atomic partials per node)."""
    import torch
    mesh, om, omp, lm, lmp, eta, orc, eta_t = case(tng, ctx, mt)
    rng = np.random.default_rng(9)
    f = rng.standard_normal((om.n_nodes, 3))
    f[om.boundary_nodes()] = 0.0
    eta2 = torch.tensor(rng.uniform(0.5, 50.0, eta_t.numel()), device="cuda").reshape(eta_t.shape)
    out = {}
    for graphs in (0, 1):
        s = tng.StokesSolver(ctx, mesh, mixed=mixed, rtol=1e-9, max_iters=400, graphs=graphs)
        for k, e in (("a", eta_t), ("b", eta2), ("a2", eta_t)):
            u = torch.empty((3,) + mesh.shape(0), dtype=torch.float64, device="cuda")
            p = torch.empty(mesh.shape(1), dtype=torch.float64, device="cuda")
            info = s.solve(vel(lm, f), None, u, p, eta=e)
            assert info["rel_res"] <= 1e-9
            out[(graphs, k)] = (u.cpu().numpy(), p.cpu().numpy(), info["inner_its"])
        s.close()
    for k in ("a", "b", "a2"):
        ue, pe, ie = out[(0, k)]
        ug, pg, ig = out[(1, k)]
        assert ie == ig and np.array_equal(ug, ue) and np.array_equal(pg, pe), (k, ie, ig)
    # the replays after re-setup reproduce the first solve bit for bit as well
    assert np.array_equal(out[(1, "a2")][0], out[(1, "a")][0])
    assert np.array_equal(out[(1, "a2")][1], out[(1, "a")][1])


# ---- operator variants of the solve: two-radial-point rule, compressible mass rows ----------

@pytest.mark.parametrize("dtype,tol", [("float64", 1e-12), ("float32", 1e-6)])
def test_diag_twopoint(tng, ctx, dtype, tol):
    """diag(A) of the two-radial-point operator against the oracle's assembled
    two-point matrix, entry by entry."""
    import torch
    mesh, om, omp, lm, lmp, eta, orc, eta_t = case(tng, ctx, 8)
    or2 = StokesOracle(8, 8, eta, hierarchy=om.h, quad="two")
    dt = getattr(torch, dtype)
    d = torch.empty((3,) + mesh.shape(0), dtype=dt, device="cuda")
    tng.diag_A(ctx, mesh, 0, eta_t.to(dt), d, twopoint=True)
    got = lm.from_lib(d.double().cpu().numpy(), check_dups=0.0)
    ref = or2.diag_A()
    assert np.max(np.abs(got - ref) / np.abs(ref)) < tol
    # the rule is really the two-point one: its diagonal is not the one-point diagonal
    assert np.max(np.abs(orc.diag_A() - ref) / np.abs(ref)) > 1e-3


def _variant_solve(tng, ctx, mesh, lm, lmp, f, eta_t, mixed, op_flags):
    import torch
    s = tng.StokesSolver(ctx, mesh, mixed=mixed, rtol=1e-10, max_iters=400, op_flags=op_flags)
    u = torch.empty((3,) + mesh.shape(0), dtype=torch.float64, device="cuda")
    p = torch.empty(mesh.shape(1), dtype=torch.float64, device="cuda")
    info = s.solve(vel(lm, f), None, u, p, eta=eta_t)
    s.close()
    return (lm.from_lib(u.cpu().numpy(), check_dups=1e-12), lmp.from_lib(p.cpu().numpy(), check_dups=1e-12),
            info)


@pytest.mark.parametrize("mixed", [0, 1])
def test_twopoint_solve_matches_direct_solve(tng, ctx, mixed):
    """With TNG_OP_TWOPOINT every viscous apply of the solve (outer operator,
    smoothers, residuals, diagonal, coarsest matrix) takes the two-radial-point
    rule; the solution matches the oracle's direct solve of the two-point system
    and differs from the one-point solution."""
    mesh, om, omp, lm, lmp, eta, orc, eta_t = case(tng, ctx, 8)
    or2 = StokesOracle(8, 8, eta, hierarchy=om.h, quad="two")
    rng = np.random.default_rng(6)
    f = rng.standard_normal((om.n_nodes, 3))
    f[om.boundary_nodes()] = 0.0
    gu, gp, info = _variant_solve(tng, ctx, mesh, lm, lmp, f, eta_t, mixed, tng.OP_TWOPOINT)
    uo, po = or2.solve(f)
    eu, ep = rel(gu, uo), rel(gp, po)
    print(f"two-point solve (8,8) mixed={mixed}: its {info['inner_its']} res {info['rel_res']:.2e} "
          f"err u {eu:.2e} p {ep:.2e}")
    assert info["rel_res"] <= 1e-10
    assert eu < 1e-7 and ep < 1e-7
    u1, _ = orc.solve(f)
    assert rel(u1, uo) > 1e-4


def _rho(r):
    return np.exp(np.log(1.6) * (1.0 - r) / 0.45)


@pytest.mark.parametrize("mixed", [0, 1])
def test_tala_solve_matches_direct_solve(tng, ctx, mixed):
    """With TNG_OP_TALA the outer operator's mass rows are -(psi, div(rhobar u));
    the solution of the (non-symmetric) system matches the oracle's direct solve
    with the same reference density, and differs from the Boussinesq solution."""
    mesh, om, omp, lm, lmp, eta, orc, eta_t = case(tng, ctx, 8)
    rho = _rho(om.r)
    mesh.set_density(rho)
    ort = StokesOracle(8, 8, eta, hierarchy=om.h, rho_nodes=rho)
    rng = np.random.default_rng(9)
    f = rng.standard_normal((om.n_nodes, 3))
    f[om.boundary_nodes()] = 0.0
    gu, gp, info = _variant_solve(tng, ctx, mesh, lm, lmp, f, eta_t, mixed, tng.OP_TALA)
    uo, po = ort.solve(f)
    eu, ep = rel(gu, uo), rel(gp, po)
    print(f"TALA solve (8,8) mixed={mixed}: its {info['inner_its']} res {info['rel_res']:.2e} "
          f"err u {eu:.2e} p {ep:.2e}")
    assert info["rel_res"] <= 1e-10
    assert eu < 1e-7 and ep < 1e-7
    # the discrete mass balance of the TALA rows holds for the computed velocity
    assert np.linalg.norm(ort.B_mass @ gu.ravel()) < 1e-6 * np.linalg.norm(ort.B_D @ gu.ravel())
    u1, _ = orc.solve(f)
    assert rel(u1, uo) > 1e-4


def test_solver_variant_options_are_checked(tng, ctx):
    mesh, om, omp, lm, lmp, eta, orc, eta_t = case(tng, ctx, 8)
    with pytest.raises(tng.TngError):
        tng.StokesSolver(ctx, mesh, op_flags=tng.OP_TWOPOINT, hg_alpha=0.05)
    with pytest.raises(tng.TngError):
        tng.StokesSolver(ctx, mesh, op_flags=tng.OP_TWOPOINT | tng.OP_TALA)
    with pytest.raises(tng.TngError):        # no free-slip form of the two-point rule
        tng.StokesSolver(ctx, mesh, op_flags=tng.OP_FREESLIP_OUTER | tng.OP_TWOPOINT)
    with pytest.raises(tng.TngError):
        tng.StokesSolver(ctx, mesh, op_flags=tng.OP_FREESLIP_OUTER, hg_alpha=0.05)


@pytest.mark.parametrize("side,mixed", [("outer", 0), ("outer", 1), ("inner", 0), ("inner", 1)])
def test_freeslip_solve_matches_direct_solve(tng, ctx, side, mixed):
    """Free slip on one sphere through the whole multigrid (projected smoother,
    transfers and coarsest matrix), no slip on the other: the solution matches the
    oracle's direct solve of that system with the pressure gauge of the no-slip case
    (mass rows modulo constants, zero-mean pressure).  The body force keeps a normal
    part on the free-slip sphere, which is the prescribed normal velocity there."""
    mesh, om, omp, lm, lmp, eta, orc, eta_t = case(tng, ctx, 8)
    bc = ("noslip", "freeslip") if side == "outer" else ("freeslip", "noslip")
    flag = tng.OP_FREESLIP_OUTER if side == "outer" else tng.OP_FREESLIP_INNER
    ofs = StokesOracle(8, 8, eta, hierarchy=om.h, bc=bc)
    rng = np.random.default_rng(13)
    f = rng.standard_normal((om.n_nodes, 3))
    k = np.tile(np.arange(9), om.n_lat)
    f[k == (0 if side == "outer" else 8)] = 0.0          # the no-slip sphere
    gu, gp, info = _variant_solve(tng, ctx, mesh, lm, lmp, f, eta_t, mixed, flag)
    uo, po, c = ofs.solve_gauged(f)
    eu, ep = rel(gu, uo), rel(gp, po)
    print(f"free-slip ({side}) solve (8,8) mixed={mixed}: its {info['inner_its']} res {info['rel_res']:.2e} "
          f"err u {eu:.2e} p {ep:.2e} multiplier {c:.2e}")
    assert info["rel_res"] <= 1e-10
    assert eu < 1e-7 and ep < 1e-7
    fsn = k == (8 if side == "outer" else 0)
    rhat = om.node_xyz()[fsn]
    rhat /= np.linalg.norm(rhat, axis=1)[:, None]
    assert np.allclose(np.sum(gu[fsn] * rhat, 1), np.sum(f[fsn] * rhat, 1), rtol=0, atol=1e-7)


@pytest.mark.parametrize("mixed", [0, 1])
def test_freeslip_both_spheres_solve_matches_direct_solve(tng, ctx, mixed):
    """Free slip on both spheres: the rigid rotations are a null space as well; for a
    body force orthogonal to them the solution, returned orthogonal to them, matches
    the oracle's gauged direct solve with the rotation constraints."""
    mesh, om, omp, lm, lmp, eta, orc, eta_t = case(tng, ctx, 8)
    bc = ("freeslip", "freeslip")
    ofs = StokesOracle(8, 8, eta, hierarchy=om.h, bc=bc)
    R = ofs.rotations()
    f = np.random.default_rng(16).standard_normal(3 * om.n_nodes)
    f -= R @ np.linalg.solve(R.T @ R, R.T @ f)
    f = f.reshape(-1, 3)
    gu, gp, info = _variant_solve(tng, ctx, mesh, lm, lmp, f, eta_t, mixed,
                                  tng.OP_FREESLIP_INNER | tng.OP_FREESLIP_OUTER)
    uo, po, c = ofs.solve_gauged(f)
    eu, ep = rel(gu, uo), rel(gp, po)
    print(f"free-slip (both) solve (8,8) mixed={mixed}: its {info['inner_its']} res {info['rel_res']:.2e} "
          f"err u {eu:.2e} p {ep:.2e} rotations {np.linalg.norm(R.T @ gu.ravel()):.1e}")
    assert info["rel_res"] <= 1e-10
    assert eu < 1e-7 and ep < 1e-7
    assert np.linalg.norm(R.T @ gu.ravel()) < 1e-9 * np.linalg.norm(R) * np.linalg.norm(gu)


@pytest.mark.parametrize("flags", ["inner", "outer", "both"])
def test_buoyancy_with_freeslip_rows(tng, ctx, flags):
    """tng_rhs_buoyancy_bc: the one-point buoyancy of the oracle, rows of a no-slip
    sphere zero, rows of a free-slip sphere without their normal part; element-wise."""
    import torch
    from oracle.stokes import buoyancy_rhs
    mesh, om, omp, lm, lmp, eta, orc, eta_t = case(tng, ctx, 8)
    bits = {"inner": tng.OP_FREESLIP_INNER, "outer": tng.OP_FREESLIP_OUTER,
            "both": tng.OP_FREESLIP_INNER | tng.OP_FREESLIP_OUTER}[flags]
    T = np.random.default_rng(17).uniform(0.0, 1.0, om.n_nodes)
    ref = buoyancy_rhs(om, T, 1e5)
    k = np.tile(np.arange(9), om.n_lat)
    rhat = om.node_xyz() / np.linalg.norm(om.node_xyz(), axis=1)[:, None]
    for layer, bit in ((0, tng.OP_FREESLIP_INNER), (8, tng.OP_FREESLIP_OUTER)):
        sel = k == layer
        if bits & bit:
            ref[sel] -= np.sum(ref[sel] * rhat[sel], 1)[:, None] * rhat[sel]
        else:
            ref[sel] = 0.0
    Tt = torch.tensor(lm.to_lib(T), device="cuda")
    f = torch.empty((3,) + mesh.shape(0), dtype=torch.float64, device="cuda")
    tng.rhs_buoyancy(ctx, mesh, 0, Tt, 1e5, f, bc_flags=bits)
    got = lm.from_lib(f.cpu().numpy(), check_dups=1e-12)
    scale = np.abs(ref).max()
    assert np.max(np.abs(got - ref)) < 1e-12 * scale


@pytest.mark.parametrize("mixed", [0, 1])
def test_tala_freeslip_solve_matches_direct_solve(tng, ctx, mixed):
    """The compressible mass rows with a free-slip outer sphere (no slip inside), the
    setup of the paper's production runs in its compressible form: against the
    oracle's gauged direct solve with both."""
    mesh, om, omp, lm, lmp, eta, orc, eta_t = case(tng, ctx, 8)
    rho = _rho(om.r)
    mesh.set_density(rho)
    bc = ("noslip", "freeslip")
    ofs = StokesOracle(8, 8, eta, hierarchy=om.h, bc=bc, rho_nodes=rho)
    rng = np.random.default_rng(18)
    f = rng.standard_normal((om.n_nodes, 3))
    k = np.tile(np.arange(9), om.n_lat)
    f[k == 0] = 0.0
    gu, gp, info = _variant_solve(tng, ctx, mesh, lm, lmp, f, eta_t, mixed, tng.OP_TALA | tng.OP_FREESLIP_OUTER)
    uo, po, c = ofs.solve_gauged(f)
    eu, ep = rel(gu, uo), rel(gp, po)
    print(f"TALA + free-slip solve (8,8) mixed={mixed}: its {info['inner_its']} res {info['rel_res']:.2e} "
          f"err u {eu:.2e} p {ep:.2e}")
    assert info["rel_res"] <= 1e-10
    assert eu < 1e-7 and ep < 1e-7


def test_contrast1e6_freeslip_both_matches_direct_solve(tng, ctx):
    """Free slip on both spheres under viscosity contrast 1e6 (eta = exp(-ln(1e6) Tbar),
    the hot inner sphere 1e6 weaker than the cold lid), FP64 and mixed, against the
    oracle's gauged direct solve with the rotation constraints on the (8,8) shell."""
    import torch
    from oracle.stokes import buoyancy_rhs, eta_from_temperature
    mt = 8
    mesh, om, omp, lm, lmp, _, _, _ = case(tng, ctx, mt)
    T = synthetic.temperature(om.s, om.r, seed=1, lmin=1, lmax=8, amp=0.01).ravel()
    eta = eta_from_temperature(om, T, np.log(1e6), 0.0)
    ofs = StokesOracle(mt, mt, eta, hierarchy=om.h, bc=("freeslip", "freeslip"))
    # the buoyancy with its normal part removed on both spheres, orthogonal to the rotations
    f = buoyancy_rhs(om, T, 1e5)
    rhat = om.node_xyz() / np.linalg.norm(om.node_xyz(), axis=1)[:, None]
    k = np.tile(np.arange(mt + 1), om.n_lat)
    sph = (k == 0) | (k == mt)
    f[sph] -= np.sum(f[sph] * rhat[sph], 1)[:, None] * rhat[sph]
    R = ofs.rotations()
    f = (f.ravel() - R @ np.linalg.solve(R.T @ R, R.T @ f.ravel())).reshape(-1, 3)
    uo, po, _ = ofs.solve_gauged(f)
    eta_t = torch.tensor(eta[lm.wedge_index()], device="cuda")
    bits = tng.OP_FREESLIP_INNER | tng.OP_FREESLIP_OUTER
    for mixed in (0, 1):
        s = tng.StokesSolver(ctx, mesh, mixed=mixed, rtol=1e-10, restart=23, max_iters=2000, max_outer=40,
                             op_flags=bits)
        u = torch.empty((3,) + mesh.shape(0), dtype=torch.float64, device="cuda")
        p = torch.empty(mesh.shape(1), dtype=torch.float64, device="cuda")
        info = s.solve(vel(lm, f), None, u, p, eta=eta_t, raise_on_fail=False)
        s.close()
        eu = rel(lm.from_lib(u.cpu().numpy(), check_dups=1e-12), uo)
        ep = rel(lmp.from_lib(p.cpu().numpy(), check_dups=1e-12), po)
        print(f"contrast 1e6, free slip both (8,8) mixed={mixed}: its {info['inner_its']} "
              f"(FP64 {info['fp64_its']}) refinements {info['outer_its']} res {info['rel_res']:.2e} "
              f"err u {eu:.2e} p {ep:.2e}", flush=True)
        assert info["rc"] == 0 and info["rel_res"] <= 1e-10
        assert eu < 1e-7 and ep < 1e-7
        assert info["fp64_its"] == (0 if mixed else info["inner_its"])


def test_mixed_falls_back_to_fp64_when_refinement_stalls(tng, ctx):
    """The contrast-1e6 free-slip (both spheres) solve on the (64,64) shell: the weak core
    turning against the lid is a near-null mode that FP32 inner solves cannot resolve at
    this resolution, the mixed refinement stalls and the solve finishes with FP64 inner
    FGMRES: it reaches the tolerance with FP32 iterations first and FP64 ones after, and
    its solution is the FP64 solve's (both to relative residual 1e-9)."""
    import torch
    mt = 64
    mesh = tng.Mesh(ctx, mt, mt, levels=6)
    xyz, r = mesh.coords(0)
    T = synthetic.temperature(xyz.reshape(-1, 3), r, seed=1, lmin=1, lmax=8, amp=0.01)
    Tt = torch.tensor(T.reshape(mesh.shape(0)), device="cuda", dtype=torch.float64)
    eta = torch.empty(mesh.wedge_shape(0), device="cuda", dtype=torch.float64)
    tng.eta_from_temperature(ctx, mesh, 0, Tt, float(np.log(1e6)), 0.0, eta)
    bits = tng.OP_FREESLIP_INNER | tng.OP_FREESLIP_OUTER
    f = torch.empty((3,) + mesh.shape(0), device="cuda", dtype=torch.float64)
    tng.rhs_buoyancy(ctx, mesh, 0, Tt, 1e5, f, bc_flags=bits)
    out = {}
    for mixed in (0, 1):
        s = tng.StokesSolver(ctx, mesh, mixed=mixed, rtol=1e-9, restart=23, max_iters=2000, max_outer=40,
                             op_flags=bits)
        u = torch.empty_like(f)
        p = torch.empty(mesh.shape(1), device="cuda", dtype=torch.float64)
        info = s.solve(f, None, u, p, eta=eta, raise_on_fail=False)
        if mixed:
            # a second solve on the same solver: the viscosity set up again (the FP64 level
            # operators redone at the next stall), the FP64 scratch, basis and preconditioner
            # graphs of the first fallback reused; the solves are deterministic
            u2, p2 = torch.empty_like(u), torch.empty_like(p)
            info2 = s.solve(f, None, u2, p2, eta=eta, raise_on_fail=False)
            assert {k: info2[k] for k in ("inner_its", "fp64_its", "outer_its", "rel_res", "rc")} == \
                   {k: info[k] for k in ("inner_its", "fp64_its", "outer_its", "rel_res", "rc")}
            assert torch.equal(u2, u) and torch.equal(p2, p)
        s.close()
        out[mixed] = (info, u, p)
        print(f"contrast 1e6, free slip both (64,64) mixed={mixed}: its {info['inner_its']} "
              f"(FP64 {info['fp64_its']}) refinements {info['outer_its']} res {info['rel_res']:.2e}", flush=True)
        assert info["rc"] == 0 and info["rel_res"] <= 1e-9
    info = out[1][0]
    assert 0 < info["fp64_its"] < info["inner_its"]      # FP32 first, then FP64
    du = float((out[1][1] - out[0][1]).norm() / out[0][1].norm())
    dp = float((out[1][2] - out[0][2]).norm() / out[0][2].norm())
    print(f"mixed vs FP64 solution: u {du:.2e} p {dp:.2e}", flush=True)
    assert du < 1e-7 and dp < 1e-7
