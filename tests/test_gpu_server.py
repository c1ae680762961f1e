"""Request server (continuous admission of Stokes solves): each result is the
same alone and in the mix, requests that do not fit the budget are refused,
a failing request does not disturb the others, and a tight budget still
serves every request (slots are queued, reused and released)."""
import math

import numpy as np
import pytest

import synthetic

pytestmark = pytest.mark.gpu

LEVELS = [(8, 8), (16, 16)]


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


def request_fields(tng, ctx, mt, nr, seed):
    import torch
    mesh = tng.Mesh(None, mt, nr, levels=1)
    xyz, r = mesh.coords(0)
    T = synthetic.temperature(xyz.reshape(-1, 3), r, seed=seed, lmin=1, lmax=16)
    shape = (10, mt + 1, mt + 1, nr + 1)
    Tt = torch.tensor(T.reshape(shape), device="cuda")
    u = torch.empty((3,) + shape, dtype=torch.float64, device="cuda")
    p = torch.empty((10, mt // 2 + 1, mt // 2 + 1, nr // 2 + 1), dtype=torch.float64, device="cuda")
    return Tt, u, p


def test_alone_equals_in_mix(tng, ctx):
    import torch
    srv = tng.Server(ctx, LEVELS, budget_bytes=8 << 30, max_slots=4, mixed=1, rtol=1e-8)
    T0, u0, p0 = request_fields(tng, ctx, 16, 16, 1000)
    t = srv.submit(1, T0, 3.0, 1e5, u0, p0)
    srv.wait(t)
    r0 = srv.poll(t)
    assert r0["rc"] == 0 and r0["rel_res"] <= 1e-8
    alone_u, alone_p = u0.cpu().numpy().copy(), p0.cpu().numpy().copy()
    # the same request again, in a mix of six
    reqs = []
    for i in range(6):
        lvl = i % 2
        mt, nr = LEVELS[lvl]
        if i == 3:
            Tt, u, p = T0, torch.empty_like(u0), torch.empty_like(p0)
            lvl = 1
        else:
            Tt, u, p = request_fields(tng, ctx, mt, nr, 1001 + i)
        lc = 3.0 if i == 3 else 2.0 + 0.5 * i
        reqs.append((srv.submit(lvl, Tt, lc, 1e5, u, p), u, p))
    srv.wait(0)
    for t, u, p in reqs:
        r = srv.poll(t)
        assert r["done"] and r["rc"] == 0, r
    _, um, pm = reqs[3]
    du = np.linalg.norm(um.cpu().numpy() - alone_u) / np.linalg.norm(alone_u)
    dp = np.linalg.norm(pm.cpu().numpy() - alone_p) / np.linalg.norm(alone_p)
    print(f"alone vs mix: du {du:.2e} dp {dp:.2e}", srv.stats())
    assert du < 1e-7 and dp < 1e-7
    srv.close()


def test_budget_refusal(tng, ctx):
    srv = tng.Server(ctx, LEVELS, budget_bytes=1 << 20, max_slots=2, mixed=1)
    T, u, p = request_fields(tng, ctx, 8, 8, 5)
    with pytest.raises(tng.TngError) as e:
        srv.submit(0, T, 3.0, 1e5, u, p)
    assert e.value.code == -5
    srv.close()


def test_failed_request_is_isolated(tng, ctx):
    import torch
    srv = tng.Server(ctx, LEVELS, budget_bytes=8 << 30, max_slots=3, mixed=1)
    good = [request_fields(tng, ctx, 8, 8, 20 + i) for i in range(3)]
    bad = request_fields(tng, ctx, 8, 8, 30)
    bad[0][0, 1, 1, 2] = float("nan")
    tickets = [srv.submit(0, *g[:1], 3.0, 1e5, g[1], g[2]) for g in good[:1]]
    tb = srv.submit(0, bad[0], 3.0, 1e5, bad[1], bad[2])
    tickets += [srv.submit(0, g[0], 3.0, 1e5, g[1], g[2]) for g in good[1:]]
    srv.wait(0)
    assert srv.poll(tb)["rc"] == -4
    for t in tickets:
        r = srv.poll(t)
        assert r["rc"] == 0 and r["rel_res"] <= 1e-8
    srv.close()


def test_tight_budget_serves_everything(tng, ctx):
    """A budget of about two (16,16) slots (~20 MB each): requests queue and slots are
    reused (the release of another level's idle slot is tested below)."""
    srv = tng.Server(ctx, LEVELS, budget_bytes=45 << 20, max_slots=8, mixed=1)
    reqs = []
    for i in range(8):
        lvl = 1 if i < 5 else 0
        mt, nr = LEVELS[lvl]
        Tt, u, p = request_fields(tng, ctx, mt, nr, 40 + i)
        reqs.append(srv.submit(lvl, Tt, 2.5, 1e5, u, p))
    srv.wait(0)
    st = srv.stats()
    print("tight budget", st)
    assert st["bytes_in_use"] <= 45 << 20
    for t in reqs:
        assert srv.poll(t)["rc"] == 0
    srv.close()


def _slot_bytes(tng, ctx, level):
    """Device bytes of one solver slot of `level`, measured with a server of that level alone."""
    srv = tng.Server(ctx, [level], budget_bytes=8 << 30, max_slots=1, mixed=1)
    Tt, u, p = request_fields(tng, ctx, *level, 77)
    srv.wait(srv.submit(0, Tt, 2.0, 1e5, u, p))
    b = srv.stats()["bytes_in_use"]
    srv.close()
    return b


def _poll_until_done(srv, ticket, seconds):
    import time
    t_end = time.time() + seconds
    while time.time() < t_end:
        r = srv.poll(ticket)
        if r["done"]:
            return r
        time.sleep(0.05)
    return None


def test_starved_level_gets_an_idle_slot_released(tng, ctx):
    """The budget holds one (8,8) slot plus a little less than one (16,16) slot.  After an
    (8,8) request leaves its slot idle, a (16,16) request only fits if that idle slot is
    released; the server must do so by itself.  Polled against a host deadline, so a
    regression fails instead of waiting forever."""
    b8, b16 = _slot_bytes(tng, ctx, LEVELS[0]), _slot_bytes(tng, ctx, LEVELS[1])
    assert 0 < b8 < b16
    srv = tng.Server(ctx, LEVELS, budget_bytes=b8 + b16 - 1, max_slots=4, mixed=1)
    try:
        T8, u8, p8 = request_fields(tng, ctx, 8, 8, 61)
        r = _poll_until_done(srv, srv.submit(0, T8, 2.0, 1e5, u8, p8), 60.0)
        assert r is not None and r["rc"] == 0
        st = srv.stats()
        assert st["slots"] == 1 and st["busy"] == 0 and st["bytes_in_use"] == b8, st
        T16, u16, p16 = request_fields(tng, ctx, 16, 16, 62)
        r = _poll_until_done(srv, srv.submit(1, T16, 2.0, 1e5, u16, p16), 60.0)
        st = srv.stats()
        print("starved level:", st, flush=True)
        assert r is not None, f"the (16,16) request was never admitted: {st}"
        assert r["rc"] == 0 and st["slots"] == 1 and st["bytes_in_use"] == b16, st
    finally:
        srv.close()


@pytest.mark.parametrize("mixed,nreq", [(1, 18), (0, 3)])
def test_batched_solves_match_direct_solve(tng, ctx, mixed, nreq):
    """Requests of one level run as one lockstep batch (18 requests: two launch
    groups of at most 16 slots, joining at different Krylov indices).  Every
    result is compared with the single-problem GPU solver on the same problem
    (eta = exp(-ln(c) T) per wedge, f = Ra T rhat with zero Dirichlet rows), and
    the first and last with the oracle's sparse direct solve."""
    import torch
    from oracle.mesh import ShellMesh
    from oracle.stokes import StokesOracle, buoyancy_rhs, eta_from_temperature
    from tests._support import LayoutMap
    mt = 8
    om = ShellMesh(mt, mt)
    omp = ShellMesh(mt // 2, mt // 2, hierarchy=om.h)
    mesh = tng.Mesh(ctx, mt, mt, levels=3)          # the server's hierarchy of (8,8): down to (2,2)
    lm, lmp = LayoutMap(*mesh.coords(0), om), LayoutMap(*mesh.coords(1), omp)
    # rtol 1e-11: the buoyancy-driven velocity is small next to the pressure, so a
    # relative residual of 1e-10 leaves velocity errors near 1e-7 at contrast 10^1.5
    opts = dict(mixed=mixed, rtol=1e-11, max_iters=800)
    srv = tng.Server(ctx, LEVELS, budget_bytes=8 << 30, max_slots=nreq, **opts)
    Ra = 1e5
    reqs = []
    for i in range(nreq):
        T = synthetic.temperature(om.s, om.r, seed=500 + i, lmin=1, lmax=8).ravel()
        lc = 1.5 + 1.5 * i / max(nreq - 1, 1)
        Tt = torch.tensor(lm.to_lib(T), device="cuda")
        u = torch.empty((3,) + lm.shape, dtype=torch.float64, device="cuda")
        p = torch.empty(lmp.shape, dtype=torch.float64, device="cuda")
        reqs.append((srv.submit(0, Tt, lc, Ra, u, p), T, lc, u, p, Tt))
    srv.wait(0)
    st = srv.stats()
    single = tng.StokesSolver(ctx, mesh, **opts)
    worst_single = worst_oracle = 0.0
    for k, (t, T, lc, u, p, Tt) in enumerate(reqs):
        r = srv.poll(t)
        assert r["done"] and r["rc"] == 0 and r["rel_res"] <= 1e-11, r
        gu = lm.from_lib(u.cpu().numpy(), check_dups=1e-12)
        gp = lmp.from_lib(p.cpu().numpy(), check_dups=1e-12)
        eta = torch.empty(mesh.wedge_shape(0), dtype=torch.float64, device="cuda")
        tng.eta_from_temperature(ctx, mesh, 0, Tt, lc * np.log(10.0), 0.0, eta)
        f = torch.empty((3,) + mesh.shape(0), dtype=torch.float64, device="cuda")
        tng.rhs_buoyancy(ctx, mesh, 0, Tt, Ra, f)
        us, ps = torch.empty_like(u), torch.empty_like(p)
        info = single.solve(f, None, us, ps, eta=eta)
        assert info["rel_res"] <= 1e-11
        su, sp_ = lm.from_lib(us.cpu().numpy()), lmp.from_lib(ps.cpu().numpy())
        du = np.linalg.norm(gu - su) / np.linalg.norm(su)
        dp = np.linalg.norm(gp - sp_) / np.linalg.norm(sp_)
        worst_single = max(worst_single, du, dp)
        assert du < 1e-8 and dp < 1e-8, (k, lc, du, dp)
        if k in (0, nreq - 1):
            eta_o = eta_from_temperature(om, T, lc * np.log(10.0))
            fo = buoyancy_rhs(om, T, Ra)
            fo[om.boundary_nodes()] = 0.0
            uo, po = StokesOracle(mt, mt, eta_o, hierarchy=om.h).solve(fo)
            eu = np.linalg.norm(gu - uo) / np.linalg.norm(uo)
            ep = np.linalg.norm(gp - po) / np.linalg.norm(po)
            worst_oracle = max(worst_oracle, eu, ep)
            assert eu < 1e-7 and ep < 1e-7, (k, lc, eu, ep)
        print(f"request {k}: contrast 10^{lc:.2f}, {r['inner_its']} its, vs single {max(du, dp):.1e}", flush=True)
    single.close()
    print(f"batched mixed={mixed}: {nreq} requests, {st['slots']} slots, worst vs single solver "
          f"{worst_single:.2e}, vs direct solve {worst_oracle:.2e}")
    srv.close()
