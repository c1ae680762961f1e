#!/usr/bin/env python3
"""Benchmark of the matrix-free wedge Stokes hot path on one MI355X.

Workload (the headline configuration): the spherical shell with velocity
mesh (mt, nr) = (128, 128) -- 163,842 lateral nodes x 129 layers, 63.4 M
velocity DoFs -- and W1 pressure on (64, 64) (2.66 M DoFs); temperature =
conductive profile + seeded spherical harmonics l = 1..8 of amplitude 0.01;
viscosity eta = exp(-ln(1e3) T + ln(10) (1 - r)) per wedge.

A timed step is one full Stokes operator apply y = K_D [u; p] in FP32 (A,
B^T, B, Dirichlet rows, diamond-interface sum); `value` is its throughput in
GDoF/s.  The same line also reports the FP64 apply, the FP64 solve of the
configuration to a 1e-8 relative residual, the mixed-precision solve of the
same shell with viscosity contrast 1e6 next to the FP64 solve of that field
(FGMRES(10) as in the paper, and the same solves with FGMRES(23)), a short
serving run (p50/p99 latency), the live roofline of the dominant kernel and
the CPU oracle baseline.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def shell_fields(tng, ctx, mesh, seed=1, lmax=8):
    import torch
    import synthetic
    xyz, r = mesh.coords(0)
    T = synthetic.temperature(xyz.reshape(-1, 3), r, seed=seed, lmin=1, lmax=lmax, amp=0.01)
    return torch.tensor(T.reshape(mesh.shape(0)), device="cuda", dtype=torch.float64)


def unique_dofs(mt, nr):
    return 3 * (10 * mt * mt + 2) * (nr + 1), (10 * (mt // 2) ** 2 + 2) * (nr // 2 + 1)


COUNTERS_MD = os.path.join(ROOT, "profiles", "stokes_apply_shell128_hbm_counters.md")


def kernel_sources_digest():
    """Digest of the apply kernel's sources and build flags (what the committed
    HBM counters were measured with)."""
    import hashlib
    from paper_2609_21633_amd import build
    h = hashlib.sha256()
    for rel in ("paper_2609_21633_amd/csrc/stokes_apply.hip", "paper_2609_21633_amd/csrc/wedge.hpp"):
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    flags = [c for c in build.hipcc_command("x") if c.startswith("-") and not c.startswith("-I") and c != "-o"]
    h.update(" ".join(flags).encode())
    return h.hexdigest()[:16]


def counter_traffic(key):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None
    when the kernel has changed since the counters were taken."""
    try:
        with open(COUNTERS_MD) as f:
            kv = dict(l.strip().split(": ", 1) for l in f if ": " in l and l.strip().split(":")[0].isidentifier())
    except OSError:
        return None
    if kv.get("sources") != kernel_sources_digest() or key not in kv:
        return None
    return float(kv[key])


def algorithmic_bytes(mesh, esize):
    """Minimal traffic of one K apply: read u and write y_u (3 node fields
    each), read two wedge viscosities per cell, read p and write y_p."""
    c0, c1 = mesh.counts(0), mesh.counts(1)
    return esize * (6 * c0["node_slots"] + 2 * c0["cells"] + 2 * c1["node_slots"])


def bench_apply(tng, ctx, mesh, T64, dtype, steps, warmup):
    import torch
    eta = torch.empty(mesh.wedge_shape(0), device="cuda", dtype=dtype)
    tng.eta_from_temperature(ctx, mesh, 0, T64.to(dtype), math.log(1e3), math.log(10.0), eta)
    g = torch.Generator(device="cpu").manual_seed(2)
    u = (torch.rand((3,) + mesh.shape(0), generator=g, dtype=torch.float64) * 2 - 1).to("cuda", dtype)
    p = (torch.rand(mesh.shape(1), generator=g, dtype=torch.float64) * 2 - 1).to("cuda", dtype)
    tng.interface_sum(ctx, mesh, 0, [u[0], u[1], u[2]], mode=1)
    tng.interface_sum(ctx, mesh, 1, [p], mode=1)
    yu, yp = torch.empty_like(u), torch.empty_like(p)
    flags = tng.OP_A | tng.OP_BT | tng.OP_B | tng.OP_DIRICHLET
    for _ in range(warmup):
        tng.stokes_apply(ctx, mesh, 0, flags, eta, u, p, yu, yp)
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        tng.stokes_apply(ctx, mesh, 0, flags, eta, u, p, yu, yp)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    kms, nl = ctx.kernel_stats("stokes_apply")
    ctx.profile(False)
    del eta, u, p, yu, yp
    return wall, kms / max(nl, 1)


def bench_solve(tng, ctx, mesh, T64, E, F, mixed, reps=2, restart=10):
    """Solves/s of the Stokes problem with eta = exp(-E T + F (1 - r)) and the
    buoyancy right-hand side 1e5 T rhat, to a 1e-8 relative residual (FGMRES(restart))."""
    import torch
    eta = torch.empty(mesh.wedge_shape(0), device="cuda", dtype=torch.float64)
    tng.eta_from_temperature(ctx, mesh, 0, T64, E, F, eta)
    f = torch.empty((3,) + mesh.shape(0), device="cuda", dtype=torch.float64)
    tng.rhs_buoyancy(ctx, mesh, 0, T64, 1e5, f)
    u = torch.empty_like(f)
    p = torch.empty(mesh.shape(1), device="cuda", dtype=torch.float64)
    s = tng.StokesSolver(ctx, mesh, mixed=mixed, rtol=1e-8, max_iters=600, restart=restart)
    infos = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = s.solve(f, None, u, p, eta=eta, raise_on_fail=False)
        torch.cuda.synchronize()
        info["wall"] = time.perf_counter() - t0
        infos.append(info)
    best = min(infos, key=lambda x: x["wall"])
    s.close()
    return best, (u.clone(), p.clone())


def bench_copy_roof(tng, ctx, nbytes=2 << 30, reps=10):
    """Practical HBM roof: the library's plain streaming copy (tng_stream_copy) of
    nbytes, 2 x nbytes moved per launch, HIP-event timed on the launch stream."""
    import torch
    x = torch.full((nbytes // 4,), 1.0, dtype=torch.float32, device="cuda")
    y = torch.zeros_like(x)
    for _ in range(3):
        tng.stream_copy(ctx, x, y)
    torch.cuda.synchronize()
    ctx.profile(True)
    for _ in range(reps):
        tng.stream_copy(ctx, x, y)
    ms, n = ctx.kernel_stats("stream_copy")
    ctx.profile(False)
    del x, y
    torch.cuda.empty_cache()
    t = ms / max(n, 1) * 1e-3
    return {"kernel": "stream_copy_kernel (16-byte vectors, 4 per thread and trip)", "bytes_per_launch": 2 * nbytes,
            "kernel_ms": round(t * 1e3, 4), "gbs": round(2 * nbytes / t / 1e9, 1)}


GOLDEN16 = os.path.join(ROOT, "tests", "golden", "stokes16_contrast1e6.npz")


def golden16_errors(tng, ctx, mixed):
    """The contrast-1e6 solve on the (16,16) copy of the workload, to the benchmarked 1e-8,
    against the oracle's exact discrete solution stored in tests/golden (written by the
    committed script next to it).  The library's slots are matched to the stored node order
    by their coordinates (stored with the solution)."""
    import numpy as np
    import torch
    from scipy.spatial import cKDTree
    import synthetic
    d = np.load(GOLDEN16)
    mesh = tng.Mesh(ctx, 16, 16, levels=4)

    def node_map(level, s_ref, r_ref):
        xyz, r = mesh.coords(level)
        assert np.allclose(r, r_ref, rtol=0, atol=1e-14)
        dist, lat = cKDTree(s_ref).query(xyz.reshape(-1, 3))
        assert dist.max() < 1e-9
        first = np.full(len(s_ref), -1)
        for slot in range(len(lat) - 1, -1, -1):
            first[lat[slot]] = slot
        return lat, first

    lat_u, first_u = node_map(0, d["s_u"], d["r_u"])
    _, first_p = node_map(1, d["s_p"], d["r_p"])
    # T on the stored nodes (the generator's recipe), scattered to the library slots
    T = synthetic.temperature(d["s_u"], d["r_u"], seed=1, lmin=1, lmax=8, amp=0.01)
    T_lib = torch.tensor(T[lat_u].reshape(mesh.shape(0)), device="cuda")
    eta = torch.empty(mesh.wedge_shape(0), device="cuda", dtype=torch.float64)
    tng.eta_from_temperature(ctx, mesh, 0, T_lib, math.log(1e6), 0.0, eta)
    f = torch.empty((3,) + mesh.shape(0), device="cuda", dtype=torch.float64)
    tng.rhs_buoyancy(ctx, mesh, 0, T_lib, 1e5, f)
    u = torch.empty_like(f)
    p = torch.empty(mesh.shape(1), device="cuda", dtype=torch.float64)
    s = tng.StokesSolver(ctx, mesh, mixed=mixed, rtol=1e-8, max_iters=4000, inner_max_iters=4000, max_outer=60)
    info = s.solve(f, None, u, p, eta=eta, raise_on_fail=False)
    s.close()
    n1, nc1 = 17, 9
    ug = u.cpu().numpy().reshape(3, -1, n1)[:, first_u, :].reshape(3, -1).T
    pg = p.cpu().numpy().reshape(-1, nc1)[first_p, :].ravel()
    return {"u": float(np.linalg.norm(ug - d["u"]) / np.linalg.norm(d["u"])),
            "p": float(np.linalg.norm(pg - d["p"]) / np.linalg.norm(d["p"])),
            "rel_res": info["rel_res"], "iterations": info["inner_its"], "rc": info["rc"]}


def variant_bytes(name):
    """Algorithmic bytes of one launch from a detailed timer name
    "stokes_apply/<f32|f64>/<variant>/<m>x<n>/b<bands>" or "energy_apply/<prec>/SUPG/<m>x<n>":
    every input read and every output written once (None for batched launches)."""
    parts = name.split("/")
    if len(parts) < 4 or "batch" in parts:
        return None
    kern, prec, var, size = parts[:4]
    es = 8 if prec == "f64" else 4
    m, n = (int(v) for v in size.split("x"))
    ns = 10 * (m + 1) ** 2 * (n + 1)
    cells = 10 * m * m * n
    npr = 10 * (m // 2 + 1) ** 2 * (n // 2 + 1)
    if kern == "energy_apply":
        return es * (5 if var == "SUPG" else 2) * ns         # T, u (3) in, y out; no flow: T in, y out
    # values moved per variant: u in / y out (3 node fields each), two viscosities per cell,
    # p in and y_p out (one pressure field each)
    table = {"A": 6 * ns + 2 * cells, "BT": 3 * ns + npr, "B": 3 * ns + npr,
             "A+BT": 6 * ns + 2 * cells + npr, "A+B": 6 * ns + 2 * cells + npr,
             "BT+B": 6 * ns + 2 * npr, "K": 6 * ns + 2 * cells + 2 * npr}
    b = table[var.replace("+HG", "")]
    return es * b


def bench_energy_apply(tng, ctx, mt, nr, steps, warmup):
    """The SUPG energy apply y = E(u) T alone on the (mt, nr) shell, FP64 and FP32:
    kernel time from HIP events on the launch stream, wall time per call (with the
    tile-seam zeroing, interface sum and Dirichlet rows), and the algorithmic
    bandwidth (T and u read, y written once: 5 values per node slot)."""
    import torch
    mesh = tng.Mesh(ctx, mt, nr, levels=1)
    T64 = shell_fields(tng, ctx, mesh, seed=4, lmax=8)
    g = torch.Generator(device="cpu").manual_seed(6)
    # velocities of the coupled Ra 1e7 runs' magnitude (|u| up to a few hundred)
    u64 = ((torch.rand((3,) + mesh.shape(0), generator=g, dtype=torch.float64) * 2 - 1) * 300.0).to("cuda")
    tng.interface_sum(ctx, mesh, 0, [u64[0], u64[1], u64[2]], mode=1)
    ns = mesh.counts(0)["node_slots"]
    out = {"workload": f"SUPG energy apply on the ({mt},{nr}) shell, T = conduction + spherical harmonics "
                       "l=1..8, u = U(-300, 300) per component, dt = 1e-4",
           "node_slots": ns}
    for name, dtype, es in (("f64", torch.float64, 8), ("f32", torch.float32, 4)):
        T, u = T64.to(dtype), u64.to(dtype)
        y = torch.empty_like(T)
        for _ in range(warmup):
            tng.energy_apply(ctx, mesh, 0, u, 1e-4, T, y)
        torch.cuda.synchronize()
        ctx.profile(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            tng.energy_apply(ctx, mesh, 0, u, 1e-4, T, y)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps
        kms, nl = ctx.kernel_stats("energy_apply")
        ctx.profile(False)
        kms /= max(nl, 1)
        ab = 5 * es * ns
        out[name] = {"kernel_ms": round(kms, 4), "wall_ms": round(wall * 1e3, 4), "alg_bytes": ab,
                     "alg_gbs": round(ab / (kms * 1e-3) / 1e9, 1),
                     "frac": round(ab / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        log(f"[bench] energy apply {name}: {out[name]}")
        del T, u, y
        torch.cuda.empty_cache()
    # one plain streaming copy of known size: the practical roof, and the scale of HBM
    # byte counters taken over this run
    out["practical_roof"] = bench_copy_roof(tng, ctx, reps=2)
    return out


def bench_coupled(tng, ctx, mt, nr, steps):
    """Coupled Stokes-energy time stepping: per step a mixed-precision Stokes solve to 1e-8
    with eta(T) and the buoyancy Ra T rhat, then a backward-Euler SUPG energy step with
    internal heating.  Reports the time per step and each kernel's algorithmic GB/s."""
    import numpy as np
    import torch
    import synthetic
    levels = int(math.log2(mt))
    mesh = tng.Mesh(ctx, mt, nr, levels=levels)
    T = shell_fields(tng, ctx, mesh, seed=4, lmax=8)
    H = torch.tensor(np.random.default_rng(5).uniform(0.0, 10.0, mesh.shape(0)), device="cuda")
    tng.interface_sum(ctx, mesh, 0, [T, H], mode=1)
    u = torch.zeros((3,) + mesh.shape(0), device="cuda", dtype=torch.float64)
    p = torch.zeros(mesh.shape(1), device="cuda", dtype=torch.float64)
    sv = tng.StokesSolver(ctx, mesh, mixed=1, rtol=1e-8, max_iters=600, inner_max_iters=60, max_outer=40)
    per_step = []
    ctx.profile(True)
    for st in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = sv.energy_step(T, u, p, H=H, Ra=1e7, E=math.log(1e3), F=math.log(10.0), courant=1.0,
                              raise_on_fail=False)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        per_step.append({"seconds": round(wall, 3), "stokes_inner_its": info["stokes"]["inner_its"],
                         "stokes_outer_its": info["stokes"]["outer_its"],
                         "stokes_rel_res": info["stokes"]["rel_res"], "energy_its": info["energy_its"],
                         "dt": info["dt"]})
        log(f"[bench] coupled step {st}: {per_step[-1]}")
    kernels = {}
    for name, (ms, n) in sorted(ctx.kernel_stats_all().items()):
        b = variant_bytes(name)
        kernels[name] = {"launches": n, "avg_us": round(ms / n * 1e3, 2),
                         "alg_gbs": None if b is None else round(b / (ms / n * 1e-3) / 1e9, 1)}
    ctx.profile(False)
    sv.close()
    secs = [s["seconds"] for s in per_step]
    return {"workload": f"coupled Stokes-energy steps on the ({mt},{nr}) shell, Ra 1e7, "
                        "eta = exp(-ln(1e3) T + ln(10)(1-r)), H = U(0,10)",
            "steps": steps, "seconds_per_step_mean": round(sum(secs) / len(secs), 3),
            "seconds_per_step_after_first": round(sum(secs[1:]) / max(len(secs) - 1, 1), 3),
            "per_step": per_step, "kernels": kernels}


def vcycle_rates(tng, ctx, mesh, eta, cycles=9, **variant):
    """Residual reduction per cycle of the stand-alone V-cycle on the viscous block
    A_D (x <- x + V(b - A x), b = 0, a seeded random start holding every mode), the
    solver's V-cycle with the same operator variant on every level."""
    import torch
    s = tng.StokesSolver(ctx, mesh, mixed=0, **variant)
    s.setup(eta)
    shp = (3,) + mesh.shape(0)
    gen = torch.Generator(device="cpu").manual_seed(3)
    x = (torch.rand(shp, generator=gen, dtype=torch.float64) - 0.5).cuda()
    x[..., 0] = 0.0
    x[..., -1] = 0.0
    tng.interface_sum(ctx, mesh, 0, [x[0], x[1], x[2]], mode=1)
    y, c = torch.empty_like(x), torch.empty_like(x)
    flags = tng.OP_A | tng.OP_DIRICHLET | variant.get("op_flags", 0)
    rates, prev = [], None
    for _ in range(cycles + 1):
        tng.stokes_apply(ctx, mesh, 0, flags, eta, x, None, y, None, hg_alpha=variant.get("hg_alpha", 0.0))
        r = -y
        nrm = float(r.norm())
        if prev is not None:
            rates.append(round(nrm / prev, 3))
        prev = nrm
        s.vcycle(r, c)
        x += c
    s.close()
    return rates


def bench_variants(tng, ctx):
    """Viscous-block variants in the solve (Sec. 4): the one-point operator, hourglass
    control (eq:hgstab, alpha 0.1) and the two-radial-point rule, each on every level
    of the multigrid.  Stand-alone V-cycle rates on (32,32) and (64,64), then Stokes
    solves to 1e-8 on (64,64) and (128,128) (FGMRES iterations and wall time), also
    with free slip on the outer sphere and on both spheres."""
    import torch
    variants = (("one-point", {}), ("hourglass 0.1", {"hg_alpha": 0.1}),
                ("two-point", {"op_flags": tng.OP_TWOPOINT}))
    laws = (("const", 0.0, 0.0), ("c1e3+depth", math.log(1e3), math.log(10.0)), ("c1e6", math.log(1e6), 0.0))
    out = {"workload": "stand-alone V-cycle on A_D and Stokes solves to 1e-8 with the viscous-block variants",
           "vcycle": [], "solve": []}
    for mt in (32, 64):
        mesh = tng.Mesh(ctx, mt, mt, levels=int(math.log2(mt)))
        T64 = shell_fields(tng, ctx, mesh, seed=1, lmax=8)
        for law, E, F in (laws[0], laws[2]):
            eta = torch.empty(mesh.wedge_shape(0), device="cuda", dtype=torch.float64)
            tng.eta_from_temperature(ctx, mesh, 0, T64, E, F, eta)
            for name, v in variants:
                out["vcycle"].append({"shell": [mt, mt], "law": law, "variant": name,
                                      "rates": vcycle_rates(tng, ctx, mesh, eta, **v)})
                log(f"[variants] {out['vcycle'][-1]}")
        mesh.close()
    # solves: the variants above, then free-slip spheres (the buoyancy's normal part removed
    # there) and the one-point operator with a longer restart (FGMRES(23))
    fs_o, fs_b = tng.OP_FREESLIP_OUTER, tng.OP_FREESLIP_INNER | tng.OP_FREESLIP_OUTER
    solves = [(name, v, 0) for name, v in variants] + [
        ("restart 23", {"restart": 23}, 0),
        ("free slip outer", {"op_flags": fs_o}, fs_o),
        ("free slip outer, restart 23", {"op_flags": fs_o, "restart": 23}, fs_o),
        ("free slip both", {"op_flags": fs_b}, fs_b),
        ("free slip both, restart 23", {"op_flags": fs_b, "restart": 23}, fs_b)]
    for mt in (64, 128):
        mesh = tng.Mesh(ctx, mt, mt, levels=int(math.log2(mt)))
        T64 = shell_fields(tng, ctx, mesh, seed=1, lmax=8)
        for law, E, F in laws[1:]:
            eta = torch.empty(mesh.wedge_shape(0), device="cuda", dtype=torch.float64)
            tng.eta_from_temperature(ctx, mesh, 0, T64, E, F, eta)
            f = torch.empty((3,) + mesh.shape(0), device="cuda", dtype=torch.float64)
            u = torch.empty_like(f)
            p = torch.empty(mesh.shape(1), device="cuda", dtype=torch.float64)
            for name, v, bits in solves:
                tng.rhs_buoyancy(ctx, mesh, 0, T64, 1e5, f, bc_flags=bits)
                for mixed in (0, 1):
                    sv = tng.StokesSolver(ctx, mesh, mixed=mixed, rtol=1e-8, max_iters=1200, max_outer=40, **v)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    info = sv.solve(f, None, u, p, eta=eta, raise_on_fail=False)
                    torch.cuda.synchronize()
                    wall = time.perf_counter() - t0
                    sv.close()
                    out["solve"].append({"shell": [mt, mt], "law": law, "variant": name,
                                         "mode": "mixed" if mixed else "fp64", "its": info["inner_its"],
                                         "fp64_its": info["fp64_its"],
                                         "refinements": info["outer_its"], "rel_res": info["rel_res"],
                                         "seconds": round(wall, 3), "rc": info["rc"]})
                    log(f"[variants] {out['solve'][-1]}")
        mesh.close()
    return out


def serving_fields(tng, nreq):
    """Seeded requests over (16,16), (32,32), (64,64) shells and their device buffers."""
    import torch
    import synthetic
    levels = [(16, 16), (32, 32), (64, 64)]
    reqs = synthetic.serving_requests(nreq, levels)
    fields = []
    meshes = [tng.Mesh(None, mt, nr, levels=1) for mt, nr in levels]
    coords = [m.coords(0) for m in meshes]
    bases = [synthetic.harmonic_basis(xyz.reshape(-1, 3), 1, 16) for xyz, _ in coords]
    for i, rq in enumerate(reqs):
        mesh = meshes[rq["level"]]
        xyz, r = coords[rq["level"]]
        T = synthetic.temperature(xyz.reshape(-1, 3), r, seed=rq["seed"], lmin=1, lmax=16,
                                  basis=bases[rq["level"]])
        if (i + 1) % 32 == 0:
            log(f"[bench] serving fields: {i + 1} of {len(reqs)}")
        Tt = torch.tensor(T.reshape(mesh.shape(0)), device="cuda")
        u = torch.empty((3,) + mesh.shape(0), device="cuda", dtype=torch.float64)
        mt, nr = levels[rq["level"]]
        p = torch.empty((10, mt // 2 + 1, mt // 2 + 1, nr // 2 + 1), device="cuda", dtype=torch.float64)
        fields.append((Tt, u, p))
    return levels, reqs, fields


def serving_run(srv, reqs, fields, arrivals, tag):
    """Submits request i at arrivals[i] seconds (all at once if None); returns the
    per-request latencies (arrival -> result on the device), successes and wall time."""
    import numpy as np
    t0 = time.perf_counter()
    tk = []
    for i, rq in enumerate(reqs):
        if arrivals is not None:
            while time.perf_counter() - t0 < arrivals[i]:
                time.sleep(2e-4)
        tk.append(srv.submit(rq["level"], fields[i][0], rq["log10_contrast"], 1e5, fields[i][1], fields[i][2]))
        if (i + 1) % 64 == 0:
            log(f"[bench] serving {tag}: {i + 1} submitted")
    srv.wait(0)
    total = time.perf_counter() - t0
    lat = np.array([srv.poll(t)["latency"] for t in tk])
    ok = int(sum(srv.poll(t)["rc"] == 0 for t in tk))
    return lat, ok, total


def bench_serving(tng, ctx, nreq, rate_factor, budget):
    """Poisson-arrival request stream over (16,16), (32,32), (64,64) shells."""
    import numpy as np
    import synthetic
    levels, reqs, fields = serving_fields(tng, nreq)
    srv = tng.Server(ctx, levels, budget_bytes=budget, max_slots=16, mixed=1, rtol=1e-8)
    _, _, tsat = serving_run(srv, reqs, fields, None, "saturated")   # everything submitted at once
    mu = nreq / tsat
    lam = rate_factor * mu
    lat, ok, total = serving_run(srv, reqs, fields, synthetic.poisson_arrivals(nreq, lam, seed=7), "poisson")
    st = srv.stats()
    srv.close()
    return {"requests": nreq, "ok": ok, "saturated_solves_per_s": round(mu, 2),
            "lambda_per_s": round(lam, 2), "solves_per_s": round(nreq / total, 2),
            "p50_latency_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
            "p99_latency_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
            "slots": st["slots"], "budget_bytes": budget, "bytes_in_use": st["bytes_in_use"],
            "levels": levels}


def bench_serving_sweep(tng, ctx, nreq=256, factors=(0.25, 0.5, 0.75, 0.95), budget=200 * 10**9,
                        tight_budget=2 << 30):
    """The serving stream at its saturated rate mu and at Poisson arrival rates
    lambda = f mu, each with p50/p99 latency and throughput, then the saturated
    stream again under a tight HBM budget."""
    import numpy as np
    import synthetic
    levels, reqs, fields = serving_fields(tng, nreq)
    srv = tng.Server(ctx, levels, budget_bytes=budget, max_slots=16, mixed=1, rtol=1e-8)
    lat, ok, tsat = serving_run(srv, reqs, fields, None, "saturated")
    mu = nreq / tsat
    rows = [{"lambda_factor": None, "lambda_per_s": None, "ok": ok, "solves_per_s": round(mu, 3),
             "p50_latency_ms": round(float(np.percentile(lat, 50)) * 1e3, 1),
             "p99_latency_ms": round(float(np.percentile(lat, 99)) * 1e3, 1)}]
    log(f"[bench] serving saturated: {rows[-1]}")
    for li, f in enumerate(factors):
        lam = f * mu
        lat, ok, total = serving_run(srv, reqs, fields, synthetic.poisson_arrivals(nreq, lam, seed=7 + li),
                                     f"lambda={f}mu")
        rows.append({"lambda_factor": f, "lambda_per_s": round(lam, 3), "ok": ok,
                     "solves_per_s": round(nreq / total, 3),
                     "p50_latency_ms": round(float(np.percentile(lat, 50)) * 1e3, 1),
                     "p99_latency_ms": round(float(np.percentile(lat, 99)) * 1e3, 1)})
        log(f"[bench] serving {rows[-1]}")
    st = srv.stats()
    srv.close()
    tight = tng.Server(ctx, levels, budget_bytes=tight_budget, max_slots=16, mixed=1, rtol=1e-8)
    lat, ok, total = serving_run(tight, reqs, fields, None, "tight budget")
    tst = tight.stats()
    tight.close()
    return {"workload": f"{nreq} Stokes solve requests over the (16,16), (32,32), (64,64) shells, contrast "
                        "10^U(2,6), T with l = 1..16, mixed precision to 1e-8",
            "budget_bytes": budget, "slots_used": st["slots"], "runs": rows,
            "tight_budget": {"budget_bytes": tight_budget, "ok": ok, "solves_per_s": round(nreq / total, 3),
                             "p50_latency_ms": round(float(np.percentile(lat, 50)) * 1e3, 1),
                             "p99_latency_ms": round(float(np.percentile(lat, 99)) * 1e3, 1),
                             "slots_live_at_end": tst["slots"], "bytes_in_use_at_end": tst["bytes_in_use"]}}


def cpu_baseline(sizes=((16, 16), (32, 32)), reps=10, solve_sizes=(8,)):
    """The FP64 oracle (assembled K_D, scipy CSR SpMV) on bounded sample shells; the value
    is that of the largest one (the SpMV is memory-bound, so its GDoF/s barely depend on size)."""
    import numpy as np
    import synthetic
    from oracle.mesh import ShellMesh
    from oracle.stokes import StokesOracle, eta_from_temperature
    parts, value = [], None
    for mt, nr in sizes:
        om = ShellMesh(mt, nr)
        T = synthetic.temperature(om.s, om.r, seed=1, lmin=1, lmax=8, amp=0.01).ravel()
        eta = eta_from_temperature(om, T, math.log(1e3), math.log(10.0))
        t0 = time.perf_counter()
        orc = StokesOracle(mt, nr, eta, hierarchy=om.h)
        t_asm = time.perf_counter() - t0
        x = np.random.default_rng(2).uniform(-1, 1, orc.K.shape[0])
        for _ in range(2):
            orc.K @ x
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            orc.K @ x
            ts.append(time.perf_counter() - t0)
        t = float(np.median(ts))
        ndof = orc.K.shape[0]
        value = ndof / t / 1e9
        parts.append(f"({mt},{nr}) shell {ndof} u+p DoFs, nnz {orc.K.nnz}: {t * 1e3:.2f} ms per apply "
                     f"({value:.4f} GDoF/s), assembly {t_asm:.1f} s")
        del orc
    solves = [cpu_solve(mt) for mt in solve_sizes]
    return {"value": round(value, 5), "unit": "GDoF/s", "cores": 1, "kind": "oracle",
            "sample": (f"assembled FP64 K_D, scipy CSR SpMV (single thread), median of {reps} after 2 warm-ups: "
                       + "; ".join(parts) + f"; value from the largest; host {host_cpu()}, nproc {os.cpu_count()}"),
            "solves": solves}


def host_cpu():
    cpu = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as fh:
            cpu = next(l.split(":", 1)[1].strip() for l in fh if l.startswith("model name"))
    except Exception:
        pass
    return cpu


def cpu_solve(mt):
    """The oracle's exact discrete solve (A_D factorised, CG on the pressure Schur
    complement to 1e-13) of the contrast-1e6 workload on the (mt, mt) copy."""
    import synthetic
    from oracle.mesh import ShellMesh
    from oracle.saddle import SchurSolver
    from oracle.stokes import StokesOracle, buoyancy_rhs, eta_from_temperature
    om = ShellMesh(mt, mt)
    T = synthetic.temperature(om.s, om.r, seed=1, lmin=1, lmax=8, amp=0.01).ravel()
    eta = eta_from_temperature(om, T, math.log(1e6), 0.0)
    f = buoyancy_rhs(om, T, 1e5)
    f[om.boundary_nodes()] = 0.0
    t0 = time.perf_counter()
    orc = StokesOracle(mt, mt, eta, hierarchy=om.h)
    sol = SchurSolver(orc, eta)
    t_fac = time.perf_counter() - t0
    _, _, info = sol.solve(f)
    t = time.perf_counter() - t0
    return {"shell": [mt, mt], "dofs": orc.K.shape[0], "seconds": round(t, 2), "assembly_and_factor_s": round(t_fac, 2),
            "schur_cg_its": info["cg_its"], "rel_res": info["rel_res"], "cores": 1}


def run_solves(tng, ctx, mesh, T64):
    """The FP64 solve of the headline field, the contrast-1e6 field in FP64 and mixed
    precision (same field), and the contrast-1e6 solves on the (16,16) copy against
    the stored oracle solution."""
    import torch
    out = {}
    log("[bench] FP64 solve, contrast 1e3 x 10 (depth)")
    s1, _ = bench_solve(tng, ctx, mesh, T64, math.log(1e3), math.log(10.0), mixed=0)
    out["solve_fp64"] = {"solves_per_s": round(1.0 / s1["wall"], 4), "seconds": round(s1["wall"], 3),
                         "iterations": s1["inner_its"], "rel_res": s1["rel_res"], "rc": s1["rc"]}
    log(f"[bench] {out['solve_fp64']}")
    log("[bench] contrast 1e6: mixed vs FP64 on the same field")
    s64, (u64, p64) = bench_solve(tng, ctx, mesh, T64, math.log(1e6), 0.0, mixed=0)
    s32, (u32, p32) = bench_solve(tng, ctx, mesh, T64, math.log(1e6), 0.0, mixed=1)
    du = float(torch.linalg.vector_norm(u32 - u64) / torch.linalg.vector_norm(u64))
    dp = float(torch.linalg.vector_norm(p32 - p64) / torch.linalg.vector_norm(p64))
    del u64, p64, u32, p32
    torch.cuda.empty_cache()
    log("[bench] contrast 1e6 on the (16,16) copy vs the stored oracle solution")
    g64, g32 = golden16_errors(tng, ctx, 0), golden16_errors(tng, ctx, 1)
    out["solve_contrast_1e6"] = {
        "fp64": {"solves_per_s": round(1.0 / s64["wall"], 4), "iterations": s64["inner_its"],
                 "rel_res": s64["rel_res"], "rc": s64["rc"]},
        "mixed": {"solves_per_s": round(1.0 / s32["wall"], 4), "inner_iterations": s32["inner_its"],
                  "refinement_steps": s32["outer_its"], "rel_res": s32["rel_res"], "rc": s32["rc"]},
        "mixed_over_fp64": round(s64["wall"] / s32["wall"], 3),
        "mixed_vs_fp64_rel_err": {"u": du, "p": dp},
        "vs_oracle_on_16x16_copy": {"fp64": g64, "mixed": g32},
        "mixed_1e6_over_fp64_solve_at_contrast_1e3": round(s1["wall"] / s32["wall"], 3)}
    log(f"[bench] {out['solve_contrast_1e6']}")
    # the same solves with a longer Krylov basis, FGMRES(23) (the fields above use the
    # paper's FGMRES(10)): 23 basis vectors of the (128,128) problem hold 12 GB in FP64
    log("[bench] the same solves with FGMRES(23)")
    r1, _ = bench_solve(tng, ctx, mesh, T64, math.log(1e3), math.log(10.0), mixed=0, restart=23)
    r64, _ = bench_solve(tng, ctx, mesh, T64, math.log(1e6), 0.0, mixed=0, restart=23)
    r32, _ = bench_solve(tng, ctx, mesh, T64, math.log(1e6), 0.0, mixed=1, restart=23)
    out["solve_fgmres23"] = {
        "fp64_contrast_1e3": {"solves_per_s": round(1.0 / r1["wall"], 4), "iterations": r1["inner_its"],
                              "rel_res": r1["rel_res"], "rc": r1["rc"]},
        "fp64_contrast_1e6": {"solves_per_s": round(1.0 / r64["wall"], 4), "iterations": r64["inner_its"],
                              "rel_res": r64["rel_res"], "rc": r64["rc"]},
        "mixed_contrast_1e6": {"solves_per_s": round(1.0 / r32["wall"], 4), "inner_iterations": r32["inner_its"],
                               "refinement_steps": r32["outer_its"], "rel_res": r32["rel_res"], "rc": r32["rc"]},
        "mixed_over_fp64_contrast_1e6": round(r64["wall"] / r32["wall"], 3)}
    log(f"[bench] {out['solve_fgmres23']}")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    # a few launches leave the GPU below its sustained clock: 100 (about 40 ms of FP32
    # applies) bring it there
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--mt", type=int, default=128)
    ap.add_argument("--nr", type=int, default=128)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solve", action="store_true", help="apply only (profiling runs)")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=48)
    ap.add_argument("--serving-rate", type=float, default=0.75, help="arrival rate / saturated rate")
    ap.add_argument("--serving-budget-gb", type=float, default=200.0, help="HBM budget in GB (1e9 bytes)")
    ap.add_argument("--cpu-baseline-full", action="store_true",
                    help="instead: the CPU oracle on larger shells (SpMV up to (64,64), exact solves at (8,8) "
                         "and (16,16)); CPU only, several minutes; one JSON report line")
    ap.add_argument("--serving-sweep", action="store_true",
                    help="instead: 256-request serving stream at the saturated rate and four Poisson "
                         "rates, plus a tight 2 GiB budget; one JSON report line")
    ap.add_argument("--coupled", action="store_true",
                    help="instead: coupled Stokes-energy steps on the (--mt, --nr) shell (default (256,256), "
                         "--steps steps), one JSON report line")
    ap.add_argument("--energy-apply", action="store_true",
                    help="instead: the SUPG energy apply alone on the (--mt, --nr) shell (default (256,256)), "
                         "FP64 and FP32; one JSON report line")
    ap.add_argument("--variants", action="store_true",
                    help="instead: stand-alone V-cycle rates and Stokes solve iterations with the one-point, "
                         "hourglass-controlled and two-radial-point viscous blocks; one JSON report line")
    ap.add_argument("--profile-solve", choices=["fp64", "mixed"],
                    help="instead: one Stokes solve of the contrast-1e6 field on the (--mt, --nr) shell, for "
                         "kernel traces; one JSON report line")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: there is no multi-GPU path (the shell would shard by "
              "lateral diamond blocks, with one neighbour exchange of diamond-edge partial sums per "
              "apply).",
              file=sys.stderr)
        sys.exit(2)
    if args.cpu_baseline_full:
        print(json.dumps(cpu_baseline(sizes=((16, 16), (32, 32), (64, 64)), solve_sizes=(8, 16))), flush=True)
        return
    import torch
    import paper_2609_21633_amd as tng
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    ctx = tng.Context(0)
    if args.serving_sweep:
        print(json.dumps(bench_serving_sweep(tng, ctx)), flush=True)
        return
    if args.variants:
        print(json.dumps(bench_variants(tng, ctx)), flush=True)
        return
    if args.profile_solve:
        mesh = tng.Mesh(ctx, args.mt, args.nr, levels=int(math.log2(args.mt)))
        T64 = shell_fields(tng, ctx, mesh, seed=1, lmax=8)
        s, _ = bench_solve(tng, ctx, mesh, T64, math.log(1e6), 0.0, mixed=1 if args.profile_solve == "mixed" else 0,
                           reps=1)
        print(json.dumps({"workload": f"Stokes solve to 1e-8, contrast 1e6, ({args.mt},{args.nr}) shell",
                          "mode": args.profile_solve, "seconds": round(s["wall"], 3), "inner_its": s["inner_its"],
                          "outer_its": s["outer_its"], "rel_res": s["rel_res"], "rc": s["rc"]}), flush=True)
        return
    if args.energy_apply:
        em = args.mt if "--mt" in sys.argv else 256
        en = args.nr if "--nr" in sys.argv else 256
        es_ = args.steps if "--steps" in sys.argv else 50
        ew = args.warmup if "--warmup" in sys.argv else 20
        print(json.dumps(bench_energy_apply(tng, ctx, em, en, es_, ew)), flush=True)
        return
    if args.coupled:
        cm = args.mt if "--mt" in sys.argv else 256
        cn = args.nr if "--nr" in sys.argv else 256
        cs = args.steps if "--steps" in sys.argv else 10
        print(json.dumps(bench_coupled(tng, ctx, cm, cn, cs)), flush=True)
        return
    mt, nr = args.mt, args.nr
    nu, npr = unique_dofs(mt, nr)
    levels = int(math.log2(mt))                   # down to (2, 2)
    mesh = tng.Mesh(ctx, mt, nr, levels=levels)
    T64 = shell_fields(tng, ctx, mesh, seed=1, lmax=8)
    extra = {}
    if not args.no_solve:
        extra.update(run_solves(tng, ctx, mesh, T64))
    if not args.no_serving:
        log(f"[bench] serving: {args.serving_requests} requests at {args.serving_rate} x saturated rate")
        extra["serving"] = bench_serving(tng, ctx, args.serving_requests, args.serving_rate,
                                         int(args.serving_budget_gb * 1e9))
        log(f"[bench] {extra['serving']}")
    # the timed applies come after the solves and the serving run, so that they run at the
    # GPU's sustained clock (as inside a solve) whatever the number of warm-up steps
    res = {}
    for name, dtype, es in (("f64", torch.float64, 8), ("f32", torch.float32, 4)):
        log(f"[bench] {name} apply on ({mt},{nr})")
        wall, kms = bench_apply(tng, ctx, mesh, T64, dtype, args.steps, args.warmup)
        ab = algorithmic_bytes(mesh, es)
        res[name] = {"ms": wall * 1e3, "kernel_ms": kms, "gdofs": (nu + npr) / wall / 1e9, "alg_bytes": ab,
                     "kernel_gbs": ab / (kms * 1e-3) / 1e9}
        log(f"[bench] {name}: {wall * 1e3:.3f} ms/apply (kernel {kms:.3f} ms), {res[name]['gdofs']:.1f} GDoF/s, "
            f"{res[name]['kernel_gbs']:.0f} GB/s algorithmic")
        torch.cuda.empty_cache()
    roof = bench_copy_roof(tng, ctx)
    log(f"[bench] practical roof (stream copy): {roof}")
    head = res["f32"]
    # measured HBM traffic (scaled rocprofv3 counters) only for the (128,128) shell they were taken on
    t32 = counter_traffic("f32_traffic_bytes_per_launch") if (mt, nr) == (128, 128) else None
    t64 = counter_traffic("f64_traffic_bytes_per_launch") if (mt, nr) == (128, 128) else None
    out = {
        "metric": "GDoF/s Stokes apply FP32 vs FP64 at 1e-8 solve tol; solves/s, p50/p99 latency",
        "value": round(head["gdofs"], 3),
        "unit": "GDoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (f"Stokes K apply on the shell with velocity ({mt},{nr}) / pressure "
                                f"({mt // 2},{nr // 2}), eta = exp(-ln(1e3) T + ln(10)(1-r)), "
                                "T = conduction + spherical harmonics l=1..8"),
                   "u_dofs": nu, "p_dofs": npr},
        "roofline": {"bound": "hbm", "achieved": round(head["kernel_gbs"], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(head["kernel_gbs"] / HBM_PEAK_GBS, 4),
                     "traffic": None if t32 is None else round(t32 / (head["kernel_ms"] * 1e6), 1),
                     "traffic_bytes_per_launch": t32,
                     "kernel": "stokes_band_kernel<float,RS=1,CPL=2,A,BT,B,WG=4> (FP32 full operator)",
                     "alg_bytes_per_launch": head["alg_bytes"], "kernel_ms": round(head["kernel_ms"], 4),
                     "practical_roof": roof,
                     "frac_of_practical_roof": round(head["kernel_gbs"] / roof["gbs"], 4)},
        "f64_apply": {"gdofs": round(res["f64"]["gdofs"], 3), "ms": round(res["f64"]["ms"], 4),
                      "kernel_gbs": round(res["f64"]["kernel_gbs"], 1),
                      "traffic_gbs": None if t64 is None else round(t64 / (res["f64"]["kernel_ms"] * 1e6), 1),
                      "kernel_ms": round(res["f64"]["kernel_ms"], 4)},
    }
    out.update(extra)
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
