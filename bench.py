#!/usr/bin/env python3
"""Benchmark of the matrix-free wedge Stokes hot path on one MI355X.

Workload: the spherical shell with velocity mesh (mt, nr) = (128, 128)
(163,842 lateral nodes x 129 layers, 63.4 M velocity DoFs) and W1 pressure on
(64, 64) (2.66 M DoFs); temperature = conductive profile + seeded spherical
harmonics l = 1..8 of amplitude 0.01; viscosity eta = exp(-ln(1e3) T +
ln(10) (1 - r)) per wedge.  A step is one full Stokes operator apply
y = K_D [u; p] (A, B^T, B, Dirichlet rows, diamond-interface sum).

Prints one JSON line (see the design doc for the fields).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def setup(tng, ctx, mt, nr, dtype):
    import numpy as np
    import torch
    import synthetic
    mesh = tng.Mesh(ctx, mt, nr, levels=2)
    xyz, r = mesh.coords(0)
    T = synthetic.temperature(xyz.reshape(-1, 3), r, seed=1, lmin=1, lmax=8, amp=0.01)
    dev = torch.device("cuda", 0)
    T_t = torch.tensor(T.reshape(mesh.shape(0)), device=dev, dtype=dtype)
    eta = torch.empty(mesh.wedge_shape(0), device=dev, dtype=dtype)
    tng.eta_from_temperature(ctx, mesh, 0, T_t, math.log(1e3), math.log(10.0), eta)
    g = torch.Generator(device="cpu").manual_seed(2)
    u = (torch.rand((3,) + mesh.shape(0), generator=g, dtype=torch.float64) * 2 - 1).to(dev, dtype)
    p = (torch.rand(mesh.shape(1), generator=g, dtype=torch.float64) * 2 - 1).to(dev, dtype)
    tng.interface_sum(ctx, mesh, 0, [u[0], u[1], u[2]], mode=1)
    tng.interface_sum(ctx, mesh, 1, [p], mode=1)
    yu = torch.empty_like(u)
    yp = torch.empty_like(p)
    torch.cuda.synchronize()
    return mesh, eta, u, p, yu, yp


def unique_dofs(mt, nr):
    nu = 3 * (10 * mt * mt + 2) * (nr + 1)
    npr = (10 * (mt // 2) ** 2 + 2) * (nr // 2 + 1)
    return nu, npr


def algorithmic_bytes(mesh, esize):
    """Minimal traffic of one K apply: read u, write y_u (3 node fields each),
    read the two wedge viscosities per cell, read p and write y_p."""
    c0, c1 = mesh.counts(0), mesh.counts(1)
    return esize * (6 * c0["node_slots"] + 2 * c0["cells"] + 2 * c1["node_slots"])


def time_apply(tng, ctx, mesh, eta, u, p, yu, yp, steps, warmup):
    import torch
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
    return wall, kms / max(nl, 1)


def cpu_baseline(mt=16, nr=16, reps=10):
    """The FP64 oracle (assembled K, scipy CSR SpMV) on a bounded sample shell."""
    import numpy as np
    import synthetic
    from oracle.mesh import ShellMesh
    from oracle.stokes import StokesOracle, eta_from_temperature
    om = ShellMesh(mt, nr)
    T = synthetic.temperature(om.s, om.r, seed=1, lmin=1, lmax=8, amp=0.01).ravel()
    eta = eta_from_temperature(om, T, math.log(1e3), math.log(10.0))
    t0 = time.perf_counter()
    orc = StokesOracle(mt, nr, eta, hierarchy=om.h)
    t_asm = time.perf_counter() - t0
    rng = np.random.default_rng(2)
    x = rng.uniform(-1, 1, orc.K.shape[0])
    for _ in range(2):
        orc.K @ x
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        orc.K @ x
        ts.append(time.perf_counter() - t0)
    t = float(np.median(ts))
    ndof = orc.K.shape[0]
    return {"value": ndof / t / 1e9, "unit": "GDoF/s", "cores": 1, "kind": "oracle",
            "sample": (f"assembled FP64 K_D of the ({mt},{nr}) shell ({ndof} u+p DoFs, "
                       f"nnz {orc.K.nnz}), scipy CSR SpMV, median of {reps}; assembly took "
                       f"{t_asm:.1f} s, SpMV {t * 1e3:.2f} ms; host {platform.processor() or platform.machine()}, "
                       f"nproc {os.cpu_count()}")}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mt", type=int, default=128)
    ap.add_argument("--nr", type=int, default=128)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(the shell would shard by lateral diamond blocks with one neighbour "
              "exchange per apply; see DESIGN.md).", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2609_21633_amd as tng
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    ctx = tng.Context(0)
    mt, nr = args.mt, args.nr
    nu, npr = unique_dofs(mt, nr)
    res = {}
    for name, dtype, es in (("f64", torch.float64, 8), ("f32", torch.float32, 4)):
        log(f"[bench] setting up {name} apply on ({mt},{nr})")
        mesh, eta, u, p, yu, yp = setup(tng, ctx, mt, nr, dtype)
        wall, kms = time_apply(tng, ctx, mesh, eta, u, p, yu, yp, args.steps, args.warmup)
        ab = algorithmic_bytes(mesh, es)
        res[name] = {"ms": wall * 1e3, "kernel_ms": kms, "gdofs": (nu + npr) / wall / 1e9,
                     "alg_bytes": ab, "kernel_gbs": ab / (kms * 1e-3) / 1e9}
        log(f"[bench] {name}: {wall * 1e3:.3f} ms/apply, kernel {kms:.3f} ms, "
            f"{res[name]['gdofs']:.1f} GDoF/s, {res[name]['kernel_gbs']:.0f} GB/s algorithmic")
        del mesh, eta, u, p, yu, yp
        torch.cuda.empty_cache()
    head = res["f32"]
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
        "config": {"workload": f"Stokes K apply, shell vel ({mt},{nr}) / p ({mt // 2},{nr // 2}), "
                               "eta = exp(-ln(1e3) T + ln(10)(1-r)), T = conduction + SH l=1..8",
                   "u_dofs": nu, "p_dofs": npr},
        "roofline": {"bound": "hbm", "achieved": round(head["kernel_gbs"], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(head["kernel_gbs"] / HBM_PEAK_GBS, 4),
                     "traffic": None},
        "f64_apply": {"gdofs": round(res["f64"]["gdofs"], 3), "ms": round(res["f64"]["ms"], 4),
                      "kernel_gbs": round(res["f64"]["kernel_gbs"], 1)},
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
