"""Build libtng.so (HIP for gfx950 + C++ host code) in-tree with hipcc.

Every source is compiled to its own object in parallel (``_build/``), then the
objects are linked into ``libtng.so``.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libtng.so")
SOURCES = ["capi.cpp", "mesh.cpp", "stokes_apply.hip", "interface.hip", "fields.hip", "mg_kernels.hip", "solver.cpp",
           "energy.hip", "energy.cpp", "server.cpp", "noalloc.hip", "bandwidth.hip", "mmoc.hip",
           "energy_stream.hip"]
ARCH = "gfx950"


def _hipcc() -> str:
    return os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")


def compile_flags() -> list[str]:
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
            # the sign of a zero carries no meaning here; this lets 0 + x fold to x,
            # so accumulators start without a zero fill
            "-munsafe-fp-atomics", "-fno-signed-zeros", "-pthread",
            # no packed FP32 instructions anywhere in device code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def hipcc_command(out: str = LIB) -> list[str]:
    """One-command form of the build (all sources, one hipcc call)."""
    return [_hipcc()] + compile_flags() + ["-shared", "-o", out] + [os.path.join(CSRC, s) for s in SOURCES]


def _compile(src: str) -> tuple[str, int, str]:
    obj = os.path.join(OBJ, src + ".o")
    cmd = [_hipcc()] + compile_flags() + ["-c", "-o", obj, os.path.join(CSRC, src)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    return obj, r.returncode, " ".join(cmd) + "\n" + r.stdout + r.stderr


def build(verbose: bool = True) -> str:
    os.makedirs(OBJ, exist_ok=True)
    jobs = max(1, min(len(SOURCES), os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(_compile, SOURCES))
    failed = [log for _, rc, log in results if rc != 0]
    if failed:
        sys.stderr.write("\n".join(failed))
        raise RuntimeError("hipcc failed")
    tmp = LIB + ".tmp"
    link = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread", "-o", tmp] + [o for o, _, _ in results]
    if verbose:
        print(" ".join(link), flush=True)
    r = subprocess.run(link, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
