"""ctypes binding of include/tng.h: argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("TNG_LIB", os.path.join(HERE, "libtng.so"))

OP_A, OP_BT, OP_B, OP_DIRICHLET = 1, 2, 4, 8
OP_FREESLIP_INNER, OP_FREESLIP_OUTER, OP_TALA, OP_TWOPOINT = 16, 32, 64, 128
F64, F32 = 0, 1

_lib = None
_vp = C.c_void_p


class TngError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"tng error {code}: {msg}")
        self.code = code


def lib():
    """Load libtng.so (once).  Raises if it was not built: there is no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing; build it with __graft_entry__.build()")
    L = C.CDLL(LIB_PATH)
    L.tng_last_error.restype = C.c_char_p
    sig = {
        "tng_ctx_create": [C.c_int, _vp, C.POINTER(_vp)],
        "tng_ctx_set_stream": [_vp, _vp],
        "tng_ctx_destroy": [_vp],
        "tng_ctx_set_apply_bands": [_vp, C.c_int],
        "tng_mesh_create": [_vp, C.c_int, C.c_int, C.c_double, C.c_double, C.c_int, C.POINTER(_vp)],
        "tng_mesh_counts": [_vp, C.c_int, C.POINTER(C.c_longlong)],
        "tng_mesh_coords": [_vp, C.c_int, _vp, _vp],
        "tng_mesh_dup_groups": [_vp, C.c_int, _vp],
        "tng_mesh_destroy": [_vp],
        "tng_mesh_set_density": [_vp, _vp],
        "tng_rhs_buoyancy_tala": [_vp, _vp, C.c_int, C.c_int, _vp, C.c_double, _vp, _vp, C.POINTER(_vp)],
        "tng_stokes_apply": [_vp, _vp, C.c_int, C.c_int, C.c_uint, C.c_double, _vp, C.POINTER(_vp), _vp,
                             C.POINTER(_vp), _vp],
        "tng_interface_sum": [_vp, _vp, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(_vp)],
        "tng_stream_copy": [_vp, _vp, _vp, C.c_size_t],
        "tng_check_device_buffer": [_vp, _vp, C.c_size_t],
        "tng_stokes_apply_layout": [_vp, _vp, C.c_int, C.c_int, C.c_uint, C.c_double, C.POINTER(C.c_int)],
        "tng_ctx_profile": [_vp, C.c_int],
        "tng_ctx_kernel_stats": [_vp, C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_longlong)],
        "tng_ctx_kernel_stats_at": [_vp, C.c_int, C.c_char_p, C.c_int, C.POINTER(C.c_double),
                                    C.POINTER(C.c_longlong)],
        "tng_eta_from_temperature": [_vp, _vp, C.c_int, C.c_int, _vp, C.c_double, C.c_double, _vp],
        "tng_eta_coarsen": [_vp, _vp, C.c_int, C.c_int, _vp, _vp],
        "tng_diag_A": [_vp, _vp, C.c_int, C.c_int, _vp, C.c_double, C.POINTER(_vp)],
        "tng_diag_A_twopoint": [_vp, _vp, C.c_int, C.c_int, _vp, C.POINTER(_vp)],
        "tng_pressure_mass": [_vp, _vp, C.c_int, C.c_int, _vp, _vp],
        "tng_smooth": [_vp, _vp, C.c_int, C.c_int, _vp, C.c_double, C.POINTER(_vp), C.POINTER(_vp), C.POINTER(_vp),
                       C.c_int, C.c_int, C.c_double, C.c_double],
        "tng_smooth_noalloc": [_vp, _vp, C.c_int, C.c_int, _vp, C.c_double, C.POINTER(_vp), C.POINTER(_vp),
                               C.POINTER(_vp), C.c_int, C.c_int, C.c_double, C.c_double],
        "tng_restrict": [_vp, _vp, C.c_int, C.c_int, C.POINTER(_vp), C.POINTER(_vp)],
        "tng_prolong": [_vp, _vp, C.c_int, C.c_int, C.POINTER(_vp), C.POINTER(_vp)],
        "tng_solver_opts_default": [_vp],
        "tng_stokes_solver_create": [_vp, _vp, _vp, C.POINTER(_vp)],
        "tng_stokes_solver_destroy": [_vp],
        "tng_stokes_solver_setup": [_vp, _vp],
        "tng_stokes_solve": [_vp, _vp, C.POINTER(_vp), _vp, C.POINTER(_vp), _vp, _vp],
        "tng_stokes_solver_vcycle": [_vp, C.POINTER(_vp), C.POINTER(_vp)],
        "tng_rhs_buoyancy": [_vp, _vp, C.c_int, C.c_int, _vp, C.c_double, C.POINTER(_vp)],
        "tng_rhs_buoyancy_bc": [_vp, _vp, C.c_int, C.c_int, C.c_uint, _vp, C.c_double, C.POINTER(_vp)],
        "tng_energy_apply": [_vp, _vp, C.c_int, C.c_int, C.POINTER(_vp), C.c_double, _vp, _vp],
        "tng_energy_step": [_vp, _vp, _vp, _vp, C.POINTER(_vp), _vp, _vp],
        "tng_mmoc_advect": [_vp, _vp, C.c_int, C.POINTER(_vp), C.c_double, _vp, _vp],
        "tng_server_create": [_vp, C.POINTER(C.c_int), C.c_int, C.c_size_t, C.c_int, _vp, C.POINTER(_vp)],
        "tng_server_submit": [_vp, C.c_int, _vp, C.c_double, C.c_double, C.POINTER(_vp), _vp,
                              C.POINTER(C.c_longlong)],
        "tng_server_poll": [_vp, C.c_longlong, C.POINTER(C.c_int), _vp, C.POINTER(C.c_double),
                            C.POINTER(C.c_double)],
        "tng_server_wait": [_vp, C.c_longlong],
        "tng_server_stats": [_vp, C.POINTER(C.c_longlong), C.POINTER(C.c_int), C.POINTER(C.c_int),
                             C.POINTER(C.c_int)],
        "tng_server_destroy": [_vp],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_int
    _lib = L
    return L


def check(rc: int):
    if rc != 0:
        raise TngError(rc, lib().tng_last_error().decode())


def _ptr(t):
    return None if t is None else _vp(t.data_ptr())


def _ptr3(ts):
    if ts is None:
        return None
    arr = (_vp * 3)(*[t.data_ptr() for t in ts])
    return arr


def _prec(t):
    import torch
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError("fields must be float32 or float64")


def _chk(ctx, t, dtype, numel: int, name: str):
    """A field argument must be a contiguous tensor of `dtype` with `numel`
    values on the context's GPU (the library cannot see a torch tensor's device,
    dtype or size; a wrong one would be read as garbage or out of bounds)."""
    if t is None:
        return
    if not getattr(t, "is_cuda", False) or t.device.index != ctx.device:
        raise TypeError(f"{name} must be a tensor on cuda:{ctx.device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} has dtype {t.dtype}, the call uses {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} values, the mesh level needs {numel}")


def _chk3(ctx, ts, dtype, numel: int, name: str):
    if ts is None:
        return
    if len(ts) != 3:
        raise ValueError(f"{name} must hold three components")
    for c in range(3):
        _chk(ctx, ts[c], dtype, numel, f"{name}[{c}]")


def _counts(mesh, level: int) -> dict:
    cache = mesh.__dict__.setdefault("_counts", {})
    if level not in cache:
        cache[level] = mesh.counts(level)
    return cache[level]


def _nodes(mesh, level: int) -> int:
    return _counts(mesh, level)["node_slots"]


def _wedges(mesh, level: int) -> int:
    return _counts(mesh, level)["wedges"]


class Context:
    """HIP device + stream that every call enqueues on (torch's current stream by default)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = _vp()
        check(lib().tng_ctx_create(device, _vp(stream.cuda_stream), C.byref(h)))
        self.h = h

    def set_stream(self, stream):
        self.stream = stream
        check(lib().tng_ctx_set_stream(self.h, _vp(stream.cuda_stream)))

    def set_apply_bands(self, bands: int = 0):
        """Force the operator apply's band count (0: chosen per launch)."""
        check(lib().tng_ctx_set_apply_bands(self.h, int(bands)))

    def profile(self, enable: bool = True):
        """Record HIP events around the main kernel of every call (on this stream)."""
        check(lib().tng_ctx_profile(self.h, 1 if enable else 0))

    def kernel_stats(self, name: str):
        """(total milliseconds, launches) of a kernel since profiling was enabled."""
        ms, n = C.c_double(), C.c_longlong()
        check(lib().tng_ctx_kernel_stats(self.h, name.encode(), C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def kernel_stats_all(self) -> dict:
        """{full timer name: (total milliseconds, launches)} since profiling was enabled."""
        out = {}
        buf = C.create_string_buffer(256)
        ms, n = C.c_double(), C.c_longlong()
        i = 0
        while lib().tng_ctx_kernel_stats_at(self.h, i, buf, 256, C.byref(ms), C.byref(n)) == 0:
            out[buf.value.decode()] = (ms.value, n.value)
            i += 1
        return out

    def close(self):
        if getattr(self, "h", None):
            lib().tng_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mesh:
    """Shell mesh with `levels` levels; level l = (mt / 2^l, nr / 2^l)."""

    def __init__(self, ctx: Context | None, mt: int, nr: int, r_in: float = 0.55,
                 r_out: float = 1.0, levels: int = 2):
        """ctx=None builds the host-side description only (no device arrays)."""
        self.ctx, self.mt, self.nr, self.r_in, self.r_out, self.levels = ctx, mt, nr, r_in, r_out, levels
        h = _vp()
        check(lib().tng_mesh_create(None if ctx is None else ctx.h, mt, nr, r_in, r_out, levels,
                                    C.byref(h)))
        self.h = h

    def counts(self, level: int = 0) -> dict:
        out = (C.c_longlong * 8)()
        check(lib().tng_mesh_counts(self.h, level, out))
        keys = ("m", "n", "lat_slots", "lat_unique", "node_slots", "nodes_unique", "cells", "wedges")
        return dict(zip(keys, [int(v) for v in out]))

    def shape(self, level: int = 0):
        c = self.counts(level)
        return (10, c["m"] + 1, c["m"] + 1, c["n"] + 1)

    def wedge_shape(self, level: int = 0):
        c = self.counts(level)
        return (10, c["m"], c["m"], c["n"], 2)

    def coords(self, level: int = 0):
        import numpy as np
        c = self.counts(level)
        xyz = np.empty((10, c["m"] + 1, c["m"] + 1, 3))
        r = np.empty(c["n"] + 1)
        check(lib().tng_mesh_coords(self.h, level, _vp(xyz.ctypes.data), _vp(r.ctypes.data)))
        return xyz, r

    def unique_ids(self, level: int = 0):
        import numpy as np
        c = self.counts(level)
        uid = np.empty((10, c["m"] + 1, c["m"] + 1), dtype=np.int32)
        check(lib().tng_mesh_dup_groups(self.h, level, _vp(uid.ctypes.data)))
        return uid

    def set_density(self, rho_nodes):
        """TALA reference density at the nr + 1 radial node layers of the finest level."""
        import numpy as np
        r = np.ascontiguousarray(rho_nodes, dtype=np.float64)
        if r.shape != (self.nr + 1,):
            raise ValueError("rho_nodes must hold nr + 1 values")
        check(lib().tng_mesh_set_density(self.h, _vp(r.ctypes.data)))

    def close(self):
        if getattr(self, "h", None):
            lib().tng_mesh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def stokes_apply(ctx: Context, mesh: Mesh, level: int, flags: int, eta, u, p, y_u, y_p,
                 hg_alpha: float = 0.0):
    """y = K(eta) [u; p] on `level` (blocks selected by flags).  u, y_u: 3 node fields
    (a [3, ...] tensor or a list); p, y_p: pressure fields on level + 1; any of them
    may be None when the selected blocks do not use it.  hg_alpha > 0 adds hourglass
    control to the viscous block."""
    ref = next(t for t in (u[0] if u is not None else None, y_u[0] if y_u is not None else None,
                           p, y_p) if t is not None)
    dt = ref.dtype
    nu = _nodes(mesh, level)
    _chk(ctx, eta, dt, _wedges(mesh, level), "eta")
    _chk3(ctx, u, dt, nu, "u")
    _chk3(ctx, y_u, dt, nu, "y_u")
    if p is not None or y_p is not None:
        np_ = _nodes(mesh, level + 1)
        _chk(ctx, p, dt, np_, "p")
        _chk(ctx, y_p, dt, np_, "y_p")
    check(lib().tng_stokes_apply(ctx.h, mesh.h, level, _prec(ref), flags, float(hg_alpha), _ptr(eta), _ptr3(u),
                                 _ptr(p), _ptr3(y_u), _ptr(y_p)))


def stream_copy(ctx: Context, src, dst):
    """dst = src with the library's plain streaming copy kernel (a bandwidth probe)."""
    if src.numel() * src.element_size() != dst.numel() * dst.element_size():
        raise ValueError("src and dst differ in size")
    for name, t in (("src", src), ("dst", dst)):
        if not t.is_cuda or t.device.index != ctx.device or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous tensor on cuda:{ctx.device}")
    check(lib().tng_stream_copy(ctx.h, _ptr(src), _ptr(dst), src.numel() * src.element_size()))


def check_device_buffer(ctx: Context, ptr: int, nbytes: int):
    """The library's own check of a device pointer (raises TngError if refused)."""
    check(lib().tng_check_device_buffer(ctx.h, _vp(ptr), nbytes))


def stokes_apply_layout(ctx: Context, mesh: Mesh, level: int, flags: int, f64: bool, hg_alpha: float = 0.0) -> dict:
    """Decomposition tng_stokes_apply uses for these arguments (launches nothing)."""
    out = (C.c_int * 8)()
    check(lib().tng_stokes_apply_layout(ctx.h, mesh.h, level, F64 if f64 else F32, flags, float(hg_alpha), out))
    keys = ("tile", "rs", "cpl", "wg", "ntile", "bands", "nchunk", "range")
    return dict(zip(keys, [int(v) for v in out]))


def interface_sum(ctx: Context, mesh: Mesh, level: int, fields, mode: int = 0):
    for c, f in enumerate(fields):
        _chk(ctx, f, fields[0].dtype, _nodes(mesh, level), f"fields[{c}]")
    arr = (_vp * len(fields))(*[f.data_ptr() for f in fields])
    check(lib().tng_interface_sum(ctx.h, mesh.h, level, _prec(fields[0]), mode, len(fields), arr))


def eta_from_temperature(ctx: Context, mesh: Mesh, level: int, T, E: float, F: float, eta_out):
    """Per-wedge viscosity exp(-E Tbar + F (1 - r_m)) from a nodal temperature field."""
    _chk(ctx, T, T.dtype, _nodes(mesh, level), "T")
    _chk(ctx, eta_out, T.dtype, _wedges(mesh, level), "eta_out")
    check(lib().tng_eta_from_temperature(ctx.h, mesh.h, level, _prec(T), _ptr(T), E, F,
                                         _ptr(eta_out)))


def eta_coarsen(ctx: Context, mesh: Mesh, fine_level: int, eta_fine, eta_coarse):
    _chk(ctx, eta_fine, eta_fine.dtype, _wedges(mesh, fine_level), "eta_fine")
    _chk(ctx, eta_coarse, eta_fine.dtype, _wedges(mesh, fine_level + 1), "eta_coarse")
    check(lib().tng_eta_coarsen(ctx.h, mesh.h, fine_level, _prec(eta_fine), _ptr(eta_fine),
                                _ptr(eta_coarse)))


def diag_A(ctx: Context, mesh: Mesh, level: int, eta, diag, hg_alpha: float = 0.0, twopoint: bool = False):
    """Diagonal of the viscous block (Dirichlet rows 1) into diag ([3, ...]);
    twopoint: of the two-radial-point operator."""
    _chk(ctx, eta, eta.dtype, _wedges(mesh, level), "eta")
    _chk3(ctx, diag, eta.dtype, _nodes(mesh, level), "diag")
    if twopoint:
        if hg_alpha != 0.0:
            raise ValueError("the two-radial-point rule is an alternative to hourglass control")
        check(lib().tng_diag_A_twopoint(ctx.h, mesh.h, level, _prec(eta), _ptr(eta), _ptr3(diag)))
    else:
        check(lib().tng_diag_A(ctx.h, mesh.h, level, _prec(eta), _ptr(eta), float(hg_alpha), _ptr3(diag)))


def pressure_mass(ctx: Context, mesh: Mesh, level: int, eta, mass):
    """Lumped inverse-viscosity pressure mass on level + 1."""
    _chk(ctx, eta, eta.dtype, _wedges(mesh, level), "eta")
    _chk(ctx, mass, eta.dtype, _nodes(mesh, level + 1), "mass")
    check(lib().tng_pressure_mass(ctx.h, mesh.h, level, _prec(eta), _ptr(eta), _ptr(mass)))


def _chk_smooth(ctx, mesh, level, eta, diag, b, x):
    _chk(ctx, eta, eta.dtype, _wedges(mesh, level), "eta")
    for name, v in (("diag", diag), ("b", b), ("x", x)):
        _chk3(ctx, v, eta.dtype, _nodes(mesh, level), name)


def smooth(ctx: Context, mesh: Mesh, level: int, eta, diag, b, x, degree: int, steps: int,
           lmin: float, lmax: float, hg_alpha: float = 0.0):
    _chk_smooth(ctx, mesh, level, eta, diag, b, x)
    check(lib().tng_smooth(ctx.h, mesh.h, level, _prec(eta), _ptr(eta), float(hg_alpha), _ptr3(diag), _ptr3(b),
                           _ptr3(x), degree, steps, lmin, lmax))


def smooth_noalloc(ctx: Context, mesh: Mesh, level: int, eta, diag, b, x, degree: int, steps: int,
                   lmin: float, lmax: float, hg_alpha: float = 0.0):
    """smooth() with the library's fixed device scratch array: no allocation, no synchronisation."""
    _chk_smooth(ctx, mesh, level, eta, diag, b, x)
    check(lib().tng_smooth_noalloc(ctx.h, mesh.h, level, _prec(eta), _ptr(eta), float(hg_alpha), _ptr3(diag),
                                   _ptr3(b), _ptr3(x), degree, steps, lmin, lmax))


def restrict(ctx: Context, mesh: Mesh, fine_level: int, f, c):
    _chk3(ctx, f, f[0].dtype, _nodes(mesh, fine_level), "f")
    _chk3(ctx, c, f[0].dtype, _nodes(mesh, fine_level + 1), "c")
    check(lib().tng_restrict(ctx.h, mesh.h, fine_level, _prec(f[0]), _ptr3(f), _ptr3(c)))


def prolong(ctx: Context, mesh: Mesh, fine_level: int, c, f):
    _chk3(ctx, c, c[0].dtype, _nodes(mesh, fine_level + 1), "c")
    _chk3(ctx, f, c[0].dtype, _nodes(mesh, fine_level), "f")
    check(lib().tng_prolong(ctx.h, mesh.h, fine_level, _prec(c[0]), _ptr3(c), _ptr3(f)))


class SolverOpts(C.Structure):
    _fields_ = [("mixed", C.c_int), ("restart", C.c_int), ("max_iters", C.c_int), ("rtol", C.c_double),
                ("cheb_degree", C.c_int), ("pre", C.c_int), ("post", C.c_int), ("levels", C.c_int),
                ("cheb_lo", C.c_double), ("cheb_hi", C.c_double), ("inner_rtol", C.c_double),
                ("inner_max_iters", C.c_int), ("max_outer", C.c_int), ("power_its", C.c_int),
                ("hg_alpha", C.c_double), ("graphs", C.c_int), ("op_flags", C.c_uint)]


class SolveInfo(C.Structure):
    _fields_ = [("outer_its", C.c_int), ("inner_its", C.c_int), ("rel_res", C.c_double),
                ("seconds", C.c_double), ("status", C.c_int), ("fp64_its", C.c_int)]


class StepOpts(C.Structure):
    _fields_ = [("Ra", C.c_double), ("E", C.c_double), ("F", C.c_double), ("dt", C.c_double),
                ("courant", C.c_double), ("T_inner", C.c_double), ("T_outer", C.c_double),
                ("energy_rtol", C.c_double), ("energy_max_iters", C.c_int), ("energy_restart", C.c_int),
                ("scheme", C.c_int)]


class StepInfo(C.Structure):
    _fields_ = [("stokes", SolveInfo), ("energy_its", C.c_int), ("energy_rel_res", C.c_double),
                ("dt", C.c_double), ("seconds", C.c_double)]


def rhs_buoyancy(ctx: Context, mesh: Mesh, level: int, T, Ra: float, f, bc_flags: int = 0):
    """Buoyancy Ra T rhat; bc_flags: OP_FREESLIP_INNER / OP_FREESLIP_OUTER spheres keep the
    tangential part in their rows (others zero)."""
    _chk(ctx, T, T.dtype, _nodes(mesh, level), "T")
    _chk3(ctx, f, T.dtype, _nodes(mesh, level), "f")
    if bc_flags:
        check(lib().tng_rhs_buoyancy_bc(ctx.h, mesh.h, level, _prec(T), bc_flags, _ptr(T), Ra, _ptr3(f)))
    else:
        check(lib().tng_rhs_buoyancy(ctx.h, mesh.h, level, _prec(T), _ptr(T), Ra, _ptr3(f)))


def rhs_buoyancy_tala(ctx: Context, mesh: Mesh, level: int, T, Ra: float, Tbar_nodes, rhoalpha_nodes, f):
    """Compressible buoyancy Ra rhobar alphabar T' rhat, T' = T - Tbar(r); profiles per node layer."""
    import numpy as np
    n1 = _counts(mesh, level)["n"] + 1
    tb = np.ascontiguousarray(Tbar_nodes, dtype=np.float64)
    ra = np.ascontiguousarray(rhoalpha_nodes, dtype=np.float64)
    if tb.shape != (n1,) or ra.shape != (n1,):
        raise ValueError("profiles must hold one value per radial node layer of the level")
    _chk(ctx, T, T.dtype, _nodes(mesh, level), "T")
    _chk3(ctx, f, T.dtype, _nodes(mesh, level), "f")
    check(lib().tng_rhs_buoyancy_tala(ctx.h, mesh.h, level, _prec(T), _ptr(T), Ra, _vp(tb.ctypes.data),
                                      _vp(ra.ctypes.data), _ptr3(f)))


def mmoc_advect(ctx: Context, mesh: Mesh, level: int, u, dt: float, T, T_hat):
    """T_hat = T at the departure points of the nodes (MMOC advection step), FP64."""
    import torch
    n = _nodes(mesh, level)
    _chk3(ctx, u, torch.float64, n, "u")
    _chk(ctx, T, torch.float64, n, "T")
    _chk(ctx, T_hat, torch.float64, n, "T_hat")
    check(lib().tng_mmoc_advect(ctx.h, mesh.h, level, _ptr3(u), float(dt), _ptr(T), _ptr(T_hat)))


def energy_apply(ctx: Context, mesh: Mesh, level: int, u, dt: float, T, y):
    n = _nodes(mesh, level)
    _chk3(ctx, u, T.dtype, n, "u")
    _chk(ctx, T, T.dtype, n, "T")
    _chk(ctx, y, T.dtype, n, "y")
    check(lib().tng_energy_apply(ctx.h, mesh.h, level, _prec(T), _ptr3(u), dt, _ptr(T), _ptr(y)))


class StokesSolver:
    """FGMRES + block-triangular Schur preconditioner + multigrid (library-owned state)."""

    def __init__(self, ctx: Context, mesh: Mesh, **opts):
        o = SolverOpts()
        check(lib().tng_solver_opts_default(C.byref(o)))
        for k, v in opts.items():
            if not hasattr(o, k):
                raise KeyError(k)
            setattr(o, k, v)
        self.opts = o
        self.ctx, self.mesh = ctx, mesh
        h = _vp()
        check(lib().tng_stokes_solver_create(ctx.h, mesh.h, C.byref(o), C.byref(h)))
        self.h = h

    def _chk_f64(self, t, numel, name):
        import torch
        _chk(self.ctx, t, torch.float64, numel, name)

    def setup(self, eta):
        self._chk_f64(eta, _wedges(self.mesh, 0), "eta")
        check(lib().tng_stokes_solver_setup(self.h, _ptr(eta)))

    def solve(self, f, g, u, p, eta=None, raise_on_fail: bool = True) -> dict:
        import torch
        nu, np_ = _nodes(self.mesh, 0), _nodes(self.mesh, 1)
        self._chk_f64(eta, _wedges(self.mesh, 0), "eta")
        _chk3(self.ctx, f, torch.float64, nu, "f")
        _chk3(self.ctx, u, torch.float64, nu, "u")
        self._chk_f64(g, np_, "g")
        self._chk_f64(p, np_, "p")
        info = SolveInfo()
        rc = lib().tng_stokes_solve(self.h, _ptr(eta), _ptr3(f), _ptr(g), _ptr3(u), _ptr(p), C.byref(info))
        out = {k: getattr(info, k) for k, _ in SolveInfo._fields_}
        out["rc"] = rc
        if rc != 0 and raise_on_fail:
            check(rc)
        return out

    def energy_step(self, T, u, p, H=None, Ra=1e5, E=0.0, F=0.0, dt=0.0, courant=1.0, T_inner=1.0,
                    T_outer=0.0, energy_rtol=1e-8, energy_max_iters=200, energy_restart=20, scheme: str = "supg",
                    raise_on_fail: bool = True) -> dict:
        """One coupled step: Stokes solve with eta(T), then the energy solve (T in/out);
        scheme "supg" or "mmoc"."""
        if scheme not in ("supg", "mmoc"):
            raise ValueError("scheme must be 'supg' or 'mmoc'")
        o = StepOpts(Ra, E, F, dt, courant, T_inner, T_outer, energy_rtol, energy_max_iters, energy_restart,
                     1 if scheme == "mmoc" else 0)
        info = StepInfo()
        rc = lib().tng_energy_step(self.h, C.byref(o), _ptr(H), _ptr(T), _ptr3(u), _ptr(p), C.byref(info))
        out = {"rc": rc, "energy_its": info.energy_its, "energy_rel_res": info.energy_rel_res,
               "dt": info.dt, "seconds": info.seconds,
               "stokes": {k: getattr(info.stokes, k) for k, _ in SolveInfo._fields_}}
        if rc != 0 and raise_on_fail:
            check(rc)
        return out

    def vcycle(self, b, x):
        check(lib().tng_stokes_solver_vcycle(self.h, _ptr3(b), _ptr3(x)))

    def close(self):
        if getattr(self, "h", None):
            lib().tng_stokes_solver_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Request server: levels = [(mt, nr), ...]; the slots of a level form one
    lockstep batch (one launch per kernel for all running slots) on the level's
    own stream; solver options as for StokesSolver (normally mixed precision)."""

    def __init__(self, ctx: Context, levels, budget_bytes: int, max_slots: int = 64, **opts):
        o = SolverOpts()
        check(lib().tng_solver_opts_default(C.byref(o)))
        for k, v in opts.items():
            setattr(o, k, v)
        flat = (C.c_int * (2 * len(levels)))(*[x for lv in levels for x in lv])
        h = _vp()
        check(lib().tng_server_create(ctx.h, flat, len(levels), int(budget_bytes), max_slots, C.byref(o),
                                      C.byref(h)))
        self.h, self.ctx, self.levels = h, ctx, list(levels)
        self._keep = {}

    def submit(self, level_idx: int, T, log10_contrast: float, Ra: float, u, p) -> int:
        t = C.c_longlong()
        check(lib().tng_server_submit(self.h, level_idx, _ptr(T), log10_contrast, Ra, _ptr3(u), _ptr(p),
                                      C.byref(t)))
        self._keep[t.value] = (T, u, p)      # borrowed buffers stay alive until done
        return t.value

    def poll(self, ticket: int) -> dict:
        done = C.c_int()
        info = SolveInfo()
        lat, q = C.c_double(), C.c_double()
        rc = lib().tng_server_poll(self.h, ticket, C.byref(done), C.byref(info), C.byref(lat), C.byref(q))
        out = {"done": bool(done.value), "rc": rc}
        if done.value:
            out.update({k: getattr(info, k) for k, _ in SolveInfo._fields_})
            out["latency"] = lat.value
            out["queue"] = q.value
            self._keep.pop(ticket, None)
        return out

    def wait(self, ticket: int = 0):
        check(lib().tng_server_wait(self.h, ticket))

    def stats(self) -> dict:
        b, sl, bu, qu = C.c_longlong(), C.c_int(), C.c_int(), C.c_int()
        check(lib().tng_server_stats(self.h, C.byref(b), C.byref(sl), C.byref(bu), C.byref(qu)))
        return {"bytes_in_use": b.value, "slots": sl.value, "busy": bu.value, "queued": qu.value}

    def close(self):
        if getattr(self, "h", None):
            lib().tng_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
