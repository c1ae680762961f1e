"""MI355X-native matrix-free wedge Stokes library (TERRA-NG, arXiv 2609.21633).

The compute path is the C-ABI library ``libtng.so`` (hand-written HIP kernels
for gfx950, declared in ``include/tng.h``); this package is a thin ctypes
binding with the same names.  PyTorch tensors only carry device memory and
the stream.  Importing the binding does not load the library; the first call
does, and fails loudly if ``libtng.so`` has not been built.
"""
from .binding import (  # noqa: F401
    OP_A, OP_B, OP_BT, OP_DIRICHLET, OP_FREESLIP_INNER, OP_FREESLIP_OUTER, OP_TALA, OP_TWOPOINT, TngError, Context, Mesh, StokesSolver, diag_A, eta_coarsen,
    eta_from_temperature, interface_sum, lib, pressure_mass, prolong, restrict, smooth, stokes_apply,
    rhs_buoyancy, energy_apply, Server, smooth_noalloc, stokes_apply_layout, stream_copy, check_device_buffer, rhs_buoyancy_tala, mmoc_advect,
)
