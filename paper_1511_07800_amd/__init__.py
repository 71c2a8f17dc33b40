"""MI355X-native S-TPLS channel-flow time step (arXiv 1511.07800).

The computation lives in ``libstp.so`` (HIP kernels for gfx950 behind the C
ABI of ``include/stp.h``).  This package only marshals arguments: torch
provides the device workspace and the stream, ctypes calls the library.
Nothing here computes any part of the method, and there is no CPU fallback:
if the library is missing the calls raise.
"""
from .binding import (  # noqa: F401
    STP_OK, STP_EINVAL, STP_ENOMEM, STP_EDEVICE, STP_ENOCONV, STP_ENAN,
    STP_FP64, STP_MIXED, STP_WS_PREV, STP_WS_ZERO, STP_WS_LEARNED,
    STP_U, STP_V, STP_W, STP_P, STP_NUT, STP_RHS, STP_DTYPE_F64, STP_DTYPE_F32,
    StpError, Config, SolveStats, StepStats, Channel, load_library, library_path, residual_norm_noalloc,
)
