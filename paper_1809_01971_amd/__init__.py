"""MI355X rank-structured PCG solver for the fractional-Laplacian control equation.

The compute runs in ``libtp.so`` (hand-written HIP for gfx950); this package only
marshals arguments through its C ABI (include/tp.h).  PyTorch supplies device
memory and the stream.  Importing the package loads the library and raises if it
is missing: there is no CPU fallback.
"""
from ._tp import (  # noqa: F401
    Context, Tensor, Symbol, Rhs, TPError, cp_struct, library_path, load_library,
    TP_OK, TP_EINVAL, TP_ENOMEM, TP_ENOCONV, TP_ERANK, TP_EHIP,
    TP_FP64, TP_MIXED, TP_SYM_FIT, TP_SYM_SINC, TP_STOP_ERROR, TP_STOP_RESIDUAL,
)
