"""MI355X (gfx950) dense GEMM library: C <- alpha*A*B + beta*C.

The compute path is the C-ABI shared library libgemm_mi355x.so (hand-written
HIP kernels); this package is its thin Python binding plus tensor-level
conveniences that only marshal arguments.  Importing it fails loudly when the
library is not built: there is no CPU fallback.
"""
from ._lib import *  # noqa: F401,F403
from ._lib import GemmError, lib, ptr, stream_handle, version  # noqa: F401
from . import ops  # noqa: F401
