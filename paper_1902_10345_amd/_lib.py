"""ctypes binding of libgemm_mi355x.so -- argument marshalling only.

Every function here has the name of the C entry point it wraps (see
include/gemm_mi355x.h).  Matrix arguments may be torch tensors (their
data_ptr() is passed) or raw integer device addresses; the stream defaults to
torch's current stream on the current device.  A nonzero status raises
GemmError carrying the status and the library's thread-local message.

There is no fallback: if the shared library is missing the import fails.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgemm_mi355x.so")

STATUS_OK = 0
STATUS_HIP_ERROR = 1
STATUS_NO_MEMORY = 2
STATUS_NOT_READY = 3
STATUS_UNSUPPORTED = 4
STATUS_REJECTED = 5
STATUS_UNKNOWN = 6


class GemmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("status %d: %s" % (status, message))
        self.status = status
        self.message = message


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            "HIP library %s is not built; run `python -c 'import __graft_entry__ as g; g.build()'`"
            % LIB_PATH)
    # torch must own the HIP runtime: load it first so that the library's
    # libamdhip64 dependency resolves to the runtime torch already mapped.
    import torch  # noqa: F401
    return ctypes.CDLL(LIB_PATH)


lib = _load()

_i64, _f32, _vp, _int, _sz, _dbl = (ctypes.c_int64, ctypes.c_float, ctypes.c_void_p,
                                     ctypes.c_int, ctypes.c_size_t, ctypes.c_double)


def _sig(name, restype, *args):
    fn = getattr(lib, name)
    fn.restype = restype
    fn.argtypes = list(args)
    return fn


_sig("gemm_last_error", ctypes.c_char_p)
_sig("gemm_version", ctypes.c_char_p)
_sig("gemm_f32", _int, _i64, _i64, _i64, _f32, _vp, _i64, _vp, _i64, _f32, _vp, _i64, _vp)
_sig("gemm_f32_3xbf16", _int, _i64, _i64, _i64, _f32, _vp, _i64, _vp, _i64, _f32, _vp, _i64, _int,
     _vp)
_sig("split_bf16x3", _int, _i64, _vp, _vp, _vp, _vp, _vp)
_sig("gemm_fp8_workspace_bytes", _sz, _i64, _i64, _i64)
_sig("gemm_fp8_scaled", _int, _i64, _i64, _i64, _f32, _vp, _i64, _vp, _i64, _f32, _vp, _i64, _vp,
     _sz, _vp)
_sig("fp8_quantize", _int, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _sz, _vp)
_sig("gemm_fp8_prequantized", _int, _i64, _i64, _i64, _f32, _vp, _sz, _f32, _vp, _i64, _vp)
_sig("fp8_e4m3_encode", _int, _i64, _vp, _vp, _vp)
_sig("gemm_num_configs", _int, _int)
_sig("gemm_config_name", ctypes.c_char_p, _int, _int)
_sig("gemm_default_config", _int, _int, _i64, _i64, _i64)
_sig("gemm_run_config", _int, _int, _int, _i64, _i64, _i64, _f32, _vp, _i64, _vp, _i64, _f32, _vp,
     _i64, _int, _vp, _sz, _vp)
_sig("err_norm_workspace_bytes", _sz)
_sig("err_norm_f64", _int, _i64, _i64, _vp, _i64, _vp, _vp, _vp, _vp, _sz, _vp)


def ptr(x) -> int | None:
    """Device (or host) address of a tensor / int / None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if hasattr(x, "ctypes"):
        return x.ctypes.data
    raise TypeError("cannot take the address of %r" % type(x))


def stream_handle(stream=None) -> int:
    import torch
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def gemm_last_error() -> str:
    return lib.gemm_last_error().decode()


def gemm_version() -> str:
    return lib.gemm_version().decode()


last_error = gemm_last_error
version = gemm_version


def check(status: int) -> int:
    if status != STATUS_OK:
        raise GemmError(status, last_error())
    return status


def gemm_f32(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, stream=None):
    return check(lib.gemm_f32(M, N, K, alpha, ptr(A), lda, ptr(B), ldb, beta, ptr(C), ldc,
                              stream_handle(stream)))


def gemm_f32_3xbf16(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, n_products=3, stream=None):
    return check(lib.gemm_f32_3xbf16(M, N, K, alpha, ptr(A), lda, ptr(B), ldb, beta, ptr(C), ldc,
                                     n_products, stream_handle(stream)))


def split_bf16x3(n, x, p0, p1, p2=None, stream=None):
    return check(lib.split_bf16x3(n, ptr(x), ptr(p0), ptr(p1), ptr(p2), stream_handle(stream)))


def gemm_fp8_workspace_bytes(M, N, K) -> int:
    return int(lib.gemm_fp8_workspace_bytes(M, N, K))


def gemm_fp8_scaled(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, workspace, ws_bytes,
                    stream=None):
    return check(lib.gemm_fp8_scaled(M, N, K, alpha, ptr(A), lda, ptr(B), ldb, beta, ptr(C), ldc,
                                     ptr(workspace), ws_bytes, stream_handle(stream)))


def fp8_quantize(M, N, K, A, lda, B, ldb, workspace, ws_bytes, stream=None):
    return check(lib.fp8_quantize(M, N, K, ptr(A), lda, ptr(B), ldb, ptr(workspace), ws_bytes,
                                  stream_handle(stream)))


def gemm_fp8_prequantized(M, N, K, alpha, workspace, ws_bytes, beta, C, ldc, stream=None):
    return check(lib.gemm_fp8_prequantized(M, N, K, alpha, ptr(workspace), ws_bytes, beta, ptr(C),
                                           ldc, stream_handle(stream)))


def fp8_e4m3_encode(n, x, codes, stream=None):
    return check(lib.fp8_e4m3_encode(n, ptr(x), ptr(codes), stream_handle(stream)))


def fp8_workspace_layout(M, N, K):
    """Byte offsets of the workspace regions (qa, qbT, sa, sb) and Kp, as
    documented in the header."""
    def a256(x):
        return (x + 255) & ~255
    Kp = ((K + 127) // 128) * 128
    qa = 0
    qb = a256(qa + M * Kp)
    sa = a256(qb + N * Kp)
    sb = a256(sa + 4 * M)
    return {"Kp": Kp, "qa": qa, "qb": qb, "sa": sa, "sb": sb}


PATH_F32, PATH_3XBF16, PATH_FP8 = 0, 1, 2


def gemm_num_configs(path) -> int:
    return int(lib.gemm_num_configs(path))


def gemm_config_name(path, cfg) -> str:
    return lib.gemm_config_name(path, cfg).decode()


def gemm_default_config(path, M, N, K) -> int:
    return int(lib.gemm_default_config(path, M, N, K))


def gemm_run_config(path, cfg, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, n_products=3,
                    workspace=None, ws_bytes=0, stream=None):
    return check(lib.gemm_run_config(path, cfg, M, N, K, alpha, ptr(A), lda, ptr(B), ldb, beta,
                                     ptr(C), ldc, n_products, ptr(workspace), ws_bytes,
                                     stream_handle(stream)))


def err_norm_workspace_bytes() -> int:
    return int(lib.err_norm_workspace_bytes())


def err_norm_f64(M, N, C, ldc, Cref, den, out, workspace, ws_bytes, stream=None):
    return check(lib.err_norm_f64(M, N, ptr(C), ldc, ptr(Cref), ptr(den), ptr(out),
                                  ptr(workspace), ws_bytes, stream_handle(stream)))
