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
STATUS_CANCELLED = 7
STATUS_TIMED_OUT = 8


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
_sig("gemm_splitk_default_splits", _int, _i64, _i64, _i64)
_sig("gemm_splitk_workspace_bytes", _sz, _i64, _i64, _i64, _int)
_sig("gemm_f32_3xbf16_splitk", _int, _i64, _i64, _i64, _f32, _vp, _i64, _vp, _i64, _f32, _vp, _i64,
     _int, _int, _vp, _sz, _vp)
_sig("gemm_f32_3xbf16_splitk_noalloc", _int, _i64, _i64, _i64, _f32, _vp, _i64, _vp, _i64, _f32, _vp,
     _i64, _int, _int, _vp)
_sig("split_bf16x3", _int, _i64, _vp, _vp, _vp, _vp, _vp)
_sig("gemm_fp8_workspace_bytes", _sz, _i64, _i64, _i64)
_sig("gemm_fp8_scaled", _int, _i64, _i64, _i64, _f32, _vp, _i64, _vp, _i64, _f32, _vp, _i64, _vp,
     _sz, _vp)
_sig("fp8_quantize", _int, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _sz, _vp)
_sig("gemm_fp8_prequantized", _int, _i64, _i64, _i64, _f32, _vp, _sz, _f32, _vp, _i64, _vp)
_sig("fp8_e4m3_encode", _int, _i64, _vp, _vp, _vp)
_sig("gemm_f64", _int, _i64, _i64, _i64, _dbl, _vp, _i64, _vp, _i64, _dbl, _vp, _i64, _vp)
_sig("gemm_f64_run_config", _int, _int, _i64, _i64, _i64, _dbl, _vp, _i64, _vp, _i64, _dbl, _vp,
     _i64, _vp)
_sig("gemm_f64_strided_batched", _int, _i64, _i64, _i64, _dbl, _vp, _i64, _i64, _vp, _i64, _i64,
     _dbl, _vp, _i64, _i64, _i64, _vp)
_sig("gemm_strided_batched", _int, _int, _i64, _i64, _i64, _f32, _vp, _i64, _i64, _vp, _i64, _i64,
     _f32, _vp, _i64, _i64, _i64, _int, _vp)
_sig("gemm_ex", _int, _int, _int, _int, _i64, _i64, _i64, _f32, _vp, _i64, _vp, _i64, _f32, _vp,
     _i64, _int, _int, _vp, _sz, _vp)


class gemm_problem(ctypes.Structure):
    _fields_ = [("M", _i64), ("N", _i64), ("K", _i64), ("lda", _i64), ("ldb", _i64),
                ("ldc", _i64), ("A", _vp), ("B", _vp), ("C", _vp), ("alpha", _f32),
                ("beta", _f32)]


_PP = ctypes.POINTER(gemm_problem)
_IP = ctypes.POINTER(_int)
_sig("grouped_gemm_workspace_bytes", _sz, _int)
_sig("grouped_default_variant", _int, _i64, _i64, _i64)
_sig("grouped_gemm", _int, _PP, _int, _int, _IP, _vp, _sz, _vp)
_sig("grouped_graph_create", _int, _PP, _int, _int, _IP, _vp, _sz, _vp, ctypes.POINTER(_vp))
_sig("grouped_graph_launch", _int, _vp, _vp)
_sig("grouped_graph_destroy", _int, _vp)
_sig("server_create", _int, _vp, _sz, _int, _int, _int, ctypes.POINTER(_vp))
_sig("server_now", _dbl, _vp)
_sig("server_submit", _int, _vp, _i64, _i64, _i64, _f32, _vp, _vp, _f32, _vp, _vp, _dbl,
     ctypes.POINTER(ctypes.c_uint64))
_sig("server_poll", _int, _vp, ctypes.c_uint64, ctypes.POINTER(_dbl), ctypes.POINTER(_dbl))
_sig("server_drain", _int, _vp, _dbl)
_sig("server_stats", _int, _vp, ctypes.POINTER(_dbl), ctypes.POINTER(_dbl), ctypes.POINTER(_dbl),
     ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(_dbl), ctypes.POINTER(_dbl),
     ctypes.POINTER(_int), ctypes.POINTER(_sz), ctypes.POINTER(ctypes.c_uint64),
     ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(_int))
_sig("server_cancel", _int, _vp, ctypes.c_uint64)
_sig("server_set_queue_timeout", _int, _vp, _dbl)
_sig("server_destroy", _int, _vp)
_sig("gemm_autotune", _int, _int, _i64, _i64, _i64, _f32, _vp, _i64, _vp, _i64, _f32, _vp, _i64,
     _int, _vp, _sz, _int, _vp, ctypes.POINTER(_int))
_sig("grouped_autotune", _int, _PP, _int, _int, _vp, _sz, _int, _vp, ctypes.POINTER(_int))
_sig("gemm_tuner_save", _int, ctypes.c_char_p)
_sig("gemm_tuner_load", _int, ctypes.c_char_p)
_sig("gemm_tuner_clear", None)
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


def gemm_splitk_default_splits(M, N, K) -> int:
    return int(lib.gemm_splitk_default_splits(M, N, K))


def gemm_splitk_workspace_bytes(M, N, K, splits=0) -> int:
    return int(lib.gemm_splitk_workspace_bytes(M, N, K, splits))


def gemm_f32_3xbf16_splitk(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, n_products=3, splits=0,
                           workspace=None, ws_bytes=0, stream=None):
    return check(lib.gemm_f32_3xbf16_splitk(M, N, K, alpha, ptr(A), lda, ptr(B), ldb, beta, ptr(C),
                                            ldc, n_products, splits, ptr(workspace), ws_bytes,
                                            stream_handle(stream)))


# GEMM_NOALLOC_SCRATCH_BYTES of the header: the fixed scratch of the
# no-allocation split-K entry point
NOALLOC_SCRATCH_BYTES = 64 << 20


def gemm_f32_3xbf16_splitk_noalloc(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, n_products=3,
                                   splits=0, stream=None):
    return check(lib.gemm_f32_3xbf16_splitk_noalloc(M, N, K, alpha, ptr(A), lda, ptr(B), ldb, beta,
                                                    ptr(C), ldc, n_products, splits,
                                                    stream_handle(stream)))


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


PATH_F32, PATH_3XBF16, PATH_FP8, PATH_FP8_PREQUANTIZED, PATH_F64 = 0, 1, 2, 3, 4


def gemm_f64(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, stream=None):
    return check(lib.gemm_f64(M, N, K, alpha, ptr(A), lda, ptr(B), ldb, beta, ptr(C), ldc,
                              stream_handle(stream)))


def gemm_strided_batched(path, M, N, K, alpha, A, lda, stride_a, B, ldb, stride_b, beta, C, ldc,
                         stride_c, batch, n_products=3, stream=None):
    return check(lib.gemm_strided_batched(path, M, N, K, alpha, ptr(A), lda, stride_a, ptr(B), ldb,
                                          stride_b, beta, ptr(C), ldc, stride_c, batch, n_products,
                                          stream_handle(stream)))


def gemm_f64_run_config(cfg, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, stream=None):
    return check(lib.gemm_f64_run_config(cfg, M, N, K, alpha, ptr(A), lda, ptr(B), ldb, beta,
                                         ptr(C), ldc, stream_handle(stream)))


def gemm_f64_strided_batched(M, N, K, alpha, A, lda, stride_a, B, ldb, stride_b, beta, C, ldc,
                             stride_c, batch, stream=None):
    return check(lib.gemm_f64_strided_batched(M, N, K, alpha, ptr(A), lda, stride_a, ptr(B), ldb,
                                              stride_b, beta, ptr(C), ldc, stride_c, batch,
                                              stream_handle(stream)))
ROW_MAJOR, COL_MAJOR = 101, 102
NO_TRANS, TRANS, CONJ_TRANS = 111, 112, 113


def gemm_ex(order, trans_a, trans_b, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
            path=PATH_3XBF16, n_products=3, workspace=None, ws_bytes=0, stream=None):
    return check(lib.gemm_ex(order, trans_a, trans_b, M, N, K, alpha, ptr(A), lda, ptr(B), ldb,
                             beta, ptr(C), ldc, path, n_products, ptr(workspace), ws_bytes,
                             stream_handle(stream)))


def problem_array(problems):
    """ctypes array of gemm_problem from tuples (M, N, K, A, lda, B, ldb, C, ldc,
    alpha, beta), with A/B/C tensors or device addresses."""
    arr = (gemm_problem * len(problems))()
    for i, (M, N, K, A, lda, B, ldb, C, ldc, alpha, beta) in enumerate(problems):
        arr[i] = gemm_problem(M, N, K, lda, ldb, ldc, ptr(A), ptr(B), ptr(C), alpha, beta)
    return arr


def _variants(tile_variant, count):
    if tile_variant is None:
        return None
    v = (_int * count)(*[int(x) for x in tile_variant])
    return v


def server_create(arena, arena_bytes, max_slots, path, n_streams):
    """Returns an opaque server handle (int)."""
    h = _vp()
    check(lib.server_create(ptr(arena), arena_bytes, max_slots, path, n_streams, ctypes.byref(h)))
    return h.value


def server_now(server) -> float:
    return float(lib.server_now(server))


def server_submit(server, M, N, K, alpha, hA, hB, beta, hC0, hC_out, arrival=-1.0) -> int:
    t = ctypes.c_uint64()
    check(lib.server_submit(server, M, N, K, alpha, ptr(hA), ptr(hB), beta, ptr(hC0), ptr(hC_out),
                            arrival, ctypes.byref(t)))
    return t.value


def server_poll(server, ticket):
    """None while in flight, else (latency_ms, result_latency_ms)."""
    a, b = _dbl(), _dbl()
    st = lib.server_poll(server, ticket, ctypes.byref(a), ctypes.byref(b))
    if st == STATUS_NOT_READY:
        return None
    check(st)
    return a.value, b.value


def server_drain(server, timeout_s=60.0):
    return check(lib.server_drain(server, timeout_s))


def server_cancel(server, ticket):
    """Cancel a request that is still queued (GemmError with STATUS_NOT_READY
    once it has been admitted)."""
    return check(lib.server_cancel(server, ticket))


def server_set_queue_timeout(server, seconds):
    return check(lib.server_set_queue_timeout(server, float(seconds)))


def server_stats(server) -> dict:
    p50, p99, tf, rp50, rp99 = _dbl(), _dbl(), _dbl(), _dbl(), _dbl()
    done, rej, fail = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    mif, mcs = _int(), _int()
    hw = _sz()
    check(lib.server_stats(server, ctypes.byref(p50), ctypes.byref(p99), ctypes.byref(tf),
                           ctypes.byref(done), ctypes.byref(rp50), ctypes.byref(rp99),
                           ctypes.byref(mif), ctypes.byref(hw), ctypes.byref(rej),
                           ctypes.byref(fail), ctypes.byref(mcs)))
    return {"p50_ms": p50.value, "p99_ms": p99.value, "tflops": tf.value,
            "completed": done.value, "result_p50_ms": rp50.value, "result_p99_ms": rp99.value,
            "max_in_flight": mif.value, "arena_high_water_bytes": hw.value,
            "rejected": rej.value, "failed": fail.value, "max_concurrent_steps": mcs.value}


def server_destroy(server):
    return check(lib.server_destroy(server))


def gemm_autotune(path, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, n_products=3,
                  workspace=None, ws_bytes=0, reps=5, stream=None) -> int:
    best = _int()
    check(lib.gemm_autotune(path, M, N, K, alpha, ptr(A), lda, ptr(B), ldb, beta, ptr(C), ldc,
                            n_products, ptr(workspace), ws_bytes, reps, stream_handle(stream),
                            ctypes.byref(best)))
    return best.value


def grouped_autotune(problems, count, path, workspace, ws_bytes, reps=3, stream=None):
    out = (_int * count)()
    check(lib.grouped_autotune(problems, count, path, ptr(workspace), ws_bytes, reps,
                               stream_handle(stream), out))
    return list(out)


def gemm_tuner_save(json_path):
    return check(lib.gemm_tuner_save(json_path.encode()))


def gemm_tuner_load(json_path):
    return check(lib.gemm_tuner_load(json_path.encode()))


def gemm_tuner_clear():
    lib.gemm_tuner_clear()


def grouped_gemm_workspace_bytes(count) -> int:
    return int(lib.grouped_gemm_workspace_bytes(count))


def grouped_default_variant(M, N, K) -> int:
    return int(lib.grouped_default_variant(M, N, K))


def grouped_gemm(problems, count, path, tile_variant, workspace, ws_bytes, stream=None):
    """problems: a ctypes gemm_problem array (see problem_array)."""
    return check(lib.grouped_gemm(problems, count, path, _variants(tile_variant, count),
                                  ptr(workspace), ws_bytes, stream_handle(stream)))


def grouped_graph_create(problems, count, path, tile_variant, workspace, ws_bytes, stream=None):
    """Returns an opaque graph handle (int)."""
    h = _vp()
    check(lib.grouped_graph_create(problems, count, path, _variants(tile_variant, count),
                                   ptr(workspace), ws_bytes, stream_handle(stream),
                                   ctypes.byref(h)))
    return h.value


def grouped_graph_launch(graph, stream=None):
    return check(lib.grouped_graph_launch(graph, stream_handle(stream)))


def grouped_graph_destroy(graph):
    return check(lib.grouped_graph_destroy(graph))


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
