"""FP64 CPU oracle for the GEMM library -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports, links or calls anything here; the two share
no code.  The arithmetic lives in ``oracle.c`` (plain C, binary64); this module
only marshals numpy arrays into it.

What it computes (Ben-Nun et al., SC'19):
  * ``gemm``           -- Cref = alpha*A@B + beta*C0, the matrix multiplication
                          of Sec. 3.3 (map producing A[i,k]*B[k,j], reduce over
                          k) with the BLAS scalars of the external-code call in
                          Sec. 2.1; binary64, natural k order.
  * ``gemm_abs``       -- |alpha||A||B| + |beta||C0|, the componentwise
                          (Higham) error denominator.
  * ``split_bf16x3`` / ``gemm_bf16_split`` -- round-to-nearest-even bfloat16
                          three-way split and the exact sum of the selected
                          split products (not in the paper; IEEE-754 RNE).
  * ``e4m3_*`` / ``fp8_*`` -- OCP OFP8 E4M3 encode/decode (RNE, saturating),
                          per-row / per-column scales, and the dequantised-input
                          product (not in the paper).
  * ``gemm_op``        -- the same product over operands held in a storage
                          order with transpose flags, as the BLAS-style
                          external-code call of Sec. 2.1 passes them:
                          alpha*op(A)@op(B) + beta*C, op(X) = X or X^T.
  * ``dgemm``          -- the product for binary64 operands, evaluated in
                          double-double (compensated dot products, Ogita-Rump-
                          Oishi "Dot2") and rounded once, so it is far more
                          accurate than a binary64 result under test.
  * ``norms``          -- relative Frobenius error and componentwise maximum.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
             "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    i64, dbl, vp, ci = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_int
    lib.orc_gemm.argtypes = [i64, i64, i64, dbl, vp, i64, vp, i64, dbl, vp, i64, vp, ci, ci]
    lib.orc_gemm.restype = None
    lib.orc_bf16_rne.argtypes = [ctypes.c_float]
    lib.orc_bf16_rne.restype = ctypes.c_float
    lib.orc_split_bf16x3.argtypes = [i64, vp, vp, vp, vp]
    lib.orc_split_bf16x3.restype = None
    lib.orc_gemm_bf16_split.argtypes = [i64, i64, i64, dbl, vp, i64, vp, i64, dbl, vp, i64, ci, vp, ci]
    lib.orc_gemm_bf16_split.restype = None
    lib.orc_e4m3_value.argtypes = [ctypes.c_uint8]
    lib.orc_e4m3_value.restype = dbl
    lib.orc_e4m3_decode.argtypes = [i64, vp, vp]
    lib.orc_e4m3_decode.restype = None
    lib.orc_e4m3_encode.argtypes = [i64, vp, vp]
    lib.orc_e4m3_encode.restype = None
    lib.orc_fp8_scales_rows.argtypes = [i64, i64, vp, i64, vp]
    lib.orc_fp8_scales_rows.restype = None
    lib.orc_fp8_scales_cols.argtypes = [i64, i64, vp, i64, vp]
    lib.orc_fp8_scales_cols.restype = None
    lib.orc_fp8_quantize_rows.argtypes = [i64, i64, vp, i64, vp, vp]
    lib.orc_fp8_quantize_rows.restype = None
    lib.orc_fp8_quantize_cols.argtypes = [i64, i64, vp, i64, vp, vp]
    lib.orc_fp8_quantize_cols.restype = None
    lib.orc_gemm_fp8_dequant.argtypes = [i64, i64, i64, dbl, vp, vp, vp, vp, dbl, vp, i64, vp, ci]
    lib.orc_gemm_fp8_dequant.restype = None
    lib.orc_dgemm.argtypes = [i64, i64, i64, dbl, vp, i64, vp, i64, dbl, vp, i64, vp, ci, ci]
    lib.orc_dgemm.restype = None
    lib.orc_norms.argtypes = [i64, i64, vp, i64, vp, vp, vp]
    lib.orc_norms.restype = None
    _lib = lib
    return lib


def _p(a):
    return None if a is None else a.ctypes.data


def _f32(a):
    a = np.asarray(a)
    if a.dtype != np.float32:
        raise TypeError("oracle expects float32 inputs, got %s" % a.dtype)
    if a.ndim == 2 and a.size > 0 and a.shape[1] > 1 and a.strides[1] != 4:
        raise ValueError("rows must be contiguous")
    return a


def _ld(a, ncols):
    """Row stride in elements of a 2-D float32 array (or view)."""
    if a.ndim != 2:
        raise ValueError("expected a 2-D array")
    if a.shape[0] > 1 and a.shape[1] > 0:
        return a.strides[0] // a.itemsize
    return max(1, ncols)


def gemm(A, B, alpha=1.0, beta=0.0, C0=None, nthreads=0):
    """Cref = alpha*A@B + beta*C0 in binary64 (C0 unread when beta == 0)."""
    A, B = _f32(A), _f32(B)
    M, K = A.shape
    K2, N = B.shape
    assert K == K2
    out = np.empty((M, N), dtype=np.float64)
    c0, ldc0 = None, max(1, N)
    if beta != 0.0:
        C0 = _f32(C0)
        assert C0.shape == (M, N)
        c0, ldc0 = C0, _ld(C0, N)
    _load().orc_gemm(M, N, K, float(alpha), _p(A), _ld(A, K), _p(B), _ld(B, N),
                     float(beta), _p(c0), ldc0, _p(out), 0, int(nthreads))
    return out


def gemm_abs(A, B, alpha=1.0, beta=0.0, C0=None, nthreads=0):
    """|alpha|*|A|@|B| + |beta|*|C0| in binary64 (componentwise denominator)."""
    A, B = _f32(A), _f32(B)
    M, K = A.shape
    _, N = B.shape
    out = np.empty((M, N), dtype=np.float64)
    c0, ldc0 = None, max(1, N)
    if beta != 0.0:
        C0 = _f32(C0)
        c0, ldc0 = C0, _ld(C0, N)
    _load().orc_gemm(M, N, K, float(alpha), _p(A), _ld(A, K), _p(B), _ld(B, N),
                     float(beta), _p(c0), ldc0, _p(out), 1, int(nthreads))
    return out


ROW_MAJOR, COL_MAJOR = 101, 102
NO_TRANS, TRANS = 111, 112


def stored_matrix(buf, order, rows, cols, ld):
    """The rows x cols binary32 matrix held in the flat buffer `buf`: element
    (r, c) sits at r*ld + c in row-major order and at c*ld + r in
    column-major order."""
    buf = np.asarray(buf, dtype=np.float32).reshape(-1)
    r = np.arange(rows, dtype=np.int64)[:, None]
    c = np.arange(cols, dtype=np.int64)[None, :]
    idx = r * ld + c if order == ROW_MAJOR else c * ld + r
    return np.ascontiguousarray(buf[idx], dtype=np.float32)


def gemm_op(order, trans_a, trans_b, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
            nthreads=0):
    """alpha*op(A)@op(B) + beta*C in binary64 (M x N), reading each operand
    from its flat storage buffer.  op(A) is M x K: A itself (stored M x K) or,
    with trans_a == TRANS, the transpose of A stored K x M; op(B) likewise
    (B stored K x N, or N x K).  C (stored M x N) is unread when beta == 0."""
    a = stored_matrix(A, order, K if trans_a == TRANS else M, M if trans_a == TRANS else K, lda)
    b = stored_matrix(B, order, N if trans_b == TRANS else K, K if trans_b == TRANS else N, ldb)
    op_a = np.ascontiguousarray(a.T) if trans_a == TRANS else a
    op_b = np.ascontiguousarray(b.T) if trans_b == TRANS else b
    c0 = stored_matrix(C, order, M, N, ldc) if beta != 0.0 else None
    return gemm(op_a, op_b, alpha=alpha, beta=beta, C0=c0, nthreads=nthreads)


def _f64(a):
    a = np.asarray(a)
    if a.dtype != np.float64:
        raise TypeError("oracle expects float64 inputs, got %s" % a.dtype)
    if a.ndim == 2 and a.size > 0 and a.shape[1] > 1 and a.strides[1] != 8:
        raise ValueError("rows must be contiguous")
    return a


def dgemm(A, B, alpha=1.0, beta=0.0, C0=None, nthreads=0, absolute=False):
    """alpha*A@B + beta*C0 for binary64 A, B, C0 in double-double, rounded
    once (C0 unread when beta == 0); absolute=True gives the componentwise
    denominator |alpha||A||B| + |beta||C0| instead."""
    A, B = _f64(A), _f64(B)
    M, K = A.shape
    K2, N = B.shape
    assert K == K2
    out = np.empty((M, N), dtype=np.float64)
    c0, ldc0 = None, max(1, N)
    if beta != 0.0:
        C0 = _f64(C0)
        assert C0.shape == (M, N)
        c0, ldc0 = C0, _ld(C0, N)
    _load().orc_dgemm(M, N, K, float(alpha), _p(A), _ld(A, K), _p(B), _ld(B, N), float(beta),
                      _p(c0), ldc0, _p(out), 1 if absolute else 0, int(nthreads))
    return out


def bf16_rne(x: float) -> float:
    return float(_load().orc_bf16_rne(ctypes.c_float(x)))


def split_bf16x3(x):
    """Return (a0, a1, a2) float32 arrays holding the bfloat16 split planes."""
    x = np.ascontiguousarray(_f32(x))
    p = [np.empty_like(x) for _ in range(3)]
    _load().orc_split_bf16x3(x.size, _p(x), _p(p[0]), _p(p[1]), _p(p[2]))
    return tuple(p)


def gemm_bf16_split(A, B, n_products=3, alpha=1.0, beta=0.0, C0=None, nthreads=0):
    """Exact binary64 sum of the selected bfloat16 split products."""
    A, B = _f32(A), _f32(B)
    M, K = A.shape
    _, N = B.shape
    out = np.empty((M, N), dtype=np.float64)
    c0, ldc0 = None, max(1, N)
    if beta != 0.0:
        C0 = _f32(C0)
        c0, ldc0 = C0, _ld(C0, N)
    _load().orc_gemm_bf16_split(M, N, K, float(alpha), _p(A), _ld(A, K), _p(B), _ld(B, N),
                                float(beta), _p(c0), ldc0, int(n_products), _p(out),
                                int(nthreads))
    return out


def e4m3_value(code: int) -> float:
    return float(_load().orc_e4m3_value(ctypes.c_uint8(code)))


def e4m3_decode(codes):
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    out = np.empty(codes.shape, dtype=np.float32)
    _load().orc_e4m3_decode(codes.size, _p(codes), _p(out))
    return out


def e4m3_encode(x):
    x = np.ascontiguousarray(_f32(x))
    out = np.empty(x.shape, dtype=np.uint8)
    _load().orc_e4m3_encode(x.size, _p(x), _p(out))
    return out


def fp8_scales_rows(A):
    A = _f32(A)
    M, K = A.shape
    s = np.empty(M, dtype=np.float32)
    _load().orc_fp8_scales_rows(M, K, _p(A), _ld(A, K), _p(s))
    return s


def fp8_scales_cols(B):
    B = _f32(B)
    K, N = B.shape
    s = np.empty(N, dtype=np.float32)
    _load().orc_fp8_scales_cols(K, N, _p(B), _ld(B, N), _p(s))
    return s


def fp8_quantize_rows(A, s):
    A = _f32(A)
    M, K = A.shape
    s = np.ascontiguousarray(s, dtype=np.float32)
    q = np.empty((M, K), dtype=np.uint8)
    _load().orc_fp8_quantize_rows(M, K, _p(A), _ld(A, K), _p(s), _p(q))
    return q


def fp8_quantize_cols(B, s):
    B = _f32(B)
    K, N = B.shape
    s = np.ascontiguousarray(s, dtype=np.float32)
    q = np.empty((K, N), dtype=np.uint8)
    _load().orc_fp8_quantize_cols(K, N, _p(B), _ld(B, N), _p(s), _p(q))
    return q


def gemm_fp8_dequant(qa, sa, qb, sb, alpha=1.0, beta=0.0, C0=None, nthreads=0):
    qa = np.ascontiguousarray(qa, dtype=np.uint8)
    qb = np.ascontiguousarray(qb, dtype=np.uint8)
    sa = np.ascontiguousarray(sa, dtype=np.float32)
    sb = np.ascontiguousarray(sb, dtype=np.float32)
    M, K = qa.shape
    _, N = qb.shape
    out = np.empty((M, N), dtype=np.float64)
    c0, ldc0 = None, max(1, N)
    if beta != 0.0:
        C0 = _f32(C0)
        c0, ldc0 = C0, _ld(C0, N)
    _load().orc_gemm_fp8_dequant(M, N, K, float(alpha), _p(qa), _p(sa), _p(qb), _p(sb),
                                 float(beta), _p(c0), ldc0, _p(out), int(nthreads))
    return out


def norms(C, Cref, den=None):
    """(rel_fro, sum_sq_err, sum_sq_ref, max_componentwise) in binary64."""
    C = _f32(C)
    M, N = C.shape
    Cref = np.ascontiguousarray(Cref, dtype=np.float64)
    assert Cref.shape == (M, N)
    if den is not None:
        den = np.ascontiguousarray(den, dtype=np.float64)
    out = np.zeros(4, dtype=np.float64)
    _load().orc_norms(M, N, _p(C), _ld(C, N), _p(Cref), _p(den), _p(out))
    return tuple(float(v) for v in out)


def rel_fro(C, Cref) -> float:
    return norms(C, Cref)[0]
