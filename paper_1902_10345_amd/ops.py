"""Tensor-level helpers over the C entry points (argument marshalling only).

Tensors are torch tensors on a GPU.  C must have unit column stride (row-major
rows, any row stride >= number of columns); A and B may be row-major the same
way or column-major (unit row stride, e.g. a transposed view), which is passed
to the library as a transposed operand.
"""
from __future__ import annotations

from . import _lib


def _ld(t, cols):
    if t.dim() != 2:
        raise ValueError("expected a 2-D tensor")
    if t.shape[1] > 1 and t.stride(1) != 1:
        raise ValueError("rows must be contiguous (stride(1) == 1)")
    return max(int(t.stride(0)), max(1, cols)) if t.shape[0] > 1 else max(1, cols)


def _operand(t, rows, cols):
    """(transposed, ld) of a 2-D operand that is row- or column-contiguous."""
    if t.dim() != 2:
        raise ValueError("expected a 2-D tensor")
    if cols <= 1 or t.stride(1) == 1:
        return False, _ld(t, cols)
    if rows <= 1 or t.stride(0) == 1:
        # column-major storage: the transpose of a row-major (cols x rows) matrix
        return True, max(int(t.stride(1)), max(1, rows)) if cols > 1 else max(1, rows)
    raise ValueError("operand is neither row- nor column-contiguous")


def gemm(A, B, C=None, alpha=1.0, beta=0.0, path="f32", n_products=3, workspace=None,
         stream=None):
    """C <- alpha*A@B + beta*C on the chosen path ("f32", "3xbf16", "fp8"; float64
    tensors always run the binary64 path); allocates C (uninitialised is fine
    when beta == 0) if not given.  A and B may be transposed views."""
    import torch
    M, K = A.shape
    K2, N = B.shape
    if K != K2:
        raise ValueError("inner dimensions differ: %d vs %d" % (K, K2))
    dtype = torch.float64 if A.dtype == torch.float64 else torch.float32
    if C is None:
        C = torch.empty((M, N), dtype=dtype, device=A.device)
    ldc = _ld(C, N)
    if dtype == torch.float64:
        lda, ldb = _ld(A, K), _ld(B, N)
        _lib.gemm_f64(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, stream)
        return C
    ta, lda = _operand(A, M, K)
    tb, ldb = _operand(B, K, N)
    codes = {"f32": _lib.PATH_F32, "3xbf16": _lib.PATH_3XBF16, "fp8": _lib.PATH_FP8}
    if path not in codes:
        raise ValueError("unknown path %r" % path)
    if not ta and not tb:
        if path == "f32":
            _lib.gemm_f32(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, stream)
            return C
        if path == "3xbf16":
            _lib.gemm_f32_3xbf16(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, n_products, stream)
            return C
    nbytes = 0
    if path == "fp8":
        nbytes = _lib.gemm_fp8_workspace_bytes(M, N, K)
        if workspace is None:
            workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=A.device)
        nbytes = workspace.numel()
    _lib.gemm_ex(_lib.ROW_MAJOR, _lib.TRANS if ta else _lib.NO_TRANS,
                 _lib.TRANS if tb else _lib.NO_TRANS, M, N, K, alpha, A, lda, B, ldb, beta, C,
                 ldc, codes[path], n_products, workspace if path == "fp8" else None, nbytes,
                 stream)
    return C


def err_norm(C, Cref, den=None, stream=None):
    """(rel_fro, sum_sq_err, sum_sq_ref, max_ratio) computed on the GPU in FP64."""
    import torch
    M, N = C.shape
    out = torch.zeros(4, dtype=torch.float64, device=C.device)
    ws = torch.empty(_lib.err_norm_workspace_bytes(), dtype=torch.uint8, device=C.device)
    _lib.err_norm_f64(M, N, C, _ld(C, N), Cref.contiguous(),
                      None if den is None else den.contiguous(), out, ws, ws.numel(), stream)
    return tuple(float(v) for v in out.cpu())
