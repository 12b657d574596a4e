"""Tensor-level helpers over the C entry points (argument marshalling only).

Tensors are torch tensors on a GPU; 2-D operands must have unit column stride
(row-major rows, any row stride >= number of columns).
"""
from __future__ import annotations

from . import _lib


def _ld(t, cols):
    if t.dim() != 2:
        raise ValueError("expected a 2-D tensor")
    if t.shape[1] > 1 and t.stride(1) != 1:
        raise ValueError("rows must be contiguous (stride(1) == 1)")
    return max(int(t.stride(0)), max(1, cols)) if t.shape[0] > 1 else max(1, cols)


def gemm(A, B, C=None, alpha=1.0, beta=0.0, path="f32", n_products=3, workspace=None,
         stream=None):
    """C <- alpha*A@B + beta*C on the chosen path ("f32", "3xbf16", "fp8");
    allocates C (uninitialised is fine when beta == 0) if not given."""
    import torch
    M, K = A.shape
    K2, N = B.shape
    if K != K2:
        raise ValueError("inner dimensions differ: %d vs %d" % (K, K2))
    if C is None:
        C = torch.empty((M, N), dtype=torch.float32, device=A.device)
    lda, ldb, ldc = _ld(A, K), _ld(B, N), _ld(C, N)
    if path == "f32":
        _lib.gemm_f32(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, stream)
    elif path == "3xbf16":
        _lib.gemm_f32_3xbf16(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, n_products, stream)
    elif path == "fp8":
        nbytes = _lib.gemm_fp8_workspace_bytes(M, N, K)
        if workspace is None:
            workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=A.device)
        _lib.gemm_fp8_scaled(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, workspace,
                             workspace.numel(), stream)
    else:
        raise ValueError("unknown path %r" % path)
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
