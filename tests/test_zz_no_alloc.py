"""The no-allocation split-K entry point (gemm_f32_3xbf16_splitk_noalloc),
called through the C-ABI, against the workspace entry point
(gemm_f32_3xbf16_splitk): bitwise equal results (same kernels, same split
count) on calls in a row, each later one smaller than the first, and within
the split-precision bounds of the oracle; a split count whose partial
planes exceed the fixed scratch is refused before anything is enqueued."""
import ctypes

import numpy as np
import pytest

import oracle
import seeded_inputs as si
from gpu_util import check_split_result

F = ctypes.c_void_p(16)  # a non-null dummy pointer; never dereferenced on rejection


def test_scratch_bound_is_refused_before_the_device():
    import paper_1902_10345_amd as mm
    lim = mm.NOALLOC_SCRATCH_BYTES
    assert lim == 64 << 20
    # two planes of 2048 x 4097 floats: 16 KiB beyond the scratch
    assert 2 * 2048 * 4097 * 4 > lim
    st = mm.lib.gemm_f32_3xbf16_splitk_noalloc(2048, 4097, 8192, 1.0, F, 8192, F, 4097, 0.0, F,
                                               4097, 3, 2, None)
    assert st == mm.STATUS_NO_MEMORY
    assert "GEMM_NOALLOC_SCRATCH_BYTES" in mm.gemm_last_error()
    # argument codes follow the workspace entry point's numbering
    assert mm.lib.gemm_f32_3xbf16_splitk_noalloc(64, 64, 64, 1.0, F, 64, F, 64, 0.0, F, 64, 4, 2,
                                                 None) == -12
    assert mm.lib.gemm_f32_3xbf16_splitk_noalloc(64, 64, 64, 1.0, F, 64, F, 64, 0.0, F, 64, 3, 65,
                                                 None) == -13
    assert mm.lib.gemm_f32_3xbf16_splitk_noalloc(64, 64, 64, 1.0, F, 63, F, 64, 0.0, F, 64, 3, 2,
                                                 None) == -6


def _pair(mm, torch, M, N, K, n, splits, seed, check_oracle=True):
    A, B, C0 = si.uniform((M, K), seed), si.uniform((K, N), seed + 100), si.uniform((M, N), seed + 200)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    want, got = torch.from_numpy(C0).cuda(), torch.from_numpy(C0).cuda()
    wsb = mm.gemm_splitk_workspace_bytes(M, N, K, splits)
    ws = torch.empty(max(wsb, 256), dtype=torch.uint8, device="cuda")
    print("noalloc %dx%dx%d n=%d splits=%d (%d scratch bytes)" % (M, N, K, n, splits, wsb),
          flush=True)
    mm.gemm_f32_3xbf16_splitk(M, N, K, 1.5, dA, K, dB, N, 0.5, want, N, n, splits, ws, wsb)
    st = mm.lib.gemm_f32_3xbf16_splitk_noalloc(M, N, K, 1.5, mm.ptr(dA), K, mm.ptr(dB), N, 0.5,
                                               mm.ptr(got), N, n, splits, mm.stream_handle())
    assert st == 0, mm.gemm_last_error()
    torch.cuda.synchronize()
    C = got.cpu().numpy()
    assert np.array_equal(C, want.cpu().numpy())
    if check_oracle:
        check_split_result(oracle, A, B, C0, C, 1.5, 0.5, n)


@pytest.mark.gpu
def test_noalloc_equals_the_workspace_entry_point_on_calls_in_a_row():
    import torch
    import paper_1902_10345_amd as mm
    # eight planes, then a smaller product with three: the second call reads
    # only planes it wrote itself
    _pair(mm, torch, 300, 260, 2000, 3, 8, 61)
    _pair(mm, torch, 100, 90, 700, 3, 3, 62)
    # six products and the default split count of a skinny product (16 planes)
    M, N, K = 64, 1024, 4096
    assert mm.gemm_splitk_default_splits(M, N, K) > 1
    _pair(mm, torch, M, N, K, 6, 0, 63)
    # partial planes filling the scratch exactly (2 x 2048 x 4096 floats)
    assert 2 * 2048 * 4096 * 4 == mm.NOALLOC_SCRATCH_BYTES
    _pair(mm, torch, 2048, 4096, 512, 3, 2, 64, check_oracle=False)
    # a split count that resolves to one pass uses no scratch at all
    _pair(mm, torch, 70, 50, 40, 3, 1, 65)
