"""Batched-strided binary32 products (gemm_strided_batched) on the FP32
matrix-core path and the split-precision path: every problem of the batch
against the FP64 oracle, problems placed back to back with gaps (the gaps
never written), a shared operand (zero stride), bit equality with the
single-problem entry points, exact integer batches beyond one launch."""
import numpy as np
import pytest

import oracle
import seeded_inputs as si
from gpu_util import check_split_result, gamma

pytestmark = pytest.mark.gpu


def _check_f32(A, B, C0, C, alpha, beta):
    ref = oracle.gemm(A, B, alpha=alpha, beta=beta, C0=C0)
    den = oracle.gemm_abs(A, B, alpha=alpha, beta=beta, C0=C0)
    cw = oracle.norms(C, ref, den)[3]
    assert cw <= gamma(A.shape[1]), (cw, gamma(A.shape[1]))


def _run(mm, path, n, M, N, K, batch, seed, pad=(0, 0, 0), share_b=False, alpha=1.5, beta=0.5):
    import torch
    g = np.random.default_rng(seed)
    sa, sb, sc = M * K + pad[0], (0 if share_b else K * N + pad[1]), M * N + pad[2]
    hA = g.uniform(-1, 1, size=batch * sa).astype(np.float32)
    hB = g.uniform(-1, 1, size=batch * sb if sb else K * N).astype(np.float32)
    hC = g.uniform(-1, 1, size=batch * sc).astype(np.float32)
    dA, dB, dC = (torch.from_numpy(x).cuda() for x in (hA, hB, hC))
    mm.gemm_strided_batched(path, M, N, K, alpha, dA, K, sa, dB, N, sb, beta, dC, N, sc, batch, n)
    torch.cuda.synchronize()
    out = dC.cpu().numpy()
    for b in range(batch):
        A = hA[b * sa:b * sa + M * K].reshape(M, K)
        B = hB[b * sb:b * sb + K * N].reshape(K, N)
        C0 = hC[b * sc:b * sc + M * N].reshape(M, N)
        C = out[b * sc:b * sc + M * N].reshape(M, N)
        if path == mm.PATH_3XBF16:
            check_split_result(oracle, A, B, C0, C, alpha, beta, n)
        else:
            _check_f32(A, B, C0, C, alpha, beta)
        assert np.array_equal(out[b * sc + M * N:(b + 1) * sc], hC[b * sc + M * N:(b + 1) * sc])


CASES = [(16, 16, 16, 100), (32, 32, 32, 37), (12, 12, 12, 50), (64, 64, 64, 11),
         (70, 50, 90, 9), (130, 129, 64, 3), (1, 1, 5, 7), (33, 17, 40, 13)]


@pytest.mark.parametrize("M,N,K,batch", CASES)
@pytest.mark.parametrize("n", [3, 6])
def test_split_path_parity(M, N, K, batch, n):
    import paper_1902_10345_amd as mm
    _run(mm, mm.PATH_3XBF16, n, M, N, K, batch, M + 7 * N + K + batch)
    _run(mm, mm.PATH_3XBF16, n, M, N, K, batch, M + N + K + batch + 1, pad=(3, 5, 7))


@pytest.mark.parametrize("M,N,K,batch", CASES)
def test_f32_path_parity(M, N, K, batch):
    import paper_1902_10345_amd as mm
    _run(mm, mm.PATH_F32, 3, M, N, K, batch, 3 * M + N + K + batch, pad=(1, 2, 3))


def test_shared_b_and_one_problem_equals_the_single_gemm():
    import torch
    import paper_1902_10345_amd as mm
    _run(mm, mm.PATH_3XBF16, 3, 40, 24, 33, 20, 5, share_b=True)
    M, N, K = 130, 140, 150
    A, B, C0 = si.uniform((M, K), 51), si.uniform((K, N), 52), si.uniform((M, N), 53)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    # a batch of one takes the LDS-staged tile of the batched launcher (the
    # single-GEMM default at this shape is a small-product tile, which has no
    # batched form): the same configuration through the single-GEMM call
    for n, name in ((3, "bx3_64x64x32_4w32x32_p3"), (6, "bx3_128x128x32_4w64x64_p6")):
        cfg = [c for c in range(mm.gemm_num_configs(mm.PATH_3XBF16))
               if mm.gemm_config_name(mm.PATH_3XBF16, c) == name][0]
        d1, d2 = torch.from_numpy(C0.copy()).cuda(), torch.from_numpy(C0.copy()).cuda()
        mm.gemm_run_config(mm.PATH_3XBF16, cfg, M, N, K, 1.5, dA, K, dB, N, 0.5, d1, N, n)
        mm.gemm_strided_batched(mm.PATH_3XBF16, M, N, K, 1.5, dA, K, 0, dB, N, 0, 0.5, d2, N, 0, 1, n)
        torch.cuda.synchronize()
        assert np.array_equal(d1.cpu().numpy(), d2.cpu().numpy()), n


@pytest.mark.parametrize("M,N,K", [(32, 32, 32), (17, 29, 40), (64, 64, 64), (33, 64, 7),
                                   (1, 1, 1), (64, 40, 100), (48, 16, 1000)])
@pytest.mark.parametrize("n", [1, 3, 6])
def test_small_problems_equal_the_tile_kernels_bitwise(M, N, K, n):
    """Problems with M, N <= 64 run one wave per problem with fragments
    loaded straight from memory; every element must be the same sum as in the
    LDS-staged tile of the same arithmetic (n = 1: binary32 on the FP32
    matrix cores; 3, 6: split products), run alone on the problem (gaps
    between the problems never written)."""
    import torch
    import paper_1902_10345_amd as mm
    path = mm.PATH_F32 if n == 1 else mm.PATH_3XBF16
    batch = 9
    g = np.random.default_rng(M * 1000 + N * 10 + K + n)
    sa, sb, sc = M * K + 3, K * N + 5, M * N + 7
    hA = g.uniform(-1, 1, size=batch * sa).astype(np.float32)
    hB = g.uniform(-1, 1, size=batch * sb).astype(np.float32)
    hC = g.uniform(-1, 1, size=batch * sc).astype(np.float32)
    dA, dB, dC = (torch.from_numpy(x).cuda() for x in (hA, hB, hC))
    mm.gemm_strided_batched(path, M, N, K, 1.5, dA, K, sa, dB, N, sb, 0.5, dC, N, sc, batch,
                            max(n, 3))
    torch.cuda.synchronize()
    out = dC.cpu().numpy()
    name = {1: "f32mfma_128x128x16_4w64x64", 3: "bx3_64x64x32_4w32x32_p3",
            6: "bx3_128x128x32_4w64x64_p6"}[n]
    cfg = [c for c in range(mm.gemm_num_configs(path)) if mm.gemm_config_name(path, c) == name][0]
    for b in range(batch):
        A = dA[b * sa:b * sa + M * K]
        B = dB[b * sb:b * sb + K * N]
        solo = torch.from_numpy(hC[b * sc:b * sc + M * N].copy()).cuda()
        mm.gemm_run_config(path, cfg, M, N, K, 1.5, A, K, B, N, 0.5, solo, N, max(n, 3))
        torch.cuda.synchronize()
        assert np.array_equal(out[b * sc:b * sc + M * N], solo.cpu().numpy()), b
        assert np.array_equal(out[b * sc + M * N:(b + 1) * sc], hC[b * sc + M * N:(b + 1) * sc])


@pytest.mark.parametrize("n", [1, 3, 6])
def test_small_problems_with_padded_leading_dimensions(n):
    """The one-wave-per-problem kernel with lda > K, ldb > N, ldc > N (A rows
    not 16-byte aligned), against the oracle; padding never written."""
    import torch
    import paper_1902_10345_amd as mm
    path = mm.PATH_F32 if n == 1 else mm.PATH_3XBF16
    M, N, K, batch = 30, 21, 45, 7
    lda, ldb, ldc = K + 3, N + 5, N + 2
    sa, sb, sc = M * lda + 1, K * ldb, M * ldc + 4
    g = np.random.default_rng(91 + n)
    hA = g.uniform(-1, 1, size=batch * sa).astype(np.float32)
    hB = g.uniform(-1, 1, size=batch * sb).astype(np.float32)
    hC = g.uniform(-1, 1, size=batch * sc).astype(np.float32)
    dA, dB, dC = (torch.from_numpy(x).cuda() for x in (hA, hB, hC))
    mm.gemm_strided_batched(path, M, N, K, -0.75, dA, lda, sa, dB, ldb, sb, 1.25, dC, ldc, sc,
                            batch, max(n, 3))
    torch.cuda.synchronize()
    out = dC.cpu().numpy()
    for b in range(batch):
        A = np.ascontiguousarray(hA[b * sa:b * sa + M * lda].reshape(M, lda)[:, :K])
        B = np.ascontiguousarray(hB[b * sb:b * sb + K * ldb].reshape(K, ldb)[:, :N])
        Cb = out[b * sc:b * sc + M * ldc].reshape(M, ldc)
        C0 = hC[b * sc:b * sc + M * ldc].reshape(M, ldc)
        got, c0 = np.ascontiguousarray(Cb[:, :N]), np.ascontiguousarray(C0[:, :N])
        if n == 1:
            _check_f32(A, B, c0, got, -0.75, 1.25)
        else:
            check_split_result(oracle, A, B, c0, got, -0.75, 1.25, n)
        assert np.array_equal(Cb[:, N:], C0[:, N:])
        assert np.array_equal(out[b * sc + M * ldc:(b + 1) * sc], hC[b * sc + M * ldc:(b + 1) * sc])


@pytest.mark.parametrize("n", [1, 3, 6])
def test_small_problems_beta_zero_never_read_c(n):
    """beta == 0: C is write-only, so NaN in C must not reach the result."""
    import torch
    import paper_1902_10345_amd as mm
    path = mm.PATH_F32 if n == 1 else mm.PATH_3XBF16
    M, N, K, batch = 24, 40, 33, 5
    A = si.uniform((batch * M, K), 81 + n).reshape(batch, M, K)
    B = si.uniform((batch * K, N), 82 + n).reshape(batch, K, N)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    dC = torch.full((batch, M, N), float("nan"), device="cuda")
    mm.gemm_strided_batched(path, M, N, K, 1.0, dA, K, M * K, dB, N, K * N, 0.0, dC, N, M * N,
                            batch, max(n, 3))
    torch.cuda.synchronize()
    out = dC.cpu().numpy()
    assert np.isfinite(out).all()
    for b in range(batch):
        if n == 1:
            _check_f32(A[b], B[b], None, out[b], 1.0, 0.0)
        else:
            check_split_result(oracle, A[b], B[b], None, out[b], 1.0, 0.0, n)


@pytest.mark.parametrize("path", ["f32", "3xbf16"])
def test_more_problems_than_one_launch_exact(path):
    import torch
    import paper_1902_10345_amd as mm
    code = mm.PATH_F32 if path == "f32" else mm.PATH_3XBF16
    M = N = K = 2
    batch = 65540
    g = np.random.default_rng(61)
    hA = g.integers(-9, 10, size=(batch, M, K)).astype(np.float32)
    hB = g.integers(-9, 10, size=(batch, K, N)).astype(np.float32)
    hC = g.integers(-9, 10, size=(batch, M, N)).astype(np.float32)
    dA, dB, dC = (torch.from_numpy(x).cuda() for x in (hA, hB, hC))
    mm.gemm_strided_batched(code, M, N, K, 2.0, dA, K, M * K, dB, N, K * N, -1.0, dC, N, M * N, batch, 3)
    torch.cuda.synchronize()
    want = 2.0 * np.matmul(hA.astype(np.float64), hB.astype(np.float64)) - hC
    assert np.array_equal(dC.cpu().numpy().astype(np.float64), want)


def test_quick_path_scales_every_problem():
    import torch
    import paper_1902_10345_amd as mm
    M, N, batch = 5, 6, 70000
    hC = si.uniform((batch, M * N), 71).reshape(-1)
    d = torch.from_numpy(hC.copy()).cuda()
    mm.gemm_strided_batched(mm.PATH_3XBF16, M, N, 0, 1.0, None, 1, 0, None, N, 0, 0.5, d, N, M * N,
                            batch, 3)
    torch.cuda.synchronize()
    assert np.array_equal(d.cpu().numpy(), np.float32(0.5) * hC)
