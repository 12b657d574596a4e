"""Parity of the FP32-accurate split-precision (3xBF16 / 6xBF16) MFMA path
against the FP64 oracle, and of its staging split against the oracle's
bfloat16 split."""
import numpy as np
import pytest

import oracle
import seeded_inputs as si
from gpu_util import check_split_result, dev_matrix, sample_rows

pytestmark = pytest.mark.gpu

SHAPES = [
    (256, 256, 256),
    (1, 1, 1),
    (15, 17, 255),
    (257, 255, 17),
    (130, 200, 300),
    (513, 129, 1000),
    (64, 64, 64),
    (1, 300, 40),
    (300, 1, 40),
    (77, 33, 1),
    (129, 131, 33),
    (300, 520, 100),
]


def _run(mm, M, N, K, alpha, beta, n, seed, cfg=None, lds=(None, None, None)):
    import torch
    A = si.uniform((M, K), seed)
    B = si.uniform((K, N), seed + 1)
    C0 = si.uniform((M, N), seed + 2)
    _, dA = dev_matrix(A, lds[0])
    _, dB = dev_matrix(B, lds[1])
    cbuf, dC = dev_matrix(C0, lds[2], pad=-7.0)
    lda, ldb, ldc = dA.stride(0), dB.stride(0), dC.stride(0)
    if cfg is None:
        mm.gemm_f32_3xbf16(M, N, K, alpha, dA, lda, dB, ldb, beta, dC, ldc, n)
    else:
        mm.gemm_run_config(mm.PATH_3XBF16, cfg, M, N, K, alpha, dA, lda, dB, ldb, beta, dC, ldc,
                           n_products=n)
    torch.cuda.synchronize()
    return A, B, C0, cbuf.cpu().numpy(), dC.cpu().numpy()


def _check(A, B, C0, C, alpha, beta, n):
    return check_split_result(oracle, A, B, C0, C, alpha, beta, n)


def test_staging_split_is_bitwise_the_oracle_split():
    import torch
    import paper_1902_10345_amd as mm
    g = np.random.default_rng(3)
    x = np.concatenate([
        si.uniform((1, 100000), 1).ravel(),
        (g.standard_normal(100000) * 1e3).astype(np.float32),
        (g.standard_normal(1000) * 1e-30).astype(np.float32),
        (np.arange(1, 20001, dtype=np.uint32) << 16 | 0x8000).view(np.float32),
        np.array([0.0, -0.0, 1.0, 255.0, 257.0, 3.38e38, -3.38e38], dtype=np.float32),
    ]).astype(np.float32)
    # Domain of the split: |x| below the largest bfloat16 value plus half an
    # ulp (2^128 * (1 - 2^-9)); larger magnitudes round the leading plane to inf.
    x = x[np.isfinite(x) & (np.abs(x) < np.float32(2.0 ** 128 * (1 - 2.0 ** -9)))]
    dx = torch.from_numpy(x).cuda()
    planes = [torch.empty(x.size, dtype=torch.int16, device="cuda") for _ in range(3)]
    mm.split_bf16x3(x.size, dx, planes[0], planes[1], planes[2])
    torch.cuda.synchronize()
    ref = oracle.split_bf16x3(x)
    for level, (p, r) in enumerate(zip(planes, ref)):
        bits = p.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
        got = bits.view(np.float32)
        bad = np.nonzero(got != r)[0]
        assert bad.size == 0, (level, bad.size, [(float(x[i]).hex(), float(got[i]).hex(),
                                                  float(r[i]).hex()) for i in bad[:5]])


@pytest.mark.parametrize("n", [3, 6])
@pytest.mark.parametrize("M,N,K", SHAPES)
@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (1.5, 0.5)])
def test_parity_shapes(M, N, K, alpha, beta, n):
    import paper_1902_10345_amd as mm
    A, B, C0, _, C = _run(mm, M, N, K, alpha, beta, n, seed=M * 7 + N * 3 + K)
    _check(A, B, C0, C, alpha, beta, n)


def test_every_config():
    import paper_1902_10345_amd as mm
    M, N, K = 300, 520, 130
    for cfg in range(mm.gemm_num_configs(mm.PATH_3XBF16)):
        n = 3 if "_p3" in mm.gemm_config_name(mm.PATH_3XBF16, cfg) else 6
        A, B, C0, _, C = _run(mm, M, N, K, 1.5, 0.5, n, seed=11, cfg=cfg)
        _check(A, B, C0, C, 1.5, 0.5, n)


@pytest.mark.parametrize("K", [16, 32, 48, 64, 80, 130, 1000])
def test_ring_config_every_slab_count_parity(K):
    """The 256 x 256 x 16 tile with a ring of three LDS stages: one to four
    slabs (prologue only, one loop pass, loop plus odd tail), a partial first
    slab, ragged M and N edges."""
    import paper_1902_10345_amd as mm
    cfg = [c for c in range(mm.gemm_num_configs(mm.PATH_3XBF16))
           if mm.gemm_config_name(mm.PATH_3XBF16, c) == "bx3_256x256x16_8w128x64_p3_ring3"][0]
    M, N = 300, 520
    A, B, C0, _, C = _run(mm, M, N, K, 1.5, 0.5, 3, seed=K + 5, cfg=cfg)
    _check(A, B, C0, C, 1.5, 0.5, 3)


@pytest.mark.parametrize("K", [2, 16, 34, 130, 1000, 2048])
def test_two_group_config_parity(K):
    """The 128 x 128 tile with its k range split between two groups of four
    waves: partial first slabs in each half, ragged M and N; an odd K is
    refused (no equal halves)."""
    import paper_1902_10345_amd as mm
    cfg = [c for c in range(mm.gemm_num_configs(mm.PATH_3XBF16))
           if mm.gemm_config_name(mm.PATH_3XBF16, c) == "bx3_128x128x16_2x4w64x64_p3_kg2"][0]
    M, N = 300, 260
    A, B, C0, _, C = _run(mm, M, N, K, 1.5, 0.5, 3, seed=K + 9, cfg=cfg)
    _check(A, B, C0, C, 1.5, 0.5, 3)
    with pytest.raises(mm.GemmError) as e:
        _run(mm, M, N, 7, 1.5, 0.5, 3, seed=1, cfg=cfg)
    assert e.value.status == mm.STATUS_UNSUPPORTED


def test_mismatched_products_for_config_is_rejected():
    import paper_1902_10345_amd as mm
    cfg6 = [c for c in range(mm.gemm_num_configs(mm.PATH_3XBF16))
            if "_p6" in mm.gemm_config_name(mm.PATH_3XBF16, c)][0]
    with pytest.raises(mm.GemmError) as e:
        mm.gemm_run_config(mm.PATH_3XBF16, cfg6, 4, 4, 4, 1.0, 16, 4, 16, 4, 0.0, 16, 4,
                           n_products=3)
    assert e.value.status == -14


@pytest.mark.parametrize("n", [3, 6])
def test_padded_leading_dimensions_and_untouched_padding(n):
    import paper_1902_10345_amd as mm
    M, N, K = 133, 97, 71
    A, B, C0, cbuf, C = _run(mm, M, N, K, 1.5, 0.5, n, seed=21, lds=(76, 100, 104))
    _check(A, B, C0, C, 1.5, 0.5, n)
    assert np.all(cbuf[:, N:] == -7.0)


def test_unaligned_a_takes_scalar_path():
    import torch
    import paper_1902_10345_amd as mm
    M, N, K = 70, 45, 37
    A = si.uniform((M, K), 31)
    B = si.uniform((K, N), 32)
    dA = torch.from_numpy(np.concatenate([[0.0], A.ravel()]).astype(np.float32)).cuda()[1:]
    dB = torch.from_numpy(B).cuda()
    dC = torch.empty((M, N), dtype=torch.float32, device="cuda")
    mm.gemm_f32_3xbf16(M, N, K, 1.0, dA, K, dB, N, 0.0, dC, N, 3)
    torch.cuda.synchronize()
    _check(A, B, None, dC.cpu().numpy(), 1.0, 0.0, 3)


@pytest.mark.parametrize("n", [3, 6])
def test_integer_inputs_are_exact(n):
    import torch
    import paper_1902_10345_amd as mm
    M, N, K = 200, 150, 1000
    A = si.integers((M, K), 41)
    B = si.integers((K, N), 42)
    C0 = si.integers((M, N), 43)
    dA, dB, dC = (torch.from_numpy(x).cuda() for x in (A, B, C0))
    mm.gemm_f32_3xbf16(M, N, K, 2.0, dA, K, dB, N, -1.0, dC, N, n)
    torch.cuda.synchronize()
    ref = oracle.gemm(A, B, alpha=2.0, beta=-1.0, C0=C0)
    assert np.array_equal(dC.cpu().numpy().astype(np.float64), ref)


def test_identity_and_permutation_exact_with_six_products():
    import torch
    import paper_1902_10345_amd as mm
    A = si.uniform((96, 160), 51)
    I = np.eye(160, dtype=np.float32)
    perm = np.random.default_rng(5).permutation(96)
    P = np.zeros((96, 96), dtype=np.float32)
    P[np.arange(96), perm] = 1.0
    dA, dI, dP = (torch.from_numpy(x).cuda() for x in (A, I, P))
    dC = torch.empty((96, 160), device="cuda")
    mm.gemm_f32_3xbf16(96, 160, 160, 1.0, dA, 160, dI, 160, 0.0, dC, 160, 6)
    torch.cuda.synchronize()
    assert np.array_equal(dC.cpu().numpy(), A)
    mm.gemm_f32_3xbf16(96, 160, 96, 1.0, dP, 96, dA, 160, 0.0, dC, 160, 6)
    torch.cuda.synchronize()
    assert np.array_equal(dC.cpu().numpy(), A[perm])
    # with three products the identity is reproduced only to ~2^-16 relative
    mm.gemm_f32_3xbf16(96, 160, 160, 1.0, dA, 160, dI, 160, 0.0, dC, 160, 3)
    torch.cuda.synchronize()
    d = np.abs(dC.cpu().numpy().astype(np.float64) - A)
    assert np.all(d <= 2.0 ** -16 * np.abs(A))


def test_beta_zero_ignores_nan_in_c():
    import torch
    import paper_1902_10345_amd as mm
    M, N, K = 50, 60, 70
    A, B = si.uniform((M, K), 61), si.uniform((K, N), 62)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    dC = torch.full((M, N), float("nan"), device="cuda")
    mm.gemm_f32_3xbf16(M, N, K, 1.0, dA, K, dB, N, 0.0, dC, N, 3)
    torch.cuda.synchronize()
    _check(A, B, None, dC.cpu().numpy(), 1.0, 0.0, 3)


def test_deterministic():
    import paper_1902_10345_amd as mm
    r1 = _run(mm, 300, 200, 500, 1.5, 0.5, 3, seed=81)[4]
    r2 = _run(mm, 300, 200, 500, 1.5, 0.5, 3, seed=81)[4]
    assert np.array_equal(r1, r2)


@pytest.mark.parametrize("n", [3, 6])
@pytest.mark.parametrize("M,N,K,seed", [(4096, 4096, 4096, 2), (8192, 2048, 4096, 3)])
def test_full_size_sampled_rows(M, N, K, seed, n):
    import torch
    import paper_1902_10345_amd as mm
    A = si.uniform((M, K), seed)
    B = si.uniform((K, N), seed + 100)
    C0 = si.uniform((M, N), seed + 200)
    dA, dB, dC = (torch.from_numpy(x).cuda() for x in (A, B, C0))
    mm.gemm_f32_3xbf16(M, N, K, 1.5, dA, K, dB, N, 0.5, dC, N, n)
    torch.cuda.synchronize()
    rows = sample_rows(M, 32, seed)
    C = dC.cpu().numpy()[rows]
    rel = _check(A[rows], B, C0[rows], C, 1.5, 0.5, n)
    print("n=%d %dx%dx%d sampled rel_fro %.3e" % (n, M, N, K, rel))
