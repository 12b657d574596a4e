"""Parity of the plain FP32 vector-ALU path against the FP64 oracle."""
import numpy as np
import pytest

import oracle
import seeded_inputs as si
from gpu_util import dev_matrix, gamma, sample_rows

pytestmark = pytest.mark.gpu

SHAPES = [
    (256, 256, 256),      # the small square workload
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
]


def _run(mm, M, N, K, alpha, beta, seed, cfg=None, lds=(None, None, None)):
    import torch
    A = si.uniform((M, K), seed)
    B = si.uniform((K, N), seed + 1)
    C0 = si.uniform((M, N), seed + 2)
    _, dA = dev_matrix(A, lds[0])
    _, dB = dev_matrix(B, lds[1])
    cbuf, dC = dev_matrix(C0, lds[2], pad=-7.0)
    lda, ldb, ldc = dA.stride(0), dB.stride(0), dC.stride(0)
    if cfg is None:
        mm.gemm_f32(M, N, K, alpha, dA, lda, dB, ldb, beta, dC, ldc)
    else:
        mm.gemm_run_config(mm.PATH_F32, cfg, M, N, K, alpha, dA, lda, dB, ldb, beta, dC, ldc)
    torch.cuda.synchronize()
    return A, B, C0, cbuf.cpu().numpy(), dC.cpu().numpy()


def _check(A, B, C0, C, alpha, beta):
    ref = oracle.gemm(A, B, alpha=alpha, beta=beta, C0=C0)
    den = oracle.gemm_abs(A, B, alpha=alpha, beta=beta, C0=C0)
    rel, _, _, cw = oracle.norms(C, ref, den)
    K = A.shape[1]
    assert rel <= 1e-5, rel
    assert cw <= gamma(K), (cw, gamma(K))
    return rel


@pytest.mark.parametrize("M,N,K", SHAPES)
@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (1.5, 0.5)])
def test_parity_shapes(M, N, K, alpha, beta):
    import paper_1902_10345_amd as mm
    A, B, C0, _, C = _run(mm, M, N, K, alpha, beta, seed=M * 7 + N * 3 + K)
    _check(A, B, C0, C, alpha, beta)


def test_every_config():
    import paper_1902_10345_amd as mm
    M, N, K = 300, 260, 130
    for cfg in range(mm.gemm_num_configs(mm.PATH_F32)):
        A, B, C0, _, C = _run(mm, M, N, K, 1.5, 0.5, seed=11, cfg=cfg)
        _check(A, B, C0, C, 1.5, 0.5)


def test_every_config_integer_inputs_are_exact():
    """Vector-ALU and FP32 matrix-core tiles alike: integer inputs in [-8, 8]
    keep every partial sum an integer below 2^24, so each configuration is
    exact whatever its summation order."""
    import torch
    import paper_1902_10345_amd as mm
    M, N, K = 300, 260, 1000
    A, B, C0 = si.integers((M, K), 44), si.integers((K, N), 45), si.integers((M, N), 46)
    ref = oracle.gemm(A, B, alpha=2.0, beta=-1.0, C0=C0)
    for cfg in range(mm.gemm_num_configs(mm.PATH_F32)):
        dA, dB, dC = (torch.from_numpy(x).cuda() for x in (A, B, C0))
        mm.gemm_run_config(mm.PATH_F32, cfg, M, N, K, 2.0, dA, K, dB, N, -1.0, dC, N)
        torch.cuda.synchronize()
        assert np.array_equal(dC.cpu().numpy().astype(np.float64), ref), mm.gemm_config_name(0, cfg)


def test_padded_leading_dimensions_and_untouched_padding():
    import paper_1902_10345_amd as mm
    M, N, K = 133, 97, 71
    A, B, C0, cbuf, C = _run(mm, M, N, K, 1.5, 0.5, seed=21, lds=(76, 100, 104))
    _check(A, B, C0, C, 1.5, 0.5)
    assert np.all(cbuf[:, N:] == -7.0)


def test_unaligned_pointers_take_scalar_path():
    import torch
    import paper_1902_10345_amd as mm
    M, N, K = 70, 45, 37
    A = si.uniform((M, K), 31)
    B = si.uniform((K, N), 32)
    dA = torch.from_numpy(np.concatenate([[0.0], A.ravel()]).astype(np.float32)).cuda()[1:]
    dB = torch.from_numpy(B).cuda()
    dC = torch.empty(M * N + 1, dtype=torch.float32, device="cuda")[1:]
    mm.gemm_f32(M, N, K, 1.0, dA, K, dB, N, 0.0, dC, N)
    torch.cuda.synchronize()
    _check(A, B, None, dC.cpu().numpy().reshape(M, N), 1.0, 0.0)


def test_integer_inputs_are_exact():
    import torch
    import paper_1902_10345_amd as mm
    M, N, K = 200, 150, 1000
    A = si.integers((M, K), 41)
    B = si.integers((K, N), 42)
    C0 = si.integers((M, N), 43)
    dA, dB, dC = (torch.from_numpy(x).cuda() for x in (A, B, C0))
    mm.gemm_f32(M, N, K, 2.0, dA, K, dB, N, -1.0, dC, N)
    torch.cuda.synchronize()
    ref = oracle.gemm(A, B, alpha=2.0, beta=-1.0, C0=C0)
    assert np.array_equal(dC.cpu().numpy().astype(np.float64), ref)


def test_identity_and_permutation_are_exact():
    import torch
    import paper_1902_10345_amd as mm
    A = si.uniform((96, 160), 51)
    I = np.eye(160, dtype=np.float32)
    perm = np.random.default_rng(5).permutation(96)
    P = np.zeros((96, 96), dtype=np.float32)
    P[np.arange(96), perm] = 1.0
    dA, dI, dP = (torch.from_numpy(x).cuda() for x in (A, I, P))
    dC = torch.empty((96, 160), device="cuda")
    mm.gemm_f32(96, 160, 160, 1.0, dA, 160, dI, 160, 0.0, dC, 160)
    torch.cuda.synchronize()
    assert np.array_equal(dC.cpu().numpy(), A)
    mm.gemm_f32(96, 160, 96, 1.0, dP, 96, dA, 160, 0.0, dC, 160)
    torch.cuda.synchronize()
    assert np.array_equal(dC.cpu().numpy(), A[perm])


def test_beta_zero_ignores_nan_in_c():
    import torch
    import paper_1902_10345_amd as mm
    M, N, K = 50, 60, 70
    A, B = si.uniform((M, K), 61), si.uniform((K, N), 62)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    dC = torch.full((M, N), float("nan"), device="cuda")
    mm.gemm_f32(M, N, K, 1.0, dA, K, dB, N, 0.0, dC, N)
    torch.cuda.synchronize()
    _check(A, B, None, dC.cpu().numpy(), 1.0, 0.0)


@pytest.mark.parametrize("alpha,K", [(0.0, 50), (1.0, 0)])
def test_beta_only_quick_path(alpha, K):
    import torch
    import paper_1902_10345_amd as mm
    M, N = 40, 30
    C0 = si.uniform((M, N), 71)
    dC = torch.from_numpy(C0).cuda()
    dA = torch.full((M, max(K, 1)), float("nan"), device="cuda")
    dB = torch.full((max(K, 1), N), float("nan"), device="cuda")
    mm.gemm_f32(M, N, K, alpha, dA, max(K, 1), dB, N, 0.5, dC, N)
    torch.cuda.synchronize()
    assert np.array_equal(dC.cpu().numpy(), (np.float32(0.5) * C0).astype(np.float32))
    mm.gemm_f32(M, N, K, alpha, dA, max(K, 1), dB, N, 0.0, dC, N)
    torch.cuda.synchronize()
    assert np.all(dC.cpu().numpy() == 0.0)


def test_deterministic():
    import paper_1902_10345_amd as mm
    r1 = _run(mm, 300, 200, 500, 1.5, 0.5, seed=81)[4]
    r2 = _run(mm, 300, 200, 500, 1.5, 0.5, seed=81)[4]
    assert np.array_equal(r1, r2)


@pytest.mark.parametrize("M,N,K,seed", [(4096, 4096, 4096, 2), (8192, 2048, 4096, 3)])
def test_full_size_sampled_rows(M, N, K, seed):
    """The paper-scale workloads, alpha = 1.5, beta = 0.5, in the launch the
    benchmark times; 48 seeded rows are checked against the oracle."""
    import torch
    import paper_1902_10345_amd as mm
    A = si.uniform((M, K), seed)
    B = si.uniform((K, N), seed + 100)
    C0 = si.uniform((M, N), seed + 200)
    dA, dB, dC = (torch.from_numpy(x).cuda() for x in (A, B, C0))
    mm.gemm_f32(M, N, K, 1.5, dA, K, dB, N, 0.5, dC, N)
    torch.cuda.synchronize()
    rows = sample_rows(M, 48, seed)
    C = dC.cpu().numpy()[rows]
    _check(A[rows], B, C0[rows], C, 1.5, 0.5)


def test_err_norm_matches_oracle():
    import torch
    import paper_1902_10345_amd as mm
    M, N = 300, 257
    C = si.uniform((M, N), 91)
    R = si.uniform((M, N), 92).astype(np.float64)
    D = np.abs(si.uniform((M, N), 93)).astype(np.float64) + 0.5
    got = mm.ops.err_norm(torch.from_numpy(C).cuda(), torch.from_numpy(R).cuda(),
                          torch.from_numpy(D).cuda())
    exp = oracle.norms(C, R, D)
    for g, e in zip(got[:3], exp[:3]):
        assert abs(g - e) <= 1e-12 * abs(e)
    assert got[3] == exp[3]
    got2 = mm.ops.err_norm(torch.from_numpy(C).cuda(), torch.from_numpy(R).cuda())
    assert got2[3] == oracle.norms(C, R)[3]
