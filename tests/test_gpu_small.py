"""Small-product configurations (one tile per workgroup, k split over its
eight waves, ordered sum through LDS): parity of every small configuration of
the plain and the split-precision paths against the FP64 oracle, on shapes
that span several tiles, ragged edges in M, N and K, K below one k-step per
wave, padded leading dimensions (padding never written), beta == 0 with NaN
in C, and transposed operands through gemm_ex."""
import numpy as np
import pytest

import oracle
import seeded_inputs as si
from gpu_util import check_split_result, dev_matrix, gamma

pytestmark = pytest.mark.gpu

SHAPES = [
    (256, 256, 256),   # the small square workload
    (1, 1, 1),
    (33, 65, 17),
    (100, 70, 333),
    (64, 64, 4096),    # many k-steps per wave
    (130, 31, 7),      # K below one k-step: only wave 0 works
    (97, 129, 130),    # K % 4 == 2: element loads
]


def _configs(mm, path):
    out = []
    for cfg in range(mm.gemm_num_configs(path)):
        name = mm.gemm_config_name(path, cfg)
        if "small" in name:
            out.append((cfg, name))
    assert len(out) == (2 if path == mm.PATH_F32 else 4), out
    return out


def _products(name):
    return 6 if name.endswith("_p6") else 3


def _run(mm, path, cfg, M, N, K, alpha, beta, seed, lds=(None, None, None)):
    n = _products(mm.gemm_config_name(path, cfg))
    import torch
    A = si.uniform((M, K), seed)
    B = si.uniform((K, N), seed + 1)
    C0 = si.uniform((M, N), seed + 2)
    _, dA = dev_matrix(A, lds[0])
    _, dB = dev_matrix(B, lds[1])
    cbuf, dC = dev_matrix(C0 if beta != 0 else np.full_like(C0, np.nan), lds[2], pad=-7.0)
    mm.gemm_run_config(path, cfg, M, N, K, alpha, dA, dA.stride(0), dB, dB.stride(0), beta,
                       dC, dC.stride(0), n_products=n)
    torch.cuda.synchronize()
    return A, B, C0, cbuf.cpu().numpy(), dC.cpu().numpy()


def _check_f32(A, B, C0, C, alpha, beta):
    ref = oracle.gemm(A, B, alpha=alpha, beta=beta, C0=C0)
    den = oracle.gemm_abs(A, B, alpha=alpha, beta=beta, C0=C0)
    rel, _, _, cw = oracle.norms(C, ref, den)
    assert cw <= gamma(A.shape[1]), (cw, gamma(A.shape[1]))
    assert rel <= 1e-5, rel


@pytest.mark.parametrize("M,N,K", SHAPES)
@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (1.5, 0.5)])
def test_f32_small_configs(M, N, K, alpha, beta):
    import paper_1902_10345_amd as mm
    for cfg, name in _configs(mm, mm.PATH_F32):
        print("f32 %s %dx%dx%d" % (name, M, N, K), flush=True)
        A, B, C0, _, C = _run(mm, mm.PATH_F32, cfg, M, N, K, alpha, beta, seed=M + 3 * N + K)
        _check_f32(A, B, C0 if beta != 0 else None, C, alpha, beta)


@pytest.mark.parametrize("M,N,K", SHAPES)
@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (1.5, 0.5)])
def test_split_small_configs(M, N, K, alpha, beta):
    import paper_1902_10345_amd as mm
    for cfg, name in _configs(mm, mm.PATH_3XBF16):
        print("3xbf16 %s %dx%dx%d" % (name, M, N, K), flush=True)
        A, B, C0, _, C = _run(mm, mm.PATH_3XBF16, cfg, M, N, K, alpha, beta, seed=M + 5 * N + K)
        check_split_result(oracle, A, B, C0 if beta != 0 else None, C, alpha, beta,
                           _products(name))


def test_padding_untouched_and_integer_exact():
    """Integer inputs in [-8, 8]: every partial sum (per wave and over the
    waves) is an integer below 2^24, so each configuration is exact; the
    padding of C's rows keeps its value."""
    import torch
    import paper_1902_10345_amd as mm
    M, N, K = 75, 90, 1000
    A, B, C0 = si.integers((M, K), 7), si.integers((K, N), 8), si.integers((M, N), 9)
    ref = oracle.gemm(A, B, alpha=2.0, beta=-1.0, C0=C0)
    for path in (mm.PATH_F32, mm.PATH_3XBF16):
        for cfg, name in _configs(mm, path):
            _, dA = dev_matrix(A, K + 3)
            _, dB = dev_matrix(B, N + 5)
            cbuf, dC = dev_matrix(C0, N + 7, pad=-7.0)
            mm.gemm_run_config(path, cfg, M, N, K, 2.0, dA, K + 3, dB, N + 5, -1.0, dC, N + 7,
                               n_products=_products(name))
            torch.cuda.synchronize()
            assert np.array_equal(dC.cpu().numpy(), ref.astype(np.float32)), name
            assert (cbuf.cpu().numpy()[:, N:] == -7.0).all(), name


def test_deterministic_and_equal_to_ordered_sum_of_chunks():
    """Two runs give the same bits; with K within one k-step only wave 0
    contributes, and the result equals the 32 x 32 and 64 x 64 tiles'
    (same single-chunk reduction) bit for bit."""
    import torch
    import paper_1902_10345_amd as mm
    for path in (mm.PATH_F32, mm.PATH_3XBF16):
        cfgs = [c for c, n in _configs(mm, path) if not n.endswith("_p6")]
        M, N, K = 200, 150, 777
        outs = []
        for cfg in cfgs:
            for _ in range(2):
                _, _, _, _, C = _run(mm, path, cfg, M, N, K, 1.0, 0.0, seed=3)
                outs.append(C)
        assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[2], outs[3])
        K = 8 if path == mm.PATH_F32 else 16
        one = [_run(mm, path, cfg, M, N, K, 1.0, 0.0, seed=4)[4] for cfg in cfgs]
        assert np.array_equal(one[0], one[1])


@pytest.mark.parametrize("ta,tb", [(True, False), (False, True), (True, True)])
def test_transposed_operands_on_small_shapes(ta, tb):
    """gemm_ex with transposed operands at 256^3 (the library routes this size
    to a small configuration) against the oracle on the logical operands."""
    import torch
    import paper_1902_10345_amd as mm
    M, N, K = 256, 192, 320
    A = si.uniform((M, K), 21)
    B = si.uniform((K, N), 22)
    C0 = si.uniform((M, N), 23)
    for path, n in ((mm.PATH_F32, 0), (mm.PATH_3XBF16, 3)):
        sa = np.ascontiguousarray(A.T) if ta else A
        sb = np.ascontiguousarray(B.T) if tb else B
        dA, dB = torch.from_numpy(sa).cuda(), torch.from_numpy(sb).cuda()
        dC = torch.from_numpy(C0).cuda()
        mm.gemm_ex(mm.ROW_MAJOR, mm.TRANS if ta else mm.NO_TRANS, mm.TRANS if tb else mm.NO_TRANS,
                   M, N, K, 1.5, dA, sa.shape[1], dB, sb.shape[1], 0.5, dC, N, path, n)
        torch.cuda.synchronize()
        C = dC.cpu().numpy()
        if path == mm.PATH_F32:
            _check_f32(A, B, C0, C, 1.5, 0.5)
        else:
            check_split_result(oracle, A, B, C0, C, 1.5, 0.5, 3)
