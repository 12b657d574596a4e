"""Split-K form of the split-precision path: chunks of the k reduction run as
separate workgroups and their partial products are summed in chunk order (a
write-conflict resolution by ordered sum).  Parity against the FP64 oracle,
bitwise equality with the one-pass kernel for one chunk, determinism."""
import numpy as np
import pytest

import oracle
import seeded_inputs as si
from gpu_util import check_split_result, dev_matrix, sample_rows

pytestmark = pytest.mark.gpu

ONE_PASS_CFG = {3: "bx3_128x128x16_4w64x64_p3", 6: "bx3_128x128x32_4w64x64_p6"}


def _cfg_index(mm, name):
    for c in range(mm.gemm_num_configs(mm.PATH_3XBF16)):
        if mm.gemm_config_name(mm.PATH_3XBF16, c) == name:
            return c
    raise AssertionError(name)


def _run(mm, A, B, C0, alpha, beta, n, splits, lds=(None, None, None), c_fill=None):
    import torch
    M, K = A.shape
    N = B.shape[1]
    _, dA = dev_matrix(A, lds[0])
    _, dB = dev_matrix(B, lds[1])
    cbuf, dC = dev_matrix(C0, lds[2], pad=-7.0)
    if c_fill is not None:
        dC.fill_(c_fill)
    nb = mm.gemm_splitk_workspace_bytes(M, N, K, splits)
    ws = torch.empty(max(nb, 256), dtype=torch.uint8, device="cuda")
    mm.gemm_f32_3xbf16_splitk(M, N, K, alpha, dA, dA.stride(0), dB, dB.stride(0), beta, dC,
                              dC.stride(0), n, splits, ws, nb)
    torch.cuda.synchronize()
    return cbuf.cpu().numpy(), dC.cpu().numpy()


@pytest.mark.parametrize("M,N,K,splits", [
    (130, 200, 1000, 2), (257, 129, 777, 3), (64, 300, 4096, 16), (1, 1, 512, 4),
    (300, 1, 1000, 7), (129, 131, 40, 64), (512, 512, 2048, 0), (33, 65, 3001, 5),
])
@pytest.mark.parametrize("n", [3, 6])
def test_parity(M, N, K, splits, n):
    import paper_1902_10345_amd as mm
    seed = M * 7 + N * 3 + K + splits
    A, B, C0 = si.uniform((M, K), seed), si.uniform((K, N), seed + 1), si.uniform((M, N), seed + 2)
    _, C = _run(mm, A, B, C0, 1.5, 0.5, n, splits)
    check_split_result(oracle, A, B, C0, C, 1.5, 0.5, n)


def test_padded_leading_dimensions_and_untouched_padding():
    import paper_1902_10345_amd as mm
    M, N, K = 133, 97, 1071
    A, B, C0 = si.uniform((M, K), 5), si.uniform((K, N), 6), si.uniform((M, N), 7)
    cbuf, C = _run(mm, A, B, C0, 1.5, 0.5, 3, 4, lds=(1076, 100, 104))
    check_split_result(oracle, A, B, C0, C, 1.5, 0.5, 3)
    assert np.all(cbuf[:, N:] == -7.0)


def test_beta_zero_ignores_nan_in_c():
    import paper_1902_10345_amd as mm
    M, N, K = 200, 150, 1200
    A, B = si.uniform((M, K), 11), si.uniform((K, N), 12)
    _, C = _run(mm, A, B, np.zeros((M, N), np.float32), 1.0, 0.0, 3, 3, c_fill=float("nan"))
    check_split_result(oracle, A, B, None, C, 1.0, 0.0, 3)


def test_integer_inputs_are_exact():
    import paper_1902_10345_amd as mm
    M, N, K = 150, 260, 2000
    A, B, C0 = si.integers((M, K), 21), si.integers((K, N), 22), si.integers((M, N), 23)
    for n in (3, 6):
        _, C = _run(mm, A, B, C0, 2.0, -1.0, n, 5)
        assert np.array_equal(C.astype(np.float64), oracle.gemm(A, B, alpha=2.0, beta=-1.0, C0=C0))


@pytest.mark.parametrize("n", [3, 6])
def test_one_chunk_equals_the_one_pass_kernel_bitwise(n):
    import torch
    import paper_1902_10345_amd as mm
    M, N, K = 300, 260, 700
    A, B, C0 = si.uniform((M, K), 31), si.uniform((K, N), 32), si.uniform((M, N), 33)
    _, C1 = _run(mm, A, B, C0, 1.5, 0.5, n, 1)
    dA, dB, dC = (torch.from_numpy(x).cuda() for x in (A, B, C0))
    mm.gemm_run_config(mm.PATH_3XBF16, _cfg_index(mm, ONE_PASS_CFG[n]), M, N, K, 1.5, dA, K, dB, N,
                       0.5, dC, N, n_products=n)
    torch.cuda.synchronize()
    assert np.array_equal(C1, dC.cpu().numpy())


def test_deterministic_and_split_count_changes_only_rounding():
    import paper_1902_10345_amd as mm
    M, N, K = 257, 300, 3000
    A, B, C0 = si.uniform((M, K), 41), si.uniform((K, N), 42), si.uniform((M, N), 43)
    _, C4a = _run(mm, A, B, C0, 1.5, 0.5, 3, 4)
    _, C4b = _run(mm, A, B, C0, 1.5, 0.5, 3, 4)
    assert np.array_equal(C4a, C4b)
    _, C7 = _run(mm, A, B, C0, 1.5, 0.5, 3, 7)
    check_split_result(oracle, A, B, C0, C7, 1.5, 0.5, 3)


def test_more_splits_than_slabs():
    """64 requested chunks of a 200-deep reduction: 13 slabs of 16 hold work,
    the rest are never launched; the workspace request is still for 64."""
    import paper_1902_10345_amd as mm
    M, N, K = 100, 90, 200
    A, B, C0 = si.uniform((M, K), 51), si.uniform((K, N), 52), si.uniform((M, N), 53)
    _, C = _run(mm, A, B, C0, 1.5, 0.5, 3, 64)
    check_split_result(oracle, A, B, C0, C, 1.5, 0.5, 3)


@pytest.mark.parametrize("M,N,K,seed", [(512, 4096, 4096, 8), (64, 4096, 4096, 9)])
def test_full_size_sampled_rows(M, N, K, seed):
    """The machine-underfilling shapes the benchmark times (one GPU's share of
    the 4096^3 product under eight-way row sharding, and a skinny product),
    default split count; 32 seeded rows against the oracle."""
    import torch
    import paper_1902_10345_amd as mm
    A, B, C0 = si.uniform((M, K), seed), si.uniform((K, N), seed + 100), si.uniform((M, N), seed + 200)
    dA, dB, dC = (torch.from_numpy(x).cuda() for x in (A, B, C0))
    nb = mm.gemm_splitk_workspace_bytes(M, N, K, 0)
    ws = torch.empty(max(nb, 256), dtype=torch.uint8, device="cuda")
    mm.gemm_f32_3xbf16_splitk(M, N, K, 1.5, dA, K, dB, N, 0.5, dC, N, 3, 0, ws, nb)
    torch.cuda.synchronize()
    rows = sample_rows(M, 32, seed)
    check_split_result(oracle, A[rows], B, C0[rows], dC.cpu().numpy()[rows], 1.5, 0.5, 3)
