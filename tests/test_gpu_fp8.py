"""Scaled FP8 (OCP E4M3) path: the encoder and quantiser bit for bit against
the oracle's, the matrix-core product against the dequantised-input oracle at
binary32-accumulation level, and the end-to-end error against the exact
product (the quantisation error itself)."""
import math

import numpy as np
import pytest

import oracle
import seeded_inputs as si
from gpu_util import fp8_check, fp8_group_term, gamma, sample_rows

pytestmark = pytest.mark.gpu


def test_encoder_is_bitwise_the_oracle_encoder():
    import torch
    import paper_1902_10345_amd as mm
    g = np.random.default_rng(8)
    vals = np.array([oracle.e4m3_value(c) for c in range(127)], dtype=np.float64)
    mids = (vals[:-1] + vals[1:]) / 2
    x = np.concatenate([
        g.uniform(-500, 500, 200000).astype(np.float32),
        (g.standard_normal(200000) * 0.05).astype(np.float32),
        (g.standard_normal(20000) * 1e-3).astype(np.float32),
        vals.astype(np.float32), -vals.astype(np.float32),
        mids.astype(np.float32), -mids.astype(np.float32),
        np.nextafter(mids.astype(np.float32), np.float32(np.inf)),
        np.nextafter(mids.astype(np.float32), np.float32(-np.inf)),
        np.array([0.0, -0.0, 448.0, -448.0, 464.0, -464.0, 463.99, 1e30, -1e30, 1e-40, -1e-40,
                  np.inf, -np.inf, np.nan], dtype=np.float32),
    ]).astype(np.float32)
    dx = torch.from_numpy(x).cuda()
    codes = torch.empty(x.size, dtype=torch.uint8, device="cuda")
    mm.fp8_e4m3_encode(x.size, dx, codes)
    torch.cuda.synchronize()
    got = codes.cpu().numpy()
    ref = oracle.e4m3_encode(x)
    bad = np.nonzero(got != ref)[0]
    assert bad.size == 0, [(float(x[i]), hex(got[i]), hex(ref[i])) for i in bad[:8]]


def _quantize(mm, A, B, lda=None):
    import torch
    M, K = A.shape
    _, N = B.shape
    nbytes = mm.gemm_fp8_workspace_bytes(M, N, K)
    ws = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    dA = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    dB = torch.from_numpy(B).cuda()
    mm.fp8_quantize(M, N, K, dA, K, dB, N, ws, nbytes)
    torch.cuda.synchronize()
    L = mm.fp8_workspace_layout(M, N, K)
    h = ws.cpu().numpy()
    Kp = L["Kp"]
    qa = h[L["qa"]:L["qa"] + M * Kp].reshape(M, Kp)
    qbT = h[L["qb"]:L["qb"] + N * Kp].reshape(N, Kp)
    sa = h[L["sa"]:L["sa"] + 4 * M].view(np.float32)
    sb = h[L["sb"]:L["sb"] + 4 * N].view(np.float32)
    return ws, nbytes, qa, qbT, sa, sb, Kp


@pytest.mark.parametrize("M,N,K,outliers", [(96, 80, 200, "none"), (257, 130, 1000, "A"),
                                            (64, 300, 129, "B"), (1, 1, 1, "none"),
                                            (70, 50, 450, "A"), (33, 40, 1500, "B"),
                                            (6, 9, 4097, "none")])
def test_quantiser_is_bitwise_the_oracle(M, N, K, outliers):
    import paper_1902_10345_amd as mm
    A, B, _ = si.fp8_workload(M, N, K, seed=M + N + K, outliers=outliers)
    A[0, :] = 0.0  # an all-zero row takes scale 1
    _, _, qa, qbT, sa, sb, Kp = _quantize(mm, A, B)
    rsa, rsb = oracle.fp8_scales_rows(A), oracle.fp8_scales_cols(B)
    assert np.array_equal(sa, rsa) and np.array_equal(sb, rsb)
    assert sa[0] == 1.0
    assert np.array_equal(qa[:, :K], oracle.fp8_quantize_rows(A, rsa))
    assert np.array_equal(qbT[:, :K].T, oracle.fp8_quantize_cols(B, rsb))
    assert not qa[:, K:].any() and not qbT[:, K:].any()


@pytest.mark.parametrize("K", [1024, 1025, 2048, 3072, 3073, 4096, 4100])
def test_column_quantiser_register_blocks_are_bitwise_the_oracle(K):
    """The one-pass column quantiser (a stripe of 16 columns held in
    registers, up to 4096 padded rows in blocks of 1024) at the edges of its
    row blocks, a partial last stripe (N = 37) and columns of A-transposed
    shape; K = 4100 takes the two-pass path."""
    import paper_1902_10345_amd as mm
    M, N = 5, 37
    A, B, _ = si.fp8_workload(M, N, K, seed=K, outliers="B")
    B[K - 1, 36] = np.float32(-3.5e3)  # the last row of the last column sets its scale
    _, _, qa, qbT, sa, sb, Kp = _quantize(mm, A, B)
    rsb = oracle.fp8_scales_cols(B)
    assert np.array_equal(sb, rsb)
    assert np.array_equal(qbT[:, :K].T, oracle.fp8_quantize_cols(B, rsb))
    assert not qbT[:, K:].any()


@pytest.mark.parametrize("M,N,K", [(40, 36, 200), (40, 36, 1000), (12, 20, 9000)])
def test_quantiser_special_values_are_bitwise_the_oracle(M, N, K):
    """Rows and columns with NaN, infinities, signed zeros and scales of
    2^-70 and 2^70 (outside the range where the quotient is formed from the
    reciprocal) next to ordinary ones: every code and scale as the oracle's.
    K = 200, 1000 and 9000 reach the three row-quantiser shapes."""
    import paper_1902_10345_amd as mm
    g = np.random.default_rng(K + 1)
    A = g.standard_normal((M, K)).astype(np.float32)
    B = g.standard_normal((K, N)).astype(np.float32)
    A[1] *= np.float32(2.0 ** -70)
    A[2] *= np.float32(2.0 ** 70)
    A[3, 5] = np.nan
    A[4, 7] = np.inf
    A[5, ::3] = -0.0
    A[6] = 0.0
    A[6, 0] = -0.0
    A[7] *= np.float32(2.0 ** -58)
    A[8, -1] = -np.nan
    B[:, 1] *= np.float32(2.0 ** -70)
    B[:, 2] *= np.float32(2.0 ** 70)
    B[9, 3] = np.nan
    B[4, 4] = -np.inf
    B[::2, 5] = -0.0
    B[:, 6] *= np.float32(2.0 ** 58)
    _, _, qa, qbT, sa, sb, Kp = _quantize(mm, A, B)
    rsa, rsb = oracle.fp8_scales_rows(A), oracle.fp8_scales_cols(B)
    assert np.array_equal(sa, rsa) and np.array_equal(sb, rsb)
    assert np.array_equal(qa[:, :K], oracle.fp8_quantize_rows(A, rsa))
    assert np.array_equal(qbT[:, :K].T, oracle.fp8_quantize_cols(B, rsb))
    assert not qa[:, K:].any() and not qbT[:, K:].any()


@pytest.mark.parametrize("M,N,K", [(300, 260, 1000), (40, 700, 300), (3, 2000, 64)])
def test_quantiser_reused_workspace(M, N, K):
    """Two quantisations into one workspace, the second with values 1e6 times
    smaller: the column maxima of the first must not survive into the second
    (the column scratch is cleared by the row launch of A, or by its own
    launch when A's grid is too small: M = 3, N = 2000)."""
    import torch
    import paper_1902_10345_amd as mm
    nbytes = mm.gemm_fp8_workspace_bytes(M, N, K)
    ws = torch.full((nbytes,), 0xFF, dtype=torch.uint8, device="cuda")
    g = np.random.default_rng(M + N)
    L = mm.fp8_workspace_layout(M, N, K)
    for scale in (1e3, 1e-3):
        A = (g.standard_normal((M, K)) * scale).astype(np.float32)
        B = (g.standard_normal((K, N)) * scale).astype(np.float32)
        dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
        mm.fp8_quantize(M, N, K, dA, K, dB, N, ws, nbytes)
        torch.cuda.synchronize()
        h = ws.cpu().numpy()
        Kp = L["Kp"]
        sa = h[L["sa"]:L["sa"] + 4 * M].view(np.float32)
        sb = h[L["sb"]:L["sb"] + 4 * N].view(np.float32)
        qbT = h[L["qb"]:L["qb"] + N * Kp].reshape(N, Kp)
        rsa, rsb = oracle.fp8_scales_rows(A), oracle.fp8_scales_cols(B)
        assert np.array_equal(sa, rsa) and np.array_equal(sb, rsb)
        assert np.array_equal(qbT[:, :K].T, oracle.fp8_quantize_cols(B, rsb))


@pytest.mark.parametrize("M,N,K", [(256, 256, 256), (300, 520, 130), (1, 77, 300), (130, 1, 64),
                                   (513, 257, 1000), (64, 64, 1)])
@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (1.5, 0.5)])
def test_product_matches_dequantised_oracle(M, N, K, alpha, beta):
    import torch
    import paper_1902_10345_amd as mm
    A, B, C0 = si.fp8_workload(M, N, K, seed=3 * M + N + K)
    ws, nbytes, qa, qbT, sa, sb, Kp = _quantize(mm, A, B)
    dC = torch.from_numpy(C0).cuda()
    mm.gemm_fp8_prequantized(M, N, K, alpha, ws, nbytes, beta, dC, N)
    torch.cuda.synchronize()
    C = dC.cpu().numpy()
    qb = np.ascontiguousarray(qbT[:, :K].T)
    rel, ratio, cw = fp8_check(oracle, C, qa[:, :K], qb, sa, sb, alpha, beta, C0)
    print("fp8 %dx%dx%d vs dequantised oracle: rel_fro %.2e, componentwise %.2f gamma_K, "
          "%.3f of the bound" % (M, N, K, rel, cw / gamma(K, extra=4), ratio))
    assert ratio <= 1.0, ratio


@pytest.mark.parametrize("outliers", ["none", "A", "B"])
def test_end_to_end_error_is_the_quantisation_error(outliers):
    """gemm_fp8_scaled against the exact product: the relative Frobenius and
    componentwise (|A||B|-relative) errors stay within the E4M3 quantisation
    error (about 4e-2 and 4e-3..3e-2 for these inputs)."""
    import torch
    import paper_1902_10345_amd as mm
    M, N, K = 256, 256, 1024
    A, B, C0 = si.fp8_workload(M, N, K, seed=4, outliers=outliers)
    dA, dB, dC = (torch.from_numpy(x).cuda() for x in (A, B, C0))
    nbytes = mm.gemm_fp8_workspace_bytes(M, N, K)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    mm.gemm_fp8_scaled(M, N, K, 1.5, dA, K, dB, N, 0.5, dC, N, ws, nbytes)
    torch.cuda.synchronize()
    C = dC.cpu().numpy()
    ref = oracle.gemm(A, B, alpha=1.5, beta=0.5, C0=C0)
    den = oracle.gemm_abs(A, B, alpha=1.5, beta=0.5, C0=C0)
    rel, _, _, cw = oracle.norms(C, ref, den)
    print("fp8 outliers=%s rel_fro=%.3e componentwise=%.3e" % (outliers, rel, cw))
    assert rel <= 0.08
    assert cw <= 0.08


def test_full_size_sampled_rows():
    """The 4096^3 workload with A-column outliers, in the launch the benchmark
    times: sampled rows against the dequantised oracle and the exact one."""
    import torch
    import paper_1902_10345_amd as mm
    M = N = K = 4096
    A, B, C0 = si.fp8_workload(M, N, K, seed=4, outliers="A")
    dA, dB, dC = (torch.from_numpy(x).cuda() for x in (A, B, C0))
    nbytes = mm.gemm_fp8_workspace_bytes(M, N, K)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    mm.gemm_fp8_scaled(M, N, K, 1.5, dA, K, dB, N, 0.5, dC, N, ws, nbytes)
    torch.cuda.synchronize()
    L = mm.fp8_workspace_layout(M, N, K)
    h = ws.cpu().numpy()
    Kp = L["Kp"]
    rows = sample_rows(M, 16, 4)
    qa = h[L["qa"]:L["qa"] + M * Kp].reshape(M, Kp)[rows, :K]
    qb = np.ascontiguousarray(h[L["qb"]:L["qb"] + N * Kp].reshape(N, Kp)[:, :K].T)
    sa = h[L["sa"]:L["sa"] + 4 * M].view(np.float32)[rows]
    sb = h[L["sb"]:L["sb"] + 4 * N].view(np.float32)
    C = dC.cpu().numpy()[rows]
    assert fp8_check(oracle, C, qa, qb, sa, sb, 1.5, 0.5, C0[rows])[1] <= 1.0
    exact = oracle.gemm(A[rows], B, alpha=1.5, beta=0.5, C0=C0[rows])
    assert oracle.rel_fro(C, exact) <= 0.08


@pytest.mark.parametrize("M,N,K", [(300, 520, 130), (513, 257, 1000), (256, 512, 384)])
def test_every_config_matches_dequantised_oracle(M, N, K):
    """Each FP8 tile configuration (register-staged and direct-to-LDS) through
    gemm_run_config, which quantises into the workspace and multiplies."""
    import torch
    import paper_1902_10345_amd as mm
    A, B, C0 = si.fp8_workload(M, N, K, seed=M + 2 * N + K, outliers="A")
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    nbytes = mm.gemm_fp8_workspace_bytes(M, N, K)
    L = mm.fp8_workspace_layout(M, N, K)
    Kp = L["Kp"]
    for cfg in range(mm.gemm_num_configs(mm.PATH_FP8)):
        ws = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
        dC = torch.from_numpy(C0).cuda()
        mm.gemm_run_config(mm.PATH_FP8, cfg, M, N, K, 1.5, dA, K, dB, N, 0.5, dC, N,
                           workspace=ws, ws_bytes=nbytes)
        torch.cuda.synchronize()
        h = ws.cpu().numpy()
        qa = h[L["qa"]:L["qa"] + M * Kp].reshape(M, Kp)
        qbT = h[L["qb"]:L["qb"] + N * Kp].reshape(N, Kp)
        sa = h[L["sa"]:L["sa"] + 4 * M].view(np.float32)
        sb = h[L["sb"]:L["sb"] + 4 * N].view(np.float32)
        qb = np.ascontiguousarray(qbT[:, :K].T)
        ratio = fp8_check(oracle, dC.cpu().numpy(), qa[:, :K], qb, sa, sb, 1.5, 0.5, C0)[1]
        assert ratio <= 1.0, (mm.gemm_config_name(mm.PATH_FP8, cfg), ratio)


def _workspace_from_codes(mm, qa, qb, sa, sb):
    """A workspace holding the given codes (qa: M x K, qb: K x N) and scales."""
    import torch
    M, K = qa.shape
    N = qb.shape[1]
    L = mm.fp8_workspace_layout(M, N, K)
    Kp = L["Kp"]
    nbytes = mm.gemm_fp8_workspace_bytes(M, N, K)
    h = np.zeros(nbytes, np.uint8)
    pa = np.zeros((M, Kp), np.uint8)
    pa[:, :K] = qa
    pb = np.zeros((N, Kp), np.uint8)
    pb[:, :K] = qb.T
    h[L["qa"]:L["qa"] + M * Kp] = pa.ravel()
    h[L["qb"]:L["qb"] + N * Kp] = pb.ravel()
    h[L["sa"]:L["sa"] + 4 * M] = sa.astype(np.float32).view(np.uint8)
    h[L["sb"]:L["sb"] + 4 * N] = sb.astype(np.float32).view(np.uint8)
    return torch.from_numpy(h).cuda(), nbytes


@pytest.mark.parametrize("M,N,K", [(300, 520, 130), (64, 64, 1000), (257, 33, 64)])
def test_integer_codes_are_exact(M, N, K):
    """Codes of integers in [-8, 8] with unit scales: every product is an
    integer of magnitude <= 64 and every partial sum an integer below 2^24, so
    the result is exact whatever the summation order and the group rounding."""
    import torch
    import paper_1902_10345_amd as mm
    g = np.random.default_rng(M + N + K)
    IA = g.integers(-8, 9, size=(M, K))
    IB = g.integers(-8, 9, size=(K, N))
    qa = oracle.e4m3_encode(IA.astype(np.float32))
    qb = oracle.e4m3_encode(IB.astype(np.float32))
    assert np.array_equal(oracle.e4m3_decode(qa), IA) and np.array_equal(oracle.e4m3_decode(qb), IB)
    ws, nbytes = _workspace_from_codes(mm, qa, qb, np.ones(M), np.ones(N))
    for cfg in range(mm.gemm_num_configs(mm.PATH_FP8)):
        dC = torch.full((M, N), float("nan"), device="cuda")
        mm.gemm_run_config(mm.PATH_FP8_PREQUANTIZED, cfg, M, N, K, 1.0, None, 0, None, 0, 0.0,
                           dC, N, workspace=ws, ws_bytes=nbytes)
        torch.cuda.synchronize()
        assert np.array_equal(dC.cpu().numpy().astype(np.int64), IA @ IB), cfg


# Hand-built rows of products (b = 1 at every k, unit scales): (k, a_k) pairs.
_S5, _S6 = 2.0 ** -5, 2.0 ** -6
_GROUP_CASES = [
    [(0, 448.0)] + [(k, _S6) for k in range(1, 8)],    # seven lost in one group
    [(0, 448.0)] + [(k, _S6) for k in range(8, 15)],   # same seven, next group: exact
    [(0, 448.0)] + [(k, _S5) for k in range(1, 8)],    # on the grid: exact
    [(0, 448.0), (1, _S6)], [(0, 448.0), (7, _S6)], [(0, 448.0), (8, _S6)],
    [(0, 448.0), (63, _S6)], [(0, 448.0), (64, _S6)],
    [(0, 448.0), (1, 3 * _S6)],                        # truncated to one grid step
    [(0, 448.0), (1, -_S6)], [(0, -448.0), (1, _S6)],  # toward zero, either sign
    [(0, _S6), (1, 448.0)], [(7, 448.0)] + [(k, _S6) for k in range(7)],
    [(0, 448.0), (1, 448.0), (2, _S6)],                # grid of the largest product
    [(0, 16.0), (1, 2.0 ** -9)], [(0, 1.0), (1, 2.0 ** -9)],
]


def _group_model(row, K):
    """The matrix core's sum of one row of products as measured on gfx950:
    within each group of eight consecutive k (k = 8g .. 8g + 7) every product
    is truncated toward zero to a multiple of 2^(E - 13), E = floor(log2) of
    the group's largest |product|, the truncated products are summed exactly,
    and the group sums are accumulated in binary32 (exact for these cases)."""
    a = np.zeros(K)
    for k, v in row:
        a[k] = v
    total = 0.0
    for g in range(0, K, 8):
        p = a[g:g + 8]
        big = np.abs(p).max()
        if big == 0:
            continue
        step = 2.0 ** (math.floor(math.log2(big)) - 13)
        total += float(np.sum(np.trunc(p / step) * step))
    return total


def test_group_products_truncate_toward_zero_on_the_group_grid():
    """Pins the model behind the FP8 bound (fp8_group_term) with hand-built
    codes, unit scales, N = 1, K = 128, on every configuration: the result of
    each row equals _group_model bit for bit.  Under that model each group of
    eight loses less than one grid step 2^(E - 13) on each of at most seven
    products, i.e. less than 7 * 2^-13 of the product of the group's maxima,
    which is the bound's group term; the cases' errors are checked against it
    too."""
    import torch
    import paper_1902_10345_amd as mm
    M, K = len(_GROUP_CASES), 128
    qa = np.zeros((M, K), np.uint8)
    for r, row in enumerate(_GROUP_CASES):
        for k, v in row:
            qa[r, k] = oracle.e4m3_encode(np.array([v], np.float32))[0]
            assert float(oracle.e4m3_decode(qa[r:r + 1, k:k + 1])[0, 0]) == v
    one = oracle.e4m3_encode(np.array([1.0], np.float32))[0]
    qb = np.full((K, 1), one, np.uint8)
    ws, nbytes = _workspace_from_codes(mm, qa, qb, np.ones(M), np.ones(1))
    model = np.array([_group_model(row, K) for row in _GROUP_CASES])
    exact = np.array([sum(v for _, v in row) for row in _GROUP_CASES])
    term = fp8_group_term(qa, qb, np.ones(M, np.float32), np.ones(1, np.float32), 1.0)[:, 0]
    assert np.all(np.abs(model - exact) <= term), (model - exact, term)
    assert model[0] == 448.0 and model[1] == exact[1] and model[2] == exact[2]
    for cfg in range(mm.gemm_num_configs(mm.PATH_FP8)):
        dC = torch.full((M, 1), float("nan"), device="cuda")
        mm.gemm_run_config(mm.PATH_FP8_PREQUANTIZED, cfg, M, 1, K, 1.0, None, 0, None, 0, 0.0,
                           dC, 1, workspace=ws, ws_bytes=nbytes)
        torch.cuda.synchronize()
        got = dC.cpu().numpy()[:, 0].astype(np.float64)
        print(mm.gemm_config_name(mm.PATH_FP8, cfg), "got - model:", got - model)
        assert np.array_equal(got, model), (cfg, got - model)
