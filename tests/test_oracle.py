"""Pins for the FP64 oracle: each test checks it against something other than
itself -- hand-computed fixtures, closed forms, exact integer arithmetic,
invariants and independent library conversions -- so that a dropped term, a
wrong index or a transposed operand in the oracle fails here."""
import itertools
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import seeded_inputs as si

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_gemm_golden():
    cases, cur = [], {}
    with open(os.path.join(GOLDEN, "gemm_small.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            if key == "M" and cur:
                cases.append(cur)
                cur = {}
            cur[key] = [float(v) for v in vals]
    cases.append(cur)
    return cases


@pytest.mark.parametrize("case", _read_gemm_golden())
def test_gemm_hand_computed(case):
    M, N, K = int(case["M"][0]), int(case["N"][0]), int(case["K"][0])
    A = np.array(case["A"], dtype=np.float32).reshape(M, K)
    B = np.array(case["B"], dtype=np.float32).reshape(K, N)
    C0 = np.array(case["C0"], dtype=np.float32).reshape(M, N)
    out = oracle.gemm(A, B, alpha=case["alpha"][0], beta=case["beta"][0], C0=C0)
    assert np.array_equal(out, np.array(case["C"]).reshape(M, N))


def test_identity_exact():
    A = si.uniform((37, 53), 11)
    I = np.eye(53, dtype=np.float32)
    assert np.array_equal(oracle.gemm(A, I), A.astype(np.float64))
    I2 = np.eye(37, dtype=np.float32)
    assert np.array_equal(oracle.gemm(I2, A), A.astype(np.float64))


def test_permutation_exact():
    A = si.uniform((29, 31), 12)
    perm = np.random.default_rng(3).permutation(29)
    P = np.zeros((29, 29), dtype=np.float32)
    P[np.arange(29), perm] = 1.0
    assert np.array_equal(oracle.gemm(P, A), A[perm].astype(np.float64))
    perm2 = np.random.default_rng(4).permutation(31)
    Q = np.zeros((31, 31), dtype=np.float32)
    Q[perm2, np.arange(31)] = 1.0
    # (A Q)[:, j] = A[:, perm2[j]]
    assert np.array_equal(oracle.gemm(A, Q), A[:, perm2].astype(np.float64))


@pytest.mark.parametrize("K", [1, 7, 64, 1000, 4096])
def test_rank1_closed_form(K):
    # A[i,k] = x_i (k+1), B[k,j] = (k+1) z_j  =>  C[i,j] = x_i z_j K(K+1)(2K+1)/6
    x = np.array([1, -2, 3, 5], dtype=np.float32)
    z = np.array([2, -1, 7], dtype=np.float32)
    kk = np.arange(1, K + 1, dtype=np.float32)
    A = np.outer(x, kk).astype(np.float32)
    B = np.outer(kk, z).astype(np.float32)
    s = K * (K + 1) * (2 * K + 1) // 6
    expect = np.outer(x.astype(np.float64), z.astype(np.float64)) * s
    assert np.array_equal(oracle.gemm(A, B), expect)


def test_integer_inputs_match_python_ints():
    A = si.integers((23, 41), 21)
    B = si.integers((41, 19), 22)
    Ai = [[int(v) for v in row] for row in A]
    Bi = [[int(v) for v in row] for row in B]
    expect = [[sum(Ai[i][k] * Bi[k][j] for k in range(41)) for j in range(19)] for i in range(23)]
    assert np.array_equal(oracle.gemm(A, B), np.array(expect, dtype=np.float64))


def test_brute_force_all_tiny_shapes():
    """Every M, N, K in 1..5 with integer entries, alpha = 1.5, beta = -0.5,
    against exact rational arithmetic."""
    g = np.random.default_rng(99)
    alpha, beta = Fraction(3, 2), Fraction(-1, 2)
    for M, N, K in itertools.product(range(1, 6), repeat=3):
        A = g.integers(-6, 7, size=(M, K)).astype(np.float32)
        B = g.integers(-6, 7, size=(K, N)).astype(np.float32)
        C0 = g.integers(-6, 7, size=(M, N)).astype(np.float32)
        out = oracle.gemm(A, B, alpha=1.5, beta=-0.5, C0=C0)
        for i in range(M):
            for j in range(N):
                s = sum(Fraction(int(A[i, k])) * Fraction(int(B[k, j])) for k in range(K))
                e = alpha * s + beta * Fraction(int(C0[i, j]))
                assert Fraction(out[i, j]) == e, (M, N, K, i, j)


def test_random_matches_float64_matmul():
    # special case that reduces to a library routine: numpy's float64 matmul
    A = si.uniform((67, 45), 31)
    B = si.uniform((45, 53), 32)
    C0 = si.uniform((67, 53), 33)
    ref = 1.5 * (A.astype(np.float64) @ B.astype(np.float64)) + 0.5 * C0.astype(np.float64)
    out = oracle.gemm(A, B, alpha=1.5, beta=0.5, C0=C0)
    assert np.max(np.abs(out - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_beta_zero_never_reads_c0():
    A = si.uniform((8, 9), 41)
    B = si.uniform((9, 10), 42)
    C0 = np.full((8, 10), np.nan, dtype=np.float32)
    out = oracle.gemm(A, B, alpha=1.0, beta=0.0, C0=C0)
    assert np.all(np.isfinite(out))


def test_alpha_zero_and_k_zero():
    C0 = si.uniform((6, 7), 43)
    A = si.uniform((6, 5), 44)
    B = si.uniform((5, 7), 45)
    out = oracle.gemm(A, B, alpha=0.0, beta=0.5, C0=C0)
    assert np.array_equal(out, 0.5 * C0.astype(np.float64))
    A0 = np.zeros((6, 0), dtype=np.float32)
    B0 = np.zeros((0, 7), dtype=np.float32)
    out = oracle.gemm(A0, B0, alpha=2.0, beta=-1.0, C0=C0)
    assert np.array_equal(out, -C0.astype(np.float64))


def test_leading_dimension_padding_is_ignored():
    A = si.uniform((13, 17), 51, ld=24, pad_value=np.nan)
    B = si.uniform((17, 11), 52, ld=16, pad_value=np.nan)
    C0 = si.uniform((13, 11), 53, ld=12, pad_value=np.nan)
    out = oracle.gemm(A, B, alpha=1.5, beta=0.5, C0=C0)
    ref = oracle.gemm(np.ascontiguousarray(A), np.ascontiguousarray(B), alpha=1.5, beta=0.5,
                      C0=np.ascontiguousarray(C0))
    assert np.all(np.isfinite(out))
    assert np.array_equal(out, ref)


def test_gemm_abs_is_componentwise_denominator():
    A = si.integers((5, 6), 61)
    B = si.integers((6, 4), 62)
    C0 = si.integers((5, 4), 63)
    out = oracle.gemm_abs(A, B, alpha=-2.0, beta=-0.5, C0=C0)
    expect = 2.0 * (np.abs(A).astype(np.int64) @ np.abs(B).astype(np.int64)) + 0.5 * np.abs(C0)
    assert np.array_equal(out, expect.astype(np.float64))


# ------------------------------------------------------------ bf16 split ---

def _read_bf16_golden():
    rows = []
    with open(os.path.join(GOLDEN, "bf16_split.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([float.fromhex(v) for v in line.split()])
    return rows


@pytest.mark.parametrize("row", _read_bf16_golden())
def test_bf16_split_hand_derived(row):
    a, a0, a1, a2 = row
    p0, p1, p2 = oracle.split_bf16x3(np.array([a], dtype=np.float32))
    assert (float(p0[0]), float(p1[0]), float(p2[0])) == (a0, a1, a2)


def test_bf16_rne_matches_torch_conversion():
    torch = pytest.importorskip("torch")
    g = np.random.default_rng(7)
    x = np.concatenate([
        si.uniform((1, 200000), 71).ravel(),
        (g.standard_normal(100000) * 1e4).astype(np.float32),
        # values with exactly-halfway low bits to exercise ties
        (np.arange(1, 50001, dtype=np.uint32) << 16 | 0x8000).view(np.float32),
    ]).astype(np.float32)
    x = x[np.isfinite(x)]
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    p0, _, _ = oracle.split_bf16x3(x)
    assert np.array_equal(p0, ref)


def test_bf16_split_last_plane_rounds_on_the_subnormal_grid():
    # r1 - a1 = 9 * 2^-134 lies below bfloat16's subnormal spacing 2^-133, so
    # the last plane rounds (9/2 -> 4, ties to even) to 2^-131.
    x = np.array([float.fromhex('0x1.7512480000000p-113')], dtype=np.float32)
    p0, p1, p2 = oracle.split_bf16x3(x)
    assert float(p2[0]) == 2.0 ** -131
    tiny = np.array([float.fromhex('0x1.8p-133')], dtype=np.float32)  # 3 * 2^-134
    p0, p1, p2 = oracle.split_bf16x3(tiny)
    assert float(p0[0]) == 2.0 ** -132 and float(p1[0]) == 0.0 and float(p2[0]) == 0.0


def test_bf16_split_invariants():
    torch = pytest.importorskip("torch")
    x = np.concatenate([si.uniform((1, 100000), 72).ravel(),
                        si.normal((1, 100000), 73).ravel() * np.float32(1e-20)]).astype(np.float32)
    p0, p1, p2 = oracle.split_bf16x3(x)
    # exact reconstruction
    s = p0.astype(np.float64) + p1.astype(np.float64) + p2.astype(np.float64)
    assert np.array_equal(s, x.astype(np.float64))
    # every plane is bfloat16-representable
    for p in (p0, p1, p2):
        rt = torch.from_numpy(p).to(torch.bfloat16).to(torch.float32).numpy()
        assert np.array_equal(rt, p)
    # magnitudes shrink by at least 2^8 per level
    ax = np.abs(x.astype(np.float64))
    assert np.all(np.abs(p1) <= ax * 2.0 ** -8)
    assert np.all(np.abs(p2) <= ax * 2.0 ** -16)


def test_bf16_split_products_bounds():
    """The 1/3/6-product sums differ from the exact product by at most the
    dropped terms' bound: 3.1*2^-16 (n=3) and 2.1*2^-24 (n=6) of |A||B|."""
    A = si.uniform((40, 300), 81)
    B = si.uniform((300, 30), 82)
    exact = oracle.gemm(A, B)
    den = oracle.gemm_abs(A, B)
    c3 = oracle.gemm_bf16_split(A, B, 3)
    c6 = oracle.gemm_bf16_split(A, B, 6)
    c1 = oracle.gemm_bf16_split(A, B, 1)
    assert np.all(np.abs(c3 - exact) <= 3.1 * 2.0 ** -16 * den)
    assert np.all(np.abs(c6 - exact) <= 2.1 * 2.0 ** -24 * den)
    # each extra level of products buys a large accuracy step, so the three
    # sums are told apart (a wrong term selection collapses one of the gaps)
    e1, e3, e6 = (np.max(np.abs(c - exact) / den) for c in (c1, c3, c6))
    assert e1 > 50 * e3 and e3 > 50 * e6 and e6 > 0


def test_bf16_split_products_exact_for_integers():
    A = si.integers((9, 12), 83)
    B = si.integers((12, 7), 84)
    C0 = si.uniform((9, 7), 85)
    exact = oracle.gemm(A, B, alpha=1.5, beta=0.5, C0=C0)
    for n in (1, 3, 6):
        assert np.array_equal(oracle.gemm_bf16_split(A, B, n, alpha=1.5, beta=0.5, C0=C0), exact)


# ----------------------------------------------------------------- e4m3 ---

def _read_e4m3_golden():
    dec, enc = [], []
    with open(os.path.join(GOLDEN, "e4m3.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            kind, a, b = line.split()
            if kind == "decode":
                dec.append((int(a, 16), b))
            else:
                enc.append((float.fromhex(a), int(b, 16)))
    return dec, enc


_DEC, _ENC = _read_e4m3_golden()


@pytest.mark.parametrize("code,val", _DEC)
def test_e4m3_decode_spec(code, val):
    v = oracle.e4m3_value(code)
    if val == "nan":
        assert math.isnan(v)
    else:
        e = float.fromhex(val)
        assert v == e and math.copysign(1, v) == math.copysign(1, e)


@pytest.mark.parametrize("x,code", _ENC)
def test_e4m3_encode_spec(x, code):
    assert int(oracle.e4m3_encode(np.array([x], dtype=np.float32))[0]) == code


def test_e4m3_encode_matches_torch_in_range():
    torch = pytest.importorskip("torch")
    if not hasattr(torch, "float8_e4m3fn"):
        pytest.skip("torch has no float8_e4m3fn")
    g = np.random.default_rng(5)
    x = np.concatenate([
        g.uniform(-448, 448, 100000).astype(np.float32),
        (g.standard_normal(100000) * 0.01).astype(np.float32),
        # every exact code value and every midpoint between neighbours
        np.array([oracle.e4m3_value(c) for c in range(127)], dtype=np.float32),
        np.array([(oracle.e4m3_value(c) + oracle.e4m3_value(c + 1)) / 2 for c in range(126)],
                 dtype=np.float32),
    ])
    x = np.concatenate([x, -x])
    ours = oracle.e4m3_encode(x)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    # compare values (the sign of zero may differ between conventions)
    assert np.array_equal(oracle.e4m3_decode(ours), oracle.e4m3_decode(ref))


def test_e4m3_encode_is_nearest():
    vals = np.array([oracle.e4m3_value(c) for c in range(127)])
    x = np.abs(si.normal((1, 20000), 91).ravel() * np.float32(40.0))
    codes = oracle.e4m3_encode(x)
    got = oracle.e4m3_decode(codes).astype(np.float64)
    dist = np.abs(x[:, None].astype(np.float64) - vals[None, :])
    assert np.all(np.abs(x - got) <= dist.min(axis=1))


def test_fp8_scales():
    A = np.array([[0, 0, 0], [1, -448, 3], [-896, 2, 1]], dtype=np.float32)
    s = oracle.fp8_scales_rows(A)
    assert list(s) == [1.0, 1.0, 2.0]
    sc = oracle.fp8_scales_cols(A)
    assert list(sc) == [np.float32(896) / np.float32(448), 1.0, np.float32(3) / np.float32(448)]


def test_fp8_dequant_oracle_reduces_to_gemm_on_exact_inputs():
    """With operands already on the E4M3 grid and each row (column) maximum
    equal to 448, the scales are 1, quantisation is the identity, and the
    dequantised product is the plain product."""
    g = np.random.default_rng(17)
    vals = np.array([oracle.e4m3_value(c) for c in range(127)], dtype=np.float32)
    A = (vals[g.integers(0, 127, size=(12, 20))] * g.choice([-1, 1], size=(12, 20))).astype(np.float32)
    B = (vals[g.integers(0, 127, size=(20, 9))] * g.choice([-1, 1], size=(20, 9))).astype(np.float32)
    A[:, 0] = 448.0
    B[0, :] = -448.0
    sa, sb = oracle.fp8_scales_rows(A), oracle.fp8_scales_cols(B)
    assert np.all(sa == 1) and np.all(sb == 1)
    qa, qb = oracle.fp8_quantize_rows(A, sa), oracle.fp8_quantize_cols(B, sb)
    assert np.array_equal(oracle.e4m3_decode(qa), A)
    C0 = si.uniform((12, 9), 18)
    d = oracle.gemm_fp8_dequant(qa, sa, qb, sb, alpha=1.5, beta=0.5, C0=C0)
    assert np.array_equal(d, oracle.gemm(A, B, alpha=1.5, beta=0.5, C0=C0))


def test_fp8_quantize_uses_scale_division():
    A = np.array([[448.0, 224.0, 1.0, -3.0]], dtype=np.float32) * np.float32(3.0)
    sa = oracle.fp8_scales_rows(A)
    assert sa[0] == np.float32(1344.0) / np.float32(448.0) == np.float32(3.0)
    q = oracle.fp8_quantize_rows(A, sa)
    assert list(oracle.e4m3_decode(q)[0]) == [448.0, 224.0, 1.0, -3.0]


def _read_fp8_scaled_golden():
    rows = {}
    with open(os.path.join(GOLDEN, "fp8_scaled.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            key, *vals = line.split()
            conv = (lambda v: int(v, 16)) if key in ("qrow", "qcol", "dq_qa", "dq_qb") else float
            rows.setdefault(key, []).append([conv(v) for v in vals])
    return rows


def test_fp8_scaled_quantisation_hand_fixture():
    """Hand-derived scales and codes for a 3 x 4 matrix quantised by rows and
    by columns with distinct, non-unit scales (tests/golden/fp8_scaled.txt):
    a scale taken from the wrong row or column, or a missing division, changes
    at least one code."""
    g = _read_fp8_scaled_golden()
    X = np.array(g["X"], dtype=np.float32)
    srow = oracle.fp8_scales_rows(X)
    scol = oracle.fp8_scales_cols(X)
    assert np.array_equal(srow, np.array(g["srow"][0], dtype=np.float32))
    assert np.array_equal(scol, np.array(g["scol"][0], dtype=np.float32))
    assert np.array_equal(oracle.fp8_quantize_rows(X, srow), np.array(g["qrow"], dtype=np.uint8))
    assert np.array_equal(oracle.fp8_quantize_cols(X, scol), np.array(g["qcol"], dtype=np.uint8))


def test_fp8_dequant_hand_fixture():
    """A 2 x 2 x 2 dequantised product with distinct row and column scales,
    computed by hand (tests/golden/fp8_scaled.txt); exchanging the roles of
    sa and sb, or applying one of them twice, changes the off-diagonal
    entries."""
    g = _read_fp8_scaled_golden()
    qa = np.array(g["dq_qa"], dtype=np.uint8)
    qb = np.array(g["dq_qb"], dtype=np.uint8)
    sa = np.array(g["dq_sa"][0], dtype=np.float32)
    sb = np.array(g["dq_sb"][0], dtype=np.float32)
    got = oracle.gemm_fp8_dequant(qa, sa, qb, sb)
    assert np.array_equal(got, np.array(g["dq_C"], dtype=np.float64))


def _e4m3_grid_matrix(g, rows, cols, exps, axis):
    """Random values on the E4M3 grid, multiplied by 2^exps along `axis`
    (exps[i] for row i when axis == 1, exps[j] for column j when axis == 0),
    with one entry of each row (column) equal to +-448 * 2^exps so that its
    maximum is exactly that."""
    vals = np.array([oracle.e4m3_value(c) for c in range(127)], dtype=np.float64)
    x = vals[g.integers(0, 127, size=(rows, cols))] * g.choice([-1.0, 1.0], size=(rows, cols))
    if axis == 1:
        x[np.arange(rows), g.integers(0, cols, size=rows)] = 448.0 * g.choice([-1.0, 1.0], size=rows)
        x *= np.exp2(np.asarray(exps, dtype=np.float64))[:, None]
    else:
        x[g.integers(0, rows, size=cols), np.arange(cols)] = 448.0 * g.choice([-1.0, 1.0], size=cols)
        x *= np.exp2(np.asarray(exps, dtype=np.float64))[None, :]
    return x.astype(np.float32)


def test_fp8_scaled_product_equals_gemm_with_power_of_two_scales():
    """Rows of A and columns of B on the E4M3 grid times distinct powers of
    two 2^e_i, 2^f_j, each with maximum 448 * 2^e_i (448 * 2^f_j), and
    M != N: the scales must be exactly 2^e_i and 2^f_j, quantisation must
    then be exact, and the dequantised product -- sa[i] * sb[j] times the sum
    of code products -- must equal the plain product bit for bit (a power of
    two applied to every term of a sum does not change its rounding).  A scale
    indexed by the wrong row or column, a missing or doubled scale, or a
    quantiser dividing by the wrong scale fails one of the assertions."""
    g = np.random.default_rng(29)
    M, N, K = 6, 9, 40
    e = g.permutation(np.arange(-12, 13))[:M]
    f = g.permutation(np.arange(-12, 13))[:N]
    A = _e4m3_grid_matrix(g, M, K, e, axis=1)
    B = _e4m3_grid_matrix(g, K, N, f, axis=0)
    sa, sb = oracle.fp8_scales_rows(A), oracle.fp8_scales_cols(B)
    assert np.array_equal(sa, np.exp2(e).astype(np.float32))
    assert np.array_equal(sb, np.exp2(f).astype(np.float32))
    qa, qb = oracle.fp8_quantize_rows(A, sa), oracle.fp8_quantize_cols(B, sb)
    assert np.array_equal(oracle.e4m3_decode(qa).astype(np.float64) * np.exp2(e)[:, None], A)
    assert np.array_equal(oracle.e4m3_decode(qb).astype(np.float64) * np.exp2(f)[None, :], B)
    C0 = si.uniform((M, N), 30)
    for alpha, beta in ((1.0, 0.0), (1.5, 0.5), (-0.75, 2.0)):
        d = oracle.gemm_fp8_dequant(qa, sa, qb, sb, alpha=alpha, beta=beta, C0=C0)
        assert np.array_equal(d, oracle.gemm(A, B, alpha=alpha, beta=beta, C0=C0))
    # sensitivity: the same codes with the scale vectors reversed differ
    d_rev = oracle.gemm_fp8_dequant(qa, sa[::-1].copy(), qb, sb[::-1].copy())
    assert not np.array_equal(d_rev, oracle.gemm(A, B))


# ---------------------------------------------------------------- norms ---

def test_norms_match_numpy():
    C = si.uniform((30, 40), 101)
    R = si.uniform((30, 40), 102).astype(np.float64)
    rel, num, den, mx = oracle.norms(C, R)
    d = C.astype(np.float64) - R
    assert math.isclose(rel, np.linalg.norm(d) / np.linalg.norm(R), rel_tol=1e-12)
    assert math.isclose(num, np.sum(d * d), rel_tol=1e-12)
    assert math.isclose(den, np.sum(R * R), rel_tol=1e-12)
    assert mx == np.max(np.abs(d))


def test_norms_componentwise_and_zero():
    C = np.array([[1.0, 2.0], [3.0, 4.0]], dtype=np.float32)
    R = np.array([[1.0, 2.5], [3.0, 4.0]])
    den = np.array([[0.0, 2.0], [1.0, 1.0]])
    rel, _, _, mx = oracle.norms(C, R, den)
    assert mx == 0.25
    assert oracle.norms(C, C.astype(np.float64))[0] == 0.0
    den2 = np.array([[1.0, 0.0], [1.0, 1.0]])
    assert math.isinf(oracle.norms(C, R, den2)[3])


# ---- storage order and transposed operands (BLAS-style call, Sec. 2.1) ----

_ORDERS = [(oracle.ROW_MAJOR, "C"), (oracle.COL_MAJOR, "F")]


@pytest.mark.parametrize("order,np_order", _ORDERS)
def test_stored_matrix_reads_numpy_strided_layouts(order, np_order):
    """The oracle's element index agrees with numpy's own strides: a row-major
    matrix with row stride ld is the (ld*4, 4)-strided view of its buffer, a
    column-major one the (4, ld*4)-strided view."""
    rows, cols = 5, 7
    x = si.uniform((rows, cols), 3)
    ld = (cols if np_order == "C" else rows) + 3
    buf = si.storage(x, np_order, ld)
    strides = (ld * 4, 4) if np_order == "C" else (4, ld * 4)
    view = np.lib.stride_tricks.as_strided(buf, shape=(rows, cols), strides=strides)
    assert np.array_equal(view, x)
    assert np.array_equal(oracle.stored_matrix(buf, order, rows, cols, ld), x)
    assert np.array_equal(si.unstorage(buf, np_order, rows, cols, ld), x)
    # the padding is never part of the matrix
    assert np.isnan(buf).sum() == buf.size - rows * cols


@pytest.mark.parametrize("order,np_order", _ORDERS)
@pytest.mark.parametrize("ta", [oracle.NO_TRANS, oracle.TRANS])
@pytest.mark.parametrize("tb", [oracle.NO_TRANS, oracle.TRANS])
def test_gemm_op_exact_integer_products(order, np_order, ta, tb):
    """alpha*op(A)op(B) + beta*C against exact Python integers, for operands
    placed in memory by numpy (C or Fortran order, padded leading
    dimensions), with M, N, K distinct so that a misread or mis-transposed
    operand cannot go unnoticed."""
    M, N, K = 4, 3, 5
    op_a, op_b, c0 = si.integers((M, K), 1), si.integers((K, N), 2), si.integers((M, N), 3)
    a_st = op_a.T.copy() if ta == oracle.TRANS else op_a
    b_st = op_b.T.copy() if tb == oracle.TRANS else op_b

    def ld_of(x):
        return (x.shape[1] if np_order == "C" else x.shape[0]) + 2

    lda, ldb, ldc = ld_of(a_st), ld_of(b_st), ld_of(c0)
    got = oracle.gemm_op(order, ta, tb, M, N, K, 2.0, si.storage(a_st, np_order, lda), lda,
                         si.storage(b_st, np_order, ldb), ldb, -1.0,
                         si.storage(c0, np_order, ldc), ldc)
    exact = [[2 * sum(int(op_a[i, k]) * int(op_b[k, j]) for k in range(K)) - int(c0[i, j])
              for j in range(N)] for i in range(M)]
    assert np.array_equal(got, np.array(exact, dtype=np.float64))


@pytest.mark.parametrize("ta", [oracle.NO_TRANS, oracle.TRANS])
@pytest.mark.parametrize("tb", [oracle.NO_TRANS, oracle.TRANS])
def test_column_major_is_the_transposed_row_major_product(ta, tb):
    """(op(A) op(B))^T = op(B)^T op(A)^T: a column-major product over given
    buffers equals the transpose of the row-major product over the same
    buffers with the operands exchanged, M and N exchanged and each operand
    keeping its flag."""
    M, N, K = 6, 4, 9
    bufA = si.uniform((1, 200), 11).reshape(-1)
    bufB = si.uniform((1, 200), 12).reshape(-1)
    bufC = si.uniform((1, 200), 13).reshape(-1)
    lda = (K if ta == oracle.TRANS else M) + 1
    ldb = (N if tb == oracle.TRANS else K) + 1
    ldc = M + 1
    col = oracle.gemm_op(oracle.COL_MAJOR, ta, tb, M, N, K, 1.5, bufA, lda, bufB, ldb, 0.5, bufC, ldc)
    row = oracle.gemm_op(oracle.ROW_MAJOR, tb, ta, N, M, K, 1.5, bufB, ldb, bufA, lda, 0.5, bufC, ldc)
    assert np.array_equal(col, row.T)


def test_gemm_op_beta_zero_never_reads_c():
    M, N, K = 3, 2, 4
    a, b = si.integers((M, K), 5), si.integers((K, N), 6)
    bufC = np.full(M * N, np.nan, dtype=np.float32)
    got = oracle.gemm_op(oracle.ROW_MAJOR, oracle.NO_TRANS, oracle.NO_TRANS, M, N, K, 1.0,
                         a.reshape(-1), K, b.reshape(-1), N, 0.0, bufC, N)
    assert np.array_equal(got, a.astype(np.float64) @ b.astype(np.float64))


# ---- binary64 product (double-double evaluation) ----------------------------

def _exact_int_product(A, B, alpha, beta, C0):
    M, K = A.shape
    N = B.shape[1]
    return [[alpha * sum(int(A[i, k]) * int(B[k, j]) for k in range(K)) +
             (beta * int(C0[i, j]) if beta else 0) for j in range(N)] for i in range(M)]


def test_dgemm_exact_beyond_2_53():
    """Integer operands up to 2^26: the products reach 2^52 and the sums pass
    2^53, where binary64 accumulation rounds.  The oracle must return the
    correctly rounded exact integer (Python ints, float() rounds to nearest
    even) -- and plain binary64 accumulation must fail, or the case would not
    test anything."""
    g = np.random.default_rng(77)
    M, N, K = 9, 7, 13
    A = g.integers(-2 ** 26, 2 ** 26, size=(M, K)).astype(np.float64)
    B = g.integers(-2 ** 26, 2 ** 26, size=(K, N)).astype(np.float64)
    C0 = g.integers(-2 ** 50, 2 ** 50, size=(M, N)).astype(np.float64)
    exact = _exact_int_product(A, B, 3, -1, C0)
    want = np.array([[float(v) for v in row] for row in exact])
    got = oracle.dgemm(A, B, alpha=3.0, beta=-1.0, C0=C0)
    assert np.array_equal(got, want)
    plain = 3.0 * (A @ B) - C0
    assert not np.array_equal(plain, want)


def test_dgemm_matches_exact_rationals():
    """Random binary64 operands on tiny shapes: the exact rational result
    (fractions.Fraction), rounded once, against the oracle; the double-double
    evaluation is faithful, so at most one unit in the last place apart, and
    equal in all but exceptional near-tie cases."""
    g = np.random.default_rng(78)
    exact_hits = total = 0
    for (M, N, K) in itertools.product((1, 3, 5), (1, 4), (1, 2, 7)):
        A = g.standard_normal((M, K)) * np.exp2(g.integers(-20, 20, size=(M, K)))
        B = g.standard_normal((K, N)) * np.exp2(g.integers(-20, 20, size=(K, N)))
        C0 = g.standard_normal((M, N))
        got = oracle.dgemm(A, B, alpha=1.25, beta=-0.75, C0=C0)
        for i in range(M):
            for j in range(N):
                r = Fraction(1.25) * sum(Fraction(A[i, k]) * Fraction(B[k, j]) for k in range(K)) \
                    + Fraction(-0.75) * Fraction(C0[i, j])
                want = float(r)
                assert abs(got[i, j] - want) <= np.spacing(abs(want)), (M, N, K, i, j)
                exact_hits += got[i, j] == want
                total += 1
    assert exact_hits >= total - 1


def test_dgemm_survives_catastrophic_cancellation():
    """x + y - x with |x| >> |y|: binary64 accumulation loses y entirely, the
    compensated sum keeps it (a dropped low part would fail here)."""
    A = np.array([[1e20, 1.0, -1e20, 3.0]])
    B = np.array([[1.0], [1.0], [1.0], [1e-30]])
    got = oracle.dgemm(A, B)
    assert got[0, 0] == float(Fraction(1) + Fraction(3.0) * Fraction(1e-30))
    assert (A @ B)[0, 0] != got[0, 0]


def test_dgemm_rank_one_closed_form_and_special_cases():
    K = 4096
    x = np.arange(1, 6, dtype=np.float64)
    z = np.arange(-3, 4, dtype=np.float64)
    kk = np.arange(1, K + 1, dtype=np.float64)
    A = np.outer(x, kk)
    B = np.outer(kk, z)
    got = oracle.dgemm(A, B)
    closed = np.outer(x, z) * (K * (K + 1) * (2 * K + 1) // 6)
    assert np.array_equal(got, closed)
    # beta == 0 never reads C0; alpha == 0 leaves beta*C0
    C0 = np.full((5, 7), np.nan)
    assert np.array_equal(oracle.dgemm(A, B, beta=0.0, C0=C0), closed)
    C1 = np.arange(35, dtype=np.float64).reshape(5, 7)
    assert np.array_equal(oracle.dgemm(A, B, alpha=0.0, beta=2.0, C0=C1), 2.0 * C1)
    den = oracle.dgemm(A, B, alpha=-1.0, beta=-2.0, C0=C1, absolute=True)
    assert np.array_equal(den, np.abs(closed) + 2.0 * C1)
