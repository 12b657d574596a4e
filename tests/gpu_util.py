"""Helpers for the GPU parity tests: device copies with padded rows, and the
tolerances every path is held to."""
from __future__ import annotations

import numpy as np

U = 2.0 ** -24  # binary32 unit roundoff


def dev_matrix(x: np.ndarray, ld: int | None = None, pad: float = float("nan")):
    """Copy a float32 matrix to the GPU as an (rows, ld) buffer whose first
    `cols` columns hold x and the rest hold `pad`.  Returns (buffer, view)."""
    import torch
    rows, cols = x.shape
    ld = max(1, cols) if ld is None else ld
    buf = np.full((max(rows, 1), ld), pad, dtype=np.float32)
    buf[:rows, :cols] = x
    t = torch.from_numpy(buf).cuda()
    return t, t[:rows, :cols]


def gamma(K: int, extra: int = 2) -> float:
    """Higham's gamma_n = n u / (1 - n u) for an n-term dot product, with
    `extra` roundings for the alpha/beta epilogue."""
    n = K + extra
    return n * U / (1 - n * U)


def sample_rows(M: int, count: int, seed: int) -> np.ndarray:
    g = np.random.default_rng(seed)
    return np.sort(g.choice(M, size=min(count, M), replace=False))


# Worst-case bound of the dropped split products relative to |A||B|
# (3.1 * 2^-16 for three products, 2.1 * 2^-24 for six); see the oracle pins.
DROPPED = {3: 3.1 * 2.0 ** -16, 6: 2.1 * 2.0 ** -24}

# Problems at least this large (M*N*K) are held to the 1e-5 relative Frobenius
# target; smaller ones, where a handful of products cannot average the split
# error, are held to the componentwise worst-case bound instead.
REL_FRO_MIN_WORK = 32768


def check_split_result(oracle, A, B, C0, C, alpha, beta, n):
    """Pins for a split-precision result: componentwise against the exact sum
    of the selected split products (binary32 accumulation of n*K terms, factor
    2 margin for the matrix core's internal summation), componentwise against
    the exact product (dropped terms + accumulation), and the relative
    Frobenius target for problems of realistic size.  Returns rel_fro."""
    M, K = A.shape
    N = B.shape[1]
    ref = oracle.gemm(A, B, alpha=alpha, beta=beta, C0=C0)
    den = oracle.gemm_abs(A, B, alpha=alpha, beta=beta, C0=C0)
    rel, _, _, cw_exact = oracle.norms(C, ref, den)
    split = oracle.gemm_bf16_split(A, B, n, alpha=alpha, beta=beta, C0=C0)
    cw_split = oracle.norms(C, split, den)[3]
    assert cw_split <= 2 * 1.01 * gamma(n * K), (cw_split, gamma(n * K))
    assert cw_exact <= DROPPED[n] + 2 * 1.01 * gamma(n * K), cw_exact
    if M * N * K >= REL_FRO_MIN_WORK:
        assert rel <= 1e-5, rel
    return rel


# ---- FP8 matrix-core bound ---------------------------------------------------
#
# Accumulation into binary32: a componentwise error of up to 2.4 gamma_K
# against the dequantised oracle was measured; the bound allows 8.
FP8_MARGIN = 8
# Within each group of eight consecutive k the f8f6f4 matrix core truncates
# every product toward zero to a multiple of 2^(E - 13), E the exponent of the
# group's largest product, before summing the group (pinned on hand-built codes
# by test_gpu_fp8.py::test_group_products_truncate_toward_zero_on_the_group_grid).
# The largest product and any of its binade are on that grid, so at most seven
# products lose less than one step each: less than 7 * 2^-13 of the group's
# largest |product|, itself at most the product of the group's maxima (which
# also covers an alignment on the maxima's exponents).
FP8_GROUP_TRUNC = 7 * 2.0 ** -13
FP8_GROUP = 8


def fp8_group_term(qa, qb, sa, sb, alpha):
    """Upper bound of the group truncation error of C[i,j]:
    7 * 2^-13 |alpha| sa[i] sb[j] sum_g max_{k in g} |qa[i,k]| * max_{k in g} |qb[k,j]|
    (the product of the group maxima bounds the group's largest product).
    qa: M x K codes, qb: K x N codes, groups of eight k from k = 0."""
    import oracle
    M, K = qa.shape
    N = qb.shape[1]
    G = (K + FP8_GROUP - 1) // FP8_GROUP
    a = np.zeros((M, G * FP8_GROUP))
    a[:, :K] = np.abs(oracle.e4m3_decode(qa).astype(np.float64))
    b = np.zeros((G * FP8_GROUP, N))
    b[:K] = np.abs(oracle.e4m3_decode(qb).astype(np.float64))
    amax = a.reshape(M, G, FP8_GROUP).max(axis=2)
    bmax = b.reshape(G, FP8_GROUP, N).max(axis=1)
    s = np.abs(alpha) * sa.astype(np.float64)[:, None] * sb.astype(np.float64)[None, :]
    return FP8_GROUP_TRUNC * s * (amax @ bmax)


def fp8_check(oracle, C, qa, qb, sa, sb, alpha, beta, C0):
    """C of a scaled FP8 product (qa: M x K codes, qb: K x N codes) against the
    dequantised-input oracle: |C - ref| <= 8 gamma_{K+4} |ref terms| + the
    group truncation term, elementwise.  Returns (rel_fro, max ratio to the
    bound, max ratio to |alpha||A||B| + |beta||C0| of the codes)."""
    K = qa.shape[1]
    ref = oracle.gemm_fp8_dequant(qa, sa, qb, sb, alpha=alpha, beta=beta, C0=C0)
    den = oracle.gemm_fp8_dequant(qa & 0x7F, sa, qb & 0x7F, sb, alpha=abs(alpha),
                                  beta=abs(beta), C0=None if C0 is None else np.abs(C0))
    bound = FP8_MARGIN * gamma(K, extra=4) * den + fp8_group_term(qa, qb, sa, sb, alpha)
    rel, _, _, ratio = oracle.norms(C, ref, bound)
    return rel, ratio, oracle.norms(C, ref, den)[3]
