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
