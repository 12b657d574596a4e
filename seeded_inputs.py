"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no arithmetic of the GEMM method: it only draws random
numbers (numpy ``default_rng``, PCG64) and shapes them into the workloads the
library is exercised on.  Both the oracle side and the GPU side consume the
same host arrays produced here.

Workloads (all matrices binary32, row-major):
  * dense uniform[-1, 1) operands (the paper's fundamental-kernel MM is a
    synthetic square single-precision product, Sec. 6.1);
  * N(0, 1) operands with a seeded 1% of columns scaled by 1e3 (outliers) for
    the scaled FP8 path;
  * integer-valued operands (exact in binary32 and bfloat16) for exactness
    checks;
  * grouped problem sets with log-uniform M, N, K (exp of a uniform draw on
    [ln lo, ln hi]), rounded to a multiple and clamped;
  * Poisson request arrivals (exponential inter-arrival gaps) for serving.
"""
from __future__ import annotations

import math

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def uniform(shape, seed: int, lo: float = -1.0, hi: float = 1.0, ld: int | None = None,
            pad_value: float = 0.0) -> np.ndarray:
    """uniform[lo, hi) binary32 matrix; optional row stride ld >= cols.

    With ld > cols the result is a view into an (rows, ld) buffer whose
    padding columns hold pad_value (e.g. NaN to prove they are never read)."""
    g = rng(seed)
    rows, cols = shape
    x = g.random((rows, cols), dtype=np.float32)
    x = (x * np.float32(hi - lo) + np.float32(lo)).astype(np.float32)
    return with_ld(x, ld, pad_value)


def normal(shape, seed: int, ld: int | None = None) -> np.ndarray:
    g = rng(seed)
    x = g.standard_normal(shape, dtype=np.float32)
    return with_ld(x, ld)


def integers(shape, seed: int, lo: int = -8, hi: int = 8) -> np.ndarray:
    """Integer-valued binary32 matrix with entries in [lo, hi]."""
    g = rng(seed)
    return g.integers(lo, hi + 1, size=shape).astype(np.float32)


def with_ld(x: np.ndarray, ld: int | None, pad_value: float = 0.0) -> np.ndarray:
    rows, cols = x.shape
    if ld is None or ld == cols:
        return np.ascontiguousarray(x)
    assert ld > cols
    buf = np.full((rows, ld), pad_value, dtype=np.float32)
    buf[:, :cols] = x
    return buf[:, :cols]


def storage(x: np.ndarray, order: str, ld: int, pad_value: float = float("nan")) -> np.ndarray:
    """Flat binary32 buffer holding matrix x in storage order `order` ("C":
    row-major, rows of ld elements; "F": column-major, columns of ld
    elements), built from numpy's own C- and Fortran-ordered arrays.  The
    ld - extent padding elements hold pad_value."""
    rows, cols = x.shape
    if order == "C":
        assert ld >= max(1, cols)
        buf = np.full((max(rows, 1), ld), pad_value, dtype=np.float32, order="C")
        buf[:rows, :cols] = x
        return buf.ravel(order="C")
    assert order == "F" and ld >= max(1, rows)
    buf = np.full((ld, max(cols, 1)), pad_value, dtype=np.float32, order="F")
    buf[:rows, :cols] = x
    return buf.ravel(order="F")


def unstorage(buf: np.ndarray, order: str, rows: int, cols: int, ld: int) -> np.ndarray:
    """Inverse of storage(): the rows x cols matrix held in a flat buffer (a
    C-contiguous copy)."""
    if order == "C":
        x = np.asarray(buf[:rows * ld]).reshape(rows, ld, order="C")[:, :cols] if rows else \
            np.zeros((0, cols), np.float32)
    else:
        x = np.asarray(buf[:cols * ld]).reshape(ld, cols, order="F")[:rows, :] if cols else \
            np.zeros((rows, 0), np.float32)
    return np.ascontiguousarray(x)


def outlier_columns(n_cols: int, frac: float, seed: int) -> np.ndarray:
    """Sorted indices of ceil(frac * n_cols) distinct seeded columns."""
    g = rng(seed)
    count = int(math.ceil(frac * n_cols))
    return np.sort(g.choice(n_cols, size=count, replace=False))


def fp8_workload(M: int, N: int, K: int, seed: int, outliers: str = "none"):
    """A (MxK), B (KxN) ~ N(0,1); C0 ~ U[-1,1).

    outliers = "A": ceil(1% of K) columns of A (k indices) scaled by 1e3;
    outliers = "B": ceil(1% of N) columns of B scaled by 1e3; "none": no scaling."""
    A = normal((M, K), seed)
    B = normal((K, N), seed + 1000)
    C0 = uniform((M, N), seed + 2000)
    if outliers == "A":
        cols = outlier_columns(K, 0.01, seed + 3000)
        A[:, cols] *= np.float32(1e3)
    elif outliers == "B":
        cols = outlier_columns(N, 0.01, seed + 3000)
        B[:, cols] *= np.float32(1e3)
    elif outliers != "none":
        raise ValueError(outliers)
    return A, B, C0


def log_uniform_sizes(count: int, lo: int, hi: int, seed: int, multiple: int = 1) -> np.ndarray:
    """count x 3 array of (M, N, K), each exp(U[ln lo, ln hi]) rounded to the
    nearest multiple of `multiple`, then clamped to [lo, hi]."""
    g = rng(seed)
    raw = np.exp(g.uniform(math.log(lo), math.log(hi), size=(count, 3)))
    r = np.rint(raw / multiple) * multiple
    return np.clip(r, lo, hi).astype(np.int64)


def grouped_problems(count: int = 512, seed: int = 5, lo: int = 32, hi: int = 1024,
                     multiple: int = 16):
    """Sizes and operands of a grouped batch: list of (M, N, K, A, B)."""
    sizes = log_uniform_sizes(count, lo, hi, seed, multiple)
    probs = []
    for t, (M, N, K) in enumerate(sizes):
        A = uniform((int(M), int(K)), seed * 100003 + 2 * t)
        B = uniform((int(K), int(N)), seed * 100003 + 2 * t + 1)
        probs.append((int(M), int(N), int(K), A, B))
    return probs


def poisson_arrivals(rate_per_s: float, duration_s: float, seed: int) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process, sorted."""
    g = rng(seed)
    n_est = int(rate_per_s * duration_s * 1.2 + 100)
    gaps = g.exponential(1.0 / rate_per_s, size=n_est)
    t = np.cumsum(gaps)
    while t[-1] < duration_s:
        more = np.cumsum(g.exponential(1.0 / rate_per_s, size=n_est)) + t[-1]
        t = np.concatenate([t, more])
    return t[t < duration_s]


def serving_requests(rate_per_s: float, duration_s: float, seed: int, lo: int = 64,
                     hi: int = 2048):
    """(arrival_times, sizes[n,3]) for the serving workload: M, N, K
    log-uniform in [lo, hi], rounded to the nearest integer."""
    t = poisson_arrivals(rate_per_s, duration_s, seed)
    sizes = log_uniform_sizes(len(t), lo, hi, seed + 1, multiple=1)
    return t, sizes


class OperandPool:
    """A pool of uniform[-1,1) binary32 values from which request operands are
    taken as slices, so that a long request stream does not need fresh random
    data per request.  operand(n, key) returns n contiguous values starting at
    a seeded offset derived from key."""

    def __init__(self, n_values: int, seed: int):
        self.values = uniform((1, n_values), seed).reshape(-1)
        self.n = n_values

    def operand(self, rows: int, cols: int, key: int) -> np.ndarray:
        n = rows * cols
        assert n <= self.n
        off = (key * 2654435761) % (self.n - n + 1)
        return self.values[off:off + n].reshape(rows, cols)
