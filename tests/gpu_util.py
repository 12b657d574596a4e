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
