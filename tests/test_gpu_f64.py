"""Binary64 path on the FP64 matrix cores: parity against the double-double
oracle (componentwise within Higham's binary64 bound gamma_{K+2}|A||B|, the
oracle being far more accurate than binary64), exactness on integer inputs,
every tile configuration, edges, quick paths, and the batched-strided form."""
import numpy as np
import pytest

import oracle
import seeded_inputs as si
from gpu_util import sample_rows

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53


def gamma64(K, extra=2):
    n = K + extra
    return n * U64 / (1 - n * U64)


def _u(shape, seed):
    return si.uniform(shape, seed).astype(np.float64)


def _dev(x, ld=None, pad=np.nan):
    import torch
    rows, cols = x.shape
    ld = max(1, cols) if ld is None else ld
    buf = np.full((max(rows, 1), ld), pad, dtype=np.float64)
    buf[:rows, :cols] = x
    t = torch.from_numpy(buf).cuda()
    return t, t[:rows, :cols]


def _check(A, B, C0, C, alpha, beta):
    ref = oracle.dgemm(A, B, alpha=alpha, beta=beta, C0=C0)
    den = oracle.dgemm(A, B, alpha=alpha, beta=beta, C0=C0, absolute=True)
    K = A.shape[1]
    err = np.abs(C - ref)
    bound = gamma64(K) * den
    bad = np.argwhere(err > bound)
    assert bad.size == 0, [(tuple(i), err[tuple(i)], bound[tuple(i)]) for i in bad[:5]]
    nref = np.linalg.norm(ref)
    if nref > 0 and A.shape[0] * B.shape[1] * K >= 32768:
        assert np.linalg.norm(C - ref) / nref <= 1e-14


def _run(mm, A, B, C0, alpha, beta, cfg=None, lds=(None, None, None)):
    import torch
    M, K = A.shape
    N = B.shape[1]
    _, dA = _dev(A, lds[0])
    _, dB = _dev(B, lds[1])
    cbuf, dC = _dev(C0, lds[2], pad=-7.0)
    if cfg is None:
        mm.gemm_f64(M, N, K, alpha, dA, dA.stride(0), dB, dB.stride(0), beta, dC, dC.stride(0))
    else:
        mm.gemm_f64_run_config(cfg, M, N, K, alpha, dA, dA.stride(0), dB, dB.stride(0), beta, dC,
                               dC.stride(0))
    torch.cuda.synchronize()
    return cbuf.cpu().numpy(), dC.cpu().numpy()


SHAPES = [(1, 1, 1), (64, 64, 16), (130, 200, 1000), (257, 129, 777), (300, 1, 33), (1, 300, 17),
          (513, 257, 64), (100, 130, 3)]


@pytest.mark.parametrize("M,N,K", SHAPES)
@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (1.5, 0.5), (-0.75, 2.0)])
def test_parity_default_config(M, N, K, alpha, beta):
    import paper_1902_10345_amd as mm
    seed = M + 5 * N + 11 * K
    A, B, C0 = _u((M, K), seed), _u((K, N), seed + 1), _u((M, N), seed + 2)
    _, C = _run(mm, A, B, C0, alpha, beta)
    _check(A, B, C0, C, alpha, beta)


def _fits(mm, cfg, M, N):
    name = mm.gemm_config_name(mm.PATH_F64, cfg)
    if not name.startswith("f64_small_"):
        return True
    lim = int(name.rsplit("_", 1)[1])
    return M <= lim and N <= lim


@pytest.mark.parametrize("M,N,K", [(300, 260, 333), (129, 67, 1001), (256, 128, 48), (16, 16, 40),
                                   (13, 7, 33), (32, 32, 32), (29, 31, 17), (64, 64, 100),
                                   (50, 3, 64), (1, 1, 1)])
def test_every_config(M, N, K):
    """Every configuration that accepts the shape (the small-problem ones take
    M, N up to their size and refuse larger problems)."""
    import paper_1902_10345_amd as mm
    A, B, C0 = _u((M, K), 3), _u((K, N), 4), _u((M, N), 5)
    ran = 0
    for cfg in range(mm.gemm_num_configs(mm.PATH_F64)):
        if not _fits(mm, cfg, M, N):
            with pytest.raises(mm.GemmError):
                _run(mm, A, B, C0, 1.5, 0.5, cfg=cfg)
            continue
        _, C = _run(mm, A, B, C0, 1.5, 0.5, cfg=cfg)
        _check(A, B, C0, C, 1.5, 0.5)
        ran += 1
    assert ran >= 3


def test_every_config_integer_inputs_are_exact():
    import paper_1902_10345_amd as mm
    M, N, K = 300, 260, 999
    A = si.integers((M, K), 7, -1000, 1000).astype(np.float64)
    B = si.integers((K, N), 8, -1000, 1000).astype(np.float64)
    C0 = si.integers((M, N), 9, -1000, 1000).astype(np.float64)
    exact = oracle.dgemm(A, B, alpha=2.0, beta=-3.0, C0=C0)
    for cfg in range(mm.gemm_num_configs(mm.PATH_F64)):
        if not _fits(mm, cfg, M, N):
            continue
        _, C = _run(mm, A, B, C0, 2.0, -3.0, cfg=cfg)
        assert np.array_equal(C, exact), mm.gemm_config_name(mm.PATH_F64, cfg)
    # and the small-problem configurations on a shape they take
    A2, B2, C2 = A[:64, :77], B[:77, :64], C0[:64, :64]
    exact2 = oracle.dgemm(np.ascontiguousarray(A2), np.ascontiguousarray(B2), alpha=2.0, beta=-3.0,
                          C0=np.ascontiguousarray(C2))
    for cfg in range(mm.gemm_num_configs(mm.PATH_F64)):
        if _fits(mm, cfg, 64, 64):
            _, C = _run(mm, np.ascontiguousarray(A2), np.ascontiguousarray(B2),
                        np.ascontiguousarray(C2), 2.0, -3.0, cfg=cfg)
            assert np.array_equal(C, exact2), mm.gemm_config_name(mm.PATH_F64, cfg)


def test_padded_odd_leading_dimensions_and_untouched_padding():
    """Odd lda takes the 64-bit load path; NaN padding in A and B must never
    be read; C's padding keeps its value."""
    import paper_1902_10345_amd as mm
    M, N, K = 133, 97, 1071
    A, B, C0 = _u((M, K), 15), _u((K, N), 16), _u((M, N), 17)
    cbuf, C = _run(mm, A, B, C0, 1.5, 0.5, lds=(1073, 99, 101))
    _check(A, B, C0, C, 1.5, 0.5)
    assert np.all(cbuf[:, N:] == -7.0)


def test_unaligned_a_pointer_takes_the_scalar_path():
    import torch
    import paper_1902_10345_amd as mm
    M, N, K = 150, 140, 300
    A, B, C0 = _u((M, K), 21), _u((K, N), 22), _u((M, N), 23)
    flat = torch.zeros(M * K + 1, dtype=torch.float64, device="cuda")
    flat[1:] = torch.from_numpy(A.reshape(-1))
    dA = flat[1:]  # 8-byte but not 16-byte aligned
    dB, dC = torch.from_numpy(B).cuda(), torch.from_numpy(C0).cuda()
    mm.gemm_f64(M, N, K, 1.5, dA, K, dB, N, 0.5, dC, N)
    torch.cuda.synchronize()
    _check(A, B, C0, dC.cpu().numpy(), 1.5, 0.5)


def test_beta_zero_ignores_nan_and_quick_paths():
    import torch
    import paper_1902_10345_amd as mm
    M, N, K = 200, 150, 400
    A, B = _u((M, K), 31), _u((K, N), 32)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    dC = torch.full((M, N), float("nan"), dtype=torch.float64, device="cuda")
    mm.gemm_f64(M, N, K, 1.0, dA, K, dB, N, 0.0, dC, N)
    torch.cuda.synchronize()
    _check(A, B, None, dC.cpu().numpy(), 1.0, 0.0)
    C0 = _u((M, N), 33)
    for alpha, k in ((0.0, K), (1.0, 0)):
        dC = torch.from_numpy(C0.copy()).cuda()
        mm.gemm_f64(M, N, k, alpha, None if alpha == 0.0 else dA, max(1, k), None, N, 0.5, dC, N)
        torch.cuda.synchronize()
        assert np.array_equal(dC.cpu().numpy(), 0.5 * C0)


def test_deterministic():
    import paper_1902_10345_amd as mm
    A, B, C0 = _u((257, 300), 41), _u((300, 259), 42), _u((257, 259), 43)
    _, C1 = _run(mm, A, B, C0, 1.5, 0.5)
    _, C2 = _run(mm, A, B, C0, 1.5, 0.5)
    assert np.array_equal(C1, C2)


@pytest.mark.parametrize("M,N,K,seed", [(4096, 4096, 4096, 2), (8192, 2048, 4096, 3)])
def test_full_size_sampled_rows(M, N, K, seed):
    import torch
    import paper_1902_10345_amd as mm
    A, B, C0 = _u((M, K), seed), _u((K, N), seed + 100), _u((M, N), seed + 200)
    dA, dB, dC = (torch.from_numpy(x).cuda() for x in (A, B, C0))
    mm.gemm_f64(M, N, K, 1.5, dA, K, dB, N, 0.5, dC, N)
    torch.cuda.synchronize()
    rows = sample_rows(M, 24, seed)
    _check(A[rows], B, C0[rows], dC.cpu().numpy()[rows], 1.5, 0.5)


# ---- batched-strided (SBSMM) ------------------------------------------------

def _batched(mm, M, N, K, batch, seed, pad=(0, 0, 0), share_b=False, alpha=1.5, beta=0.5):
    """Problems stored back to back with extra elements between them (pad)."""
    import torch
    g = np.random.default_rng(seed)
    sa, sb, sc = M * K + pad[0], (0 if share_b else K * N + pad[1]), M * N + pad[2]
    hA = g.uniform(-1, 1, size=batch * sa).astype(np.float64)
    hB = g.uniform(-1, 1, size=max(1, batch * sb if sb else K * N)).astype(np.float64)
    hC = g.uniform(-1, 1, size=batch * sc).astype(np.float64)
    dA, dB, dC = (torch.from_numpy(x).cuda() for x in (hA, hB, hC))
    mm.gemm_f64_strided_batched(M, N, K, alpha, dA, K, sa, dB, N, sb, beta, dC, N, sc, batch)
    torch.cuda.synchronize()
    out = dC.cpu().numpy()
    for b in range(batch):
        A = hA[b * sa:b * sa + M * K].reshape(M, K)
        B = hB[b * sb:b * sb + K * N].reshape(K, N)
        C0 = hC[b * sc:b * sc + M * N].reshape(M, N)
        C = out[b * sc:b * sc + M * N].reshape(M, N)
        _check(A, B, C0, C, alpha, beta)
        # the gap between problems is untouched
        assert np.array_equal(out[b * sc + M * N:(b + 1) * sc], hC[b * sc + M * N:(b + 1) * sc])


@pytest.mark.parametrize("M,N,K,batch", [(16, 16, 16, 100), (32, 32, 32, 37), (12, 12, 12, 50),
                                         (70, 50, 90, 9), (130, 129, 64, 3), (1, 1, 5, 7),
                                         (64, 64, 64, 11), (33, 17, 40, 13), (64, 40, 7, 6),
                                         (16, 32, 100, 21)])
def test_batched_strided_parity(M, N, K, batch):
    import paper_1902_10345_amd as mm
    _batched(mm, M, N, K, batch, M + N + K + batch)
    _batched(mm, M, N, K, batch, M + N + K + batch + 1, pad=(3, 5, 7))


def test_batched_strided_shared_b_and_single_problem_equals_gemm_f64():
    import torch
    import paper_1902_10345_amd as mm
    _batched(mm, 40, 24, 33, 20, 5, share_b=True)
    M, N, K = 130, 140, 150
    A, B, C0 = _u((M, K), 51), _u((K, N), 52), _u((M, N), 53)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    d1, d2 = torch.from_numpy(C0.copy()).cuda(), torch.from_numpy(C0.copy()).cuda()
    mm.gemm_f64(M, N, K, 1.5, dA, K, dB, N, 0.5, d1, N)
    mm.gemm_f64_strided_batched(M, N, K, 1.5, dA, K, 0, dB, N, 0, 0.5, d2, N, 0, 1)
    torch.cuda.synchronize()
    assert np.array_equal(d1.cpu().numpy(), d2.cpu().numpy())


def test_batched_strided_more_problems_than_one_launch():
    """65 540 problems: the grid's second dimension holds 65 535 per launch,
    the rest go in a second launch.  Integer inputs, exact results."""
    import torch
    import paper_1902_10345_amd as mm
    M = N = K = 2
    batch = 65540
    g = np.random.default_rng(61)
    hA = g.integers(-9, 10, size=(batch, M, K)).astype(np.float64)
    hB = g.integers(-9, 10, size=(batch, K, N)).astype(np.float64)
    hC = g.integers(-9, 10, size=(batch, M, N)).astype(np.float64)
    dA, dB, dC = (torch.from_numpy(x).cuda() for x in (hA, hB, hC))
    mm.gemm_f64_strided_batched(M, N, K, 2.0, dA, K, M * K, dB, N, K * N, -1.0, dC, N, M * N, batch)
    torch.cuda.synchronize()
    assert np.array_equal(dC.cpu().numpy(), 2.0 * np.matmul(hA, hB) - hC)
