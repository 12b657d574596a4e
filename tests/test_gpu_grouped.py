"""Grouped persistent launch on the 3xBF16 path: every member against the
oracle, every member bitwise equal to the same problem run alone with the
same tile shape, degenerate members, and HIP-graph replays."""
import numpy as np
import pytest

import oracle
import seeded_inputs as si
from gpu_util import check_split_result

pytestmark = pytest.mark.gpu

# tile variant of the grouped kernel -> the single-GEMM configuration with the
# same tile body
SOLO_CFG = {0: "bx3_128x128x32_4w64x64_p3", 1: "bx3_64x64x32_4w32x32_p3"}


def _cfg_index(mm, name):
    for c in range(mm.gemm_num_configs(mm.PATH_3XBF16)):
        if mm.gemm_config_name(mm.PATH_3XBF16, c) == name:
            return c
    raise KeyError(name)


def _problems(seed, count, lo=32, hi=512, multiple=16, extra=()):
    sizes = [tuple(int(v) for v in r) for r in si.log_uniform_sizes(count, lo, hi, seed, multiple)]
    sizes += list(extra)
    probs = []
    for t, (M, N, K) in enumerate(sizes):
        A = si.uniform((M, K), seed * 1000 + 3 * t)
        B = si.uniform((K, N), seed * 1000 + 3 * t + 1)
        C0 = si.uniform((M, N), seed * 1000 + 3 * t + 2)
        probs.append([M, N, K, A, B, C0])
    return probs


def _to_device(probs, alpha, beta):
    import torch
    import paper_1902_10345_amd as mm
    dev = []
    for M, N, K, A, B, C0 in probs:
        dA = torch.from_numpy(A).cuda() if A.size else torch.zeros(1, device="cuda")
        dB = torch.from_numpy(B).cuda() if B.size else torch.zeros(1, device="cuda")
        dC = torch.from_numpy(C0).cuda() if C0.size else torch.zeros(1, device="cuda")
        dev.append((M, N, K, dA, max(K, 1), dB, max(N, 1), dC, max(N, 1), alpha, beta))
    return dev, mm.problem_array(dev)


@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (1.5, 0.5)])
def test_members_match_oracle_and_solo_runs(alpha, beta):
    import torch
    import paper_1902_10345_amd as mm
    extra = [(1, 1, 1), (129, 77, 300), (0, 50, 50), (50, 0, 50), (37, 41, 0), (300, 1, 64),
             (1, 300, 64), (200, 200, 17)]
    probs = _problems(seed=5, count=40, extra=extra)
    dev, arr = _to_device(probs, alpha, beta)
    n = len(probs)
    variants = [mm.grouped_default_variant(p[0], p[1], p[2]) for p in probs]
    variants[3] = 1 - variants[3]          # exercise both shapes on one problem each
    ws_bytes = mm.grouped_gemm_workspace_bytes(n)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    mm.grouped_gemm(arr, n, mm.PATH_3XBF16, variants, ws, ws_bytes)
    torch.cuda.synchronize()
    for t, ((M, N, K, A, B, C0), d) in enumerate(zip(probs, dev)):
        if M == 0 or N == 0:
            continue
        C = d[7].cpu().numpy()
        if K == 0:
            assert np.array_equal(C, (np.float32(beta) * C0).astype(np.float32) if beta else 0 * C0)
            continue
        check_split_result(oracle, A, B, C0, C, alpha, beta, 3)
        solo = torch.from_numpy(C0).cuda()
        cfg = _cfg_index(mm, SOLO_CFG[variants[t]])
        mm.gemm_run_config(mm.PATH_3XBF16, cfg, M, N, K, alpha, d[3], d[4], d[5], d[6], beta,
                           solo, N, n_products=3)
        torch.cuda.synchronize()
        assert np.array_equal(solo.cpu().numpy(), C), (t, M, N, K)


def test_graph_replays_match_eager():
    import torch
    import paper_1902_10345_amd as mm
    probs = _problems(seed=6, count=24)
    dev, arr = _to_device(probs, 1.0, 0.0)
    n = len(probs)
    ws_bytes = mm.grouped_gemm_workspace_bytes(n)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    mm.grouped_gemm(arr, n, mm.PATH_3XBF16, None, ws, ws_bytes)
    torch.cuda.synchronize()
    eager = [d[7].cpu().numpy().copy() for d in dev]
    g = mm.grouped_graph_create(arr, n, mm.PATH_3XBF16, None, ws, ws_bytes)
    try:
        for rep in range(4):
            for d in dev:           # eager work between replays
                d[7].fill_(float("nan"))
            torch.cuda.synchronize()
            mm.grouped_graph_launch(g)
            torch.cuda.synchronize()
            for t, d in enumerate(dev):
                assert np.array_equal(d[7].cpu().numpy(), eager[t]), (rep, t)
    finally:
        mm.grouped_graph_destroy(g)


def test_full_batch_512_sampled_members():
    """The 512-problem batch (M, N, K log-uniform in [32, 1024], multiples of
    16) in one launch; 48 seeded members are checked against the oracle."""
    import torch
    import paper_1902_10345_amd as mm
    sizes = si.log_uniform_sizes(512, 32, 1024, 5, 16)
    g = np.random.default_rng(55)
    check = set(g.choice(512, size=48, replace=False).tolist())
    host, dev = {}, []
    for t, (M, N, K) in enumerate(sizes):
        M, N, K = int(M), int(N), int(K)
        if t in check:
            A = si.uniform((M, K), 100003 * 5 + 2 * t)
            B = si.uniform((K, N), 100003 * 5 + 2 * t + 1)
            host[t] = (A, B)
            dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
        else:
            dA = torch.rand(M, K, device="cuda") * 2 - 1
            dB = torch.rand(K, N, device="cuda") * 2 - 1
        dC = torch.empty(M, N, device="cuda")
        dev.append((M, N, K, dA, K, dB, N, dC, N, 1.0, 0.0))
    arr = mm.problem_array(dev)
    ws_bytes = mm.grouped_gemm_workspace_bytes(512)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    mm.grouped_gemm(arr, 512, mm.PATH_3XBF16, None, ws, ws_bytes)
    torch.cuda.synchronize()
    for t in sorted(check):
        A, B = host[t]
        check_split_result(oracle, A, B, None, dev[t][7].cpu().numpy(), 1.0, 0.0, 3)


def test_invalid_member_is_rejected_before_enqueue():
    import torch
    import paper_1902_10345_amd as mm
    probs = _problems(seed=7, count=3)
    dev, arr = _to_device(probs, 1.0, 0.0)
    arr[1].lda = 0
    ws = torch.empty(mm.grouped_gemm_workspace_bytes(3), dtype=torch.uint8, device="cuda")
    with pytest.raises(mm.GemmError) as e:
        mm.grouped_gemm(arr, 3, mm.PATH_3XBF16, None, ws, ws.numel())
    assert e.value.status == -1 and "problems[1]" in e.value.message


def test_large_batch_prefix_search_in_global_memory_and_mixed_schedule():
    """More problems than the kernel's LDS copy of the tile prefix holds
    (3500 > 3072): the owning problem is found by binary search in global
    memory.  With several rounds of tiles the first rounds are dealt
    round-robin and the rest dequeued from the counter; every tile must be
    computed exactly once."""
    import torch
    import paper_1902_10345_amd as mm
    count = 3500
    g = np.random.default_rng(77)
    sizes = [(int(g.integers(1, 70)), int(g.integers(1, 70)), int(g.integers(1, 90))) for _ in range(count)]
    sizes[17] = (300, 260, 200)   # a few multi-tile members among the small ones
    sizes[2000] = (130, 700, 64)
    probs = []
    for t, (M, N, K) in enumerate(sizes):
        probs.append([M, N, K, si.integers((M, K), 10 * t), si.integers((K, N), 10 * t + 1),
                      si.integers((M, N), 10 * t + 2)])
    dev, arr = _to_device(probs, 2.0, -1.0)
    ws_bytes = mm.grouped_gemm_workspace_bytes(count)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    for rep in range(2):   # the counter must be re-armed by each launch
        for (M, N, K, dA, lda, dB, ldb, dC, ldc, a, b), (_, _, _, _, _, C0) in zip(dev, probs):
            dC.copy_(torch.from_numpy(C0))
        mm.grouped_gemm(arr, count, mm.PATH_3XBF16, None, ws, ws_bytes)
        torch.cuda.synchronize()
        for (M, N, K, A, B, C0), d in zip(probs, dev):
            got = d[7].cpu().numpy().astype(np.float64)
            # integer inputs in [-8, 8]: exact on both split planes
            assert np.array_equal(got, oracle.gemm(A, B, alpha=2.0, beta=-1.0, C0=C0)), (M, N, K, rep)
