"""The autotuner on the GPU (size-specific tuning of the tile parameters, the
paper's last step of its matrix-multiplication chain, Sec. 6.2):
gemm_autotune times every configuration of a path on the caller's operands,
and afterwards the entry points run the winner for every shape of its size
bucket -- the tuned call returns the winning configuration's bits and meets
the oracle's bounds; grouped_autotune's per-problem tile shapes give
oracle-correct members, bitwise equal to solo runs of the same tile body, and
its winning rule becomes the library's choice; the tuned table survives a
save / load round trip on the device's library."""
import numpy as np
import pytest

import oracle
import seeded_inputs as si
from gpu_util import check_split_result, fp8_check, gamma

pytestmark = pytest.mark.gpu

SOLO_CFG = {0: "bx3_128x128x32_4w64x64_p3", 1: "bx3_64x64x32_4w32x32_p3"}

# (kind, n_products); one shape per path whose size bucket is (2^10, 2^10, 2^10)
CASES = [("f32", 0), ("3xbf16", 3), ("3xbf16", 6), ("fp8", 0)]
SHAPE = (700, 520, 600)
SAME_BUCKET = (600, 1000, 900)


@pytest.fixture(autouse=True)
def _fresh_tuner():
    import paper_1902_10345_amd as mm
    mm.gemm_tuner_clear()
    yield
    mm.gemm_tuner_clear()


def _path(mm, kind):
    return {"f32": mm.PATH_F32, "3xbf16": mm.PATH_3XBF16, "fp8": mm.PATH_FP8}[kind]


def _entry(mm, kind, n, M, N, K, dA, dB, dC, ws, nbytes):
    if kind == "f32":
        mm.gemm_f32(M, N, K, 1.5, dA, K, dB, N, 0.5, dC, N)
    elif kind == "3xbf16":
        mm.gemm_f32_3xbf16(M, N, K, 1.5, dA, K, dB, N, 0.5, dC, N, n)
    else:
        mm.gemm_fp8_scaled(M, N, K, 1.5, dA, K, dB, N, 0.5, dC, N, ws, nbytes)


@pytest.mark.parametrize("kind,n", CASES)
def test_autotuned_choice_is_used_and_correct(kind, n):
    import torch
    import paper_1902_10345_amd as mm
    path = _path(mm, kind)
    M, N, K = SHAPE
    if kind == "fp8":
        A, B, C0 = si.fp8_workload(M, N, K, seed=21, outliers="A")
    else:
        A, B, C0 = si.uniform((M, K), 21), si.uniform((K, N), 22), si.uniform((M, N), 23)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    nbytes = mm.gemm_fp8_workspace_bytes(M, N, K) if kind == "fp8" else 0
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device="cuda") if nbytes else None
    scratch = torch.from_numpy(C0).cuda()
    best = mm.gemm_autotune(path, M, N, K, 1.5, dA, K, dB, N, 0.5, scratch, N, n_products=max(n, 3),
                            workspace=ws, ws_bytes=nbytes, reps=2)
    torch.cuda.synchronize()
    assert 0 <= best < mm.gemm_num_configs(path)
    name = mm.gemm_config_name(path, best)
    print("autotune %s n=%d %dx%dx%d -> %s" % (kind, n, M, N, K, name))
    if kind != "3xbf16" or n == 3:     # gemm_default_config reports the 3-product choice
        assert mm.gemm_default_config(path, M, N, K) == best
        assert mm.gemm_default_config(path, *SAME_BUCKET) == best
    # the entry point now runs the winner: same bits as the explicit configuration
    dC = torch.from_numpy(C0).cuda()
    _entry(mm, kind, n, M, N, K, dA, dB, dC, ws, nbytes)
    dR = torch.from_numpy(C0).cuda()
    mm.gemm_run_config(path, best, M, N, K, 1.5, dA, K, dB, N, 0.5, dR, N, n_products=max(n, 3),
                       workspace=ws, ws_bytes=nbytes)
    torch.cuda.synchronize()
    C = dC.cpu().numpy()
    assert np.array_equal(C, dR.cpu().numpy())
    # and the tuned result meets the path's bounds against the oracle
    if kind == "f32":
        ref = oracle.gemm(A, B, alpha=1.5, beta=0.5, C0=C0)
        den = oracle.gemm_abs(A, B, alpha=1.5, beta=0.5, C0=C0)
        rel, _, _, cw = oracle.norms(C, ref, den)
        assert rel <= 1e-5 and cw <= gamma(K), (rel, cw)
    elif kind == "3xbf16":
        check_split_result(oracle, A, B, C0, C, 1.5, 0.5, n)
    else:
        sa, sb = oracle.fp8_scales_rows(A), oracle.fp8_scales_cols(B)
        qa, qb = oracle.fp8_quantize_rows(A, sa), oracle.fp8_quantize_cols(B, sb)
        assert fp8_check(oracle, C, qa, qb, sa, sb, 1.5, 0.5, C0)[1] <= 1.0


def test_tuned_table_round_trip_on_the_device(tmp_path):
    """A tuned choice saved to JSON, cleared and loaded back is again the
    library's choice for the bucket, and the entry point runs it."""
    import torch
    import paper_1902_10345_amd as mm
    M, N, K = SHAPE
    A, B, C0 = si.uniform((M, K), 31), si.uniform((K, N), 32), si.uniform((M, N), 33)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    scratch = torch.from_numpy(C0).cuda()
    best = mm.gemm_autotune(mm.PATH_3XBF16, M, N, K, 1.5, dA, K, dB, N, 0.5, scratch, N,
                            n_products=3, reps=2)
    path = tmp_path / "tuned.json"
    mm.gemm_tuner_save(str(path))
    mm.gemm_tuner_clear()
    mm.gemm_tuner_load(str(path))
    assert mm.gemm_default_config(mm.PATH_3XBF16, M, N, K) == best
    dC = torch.from_numpy(C0).cuda()
    mm.gemm_f32_3xbf16(M, N, K, 1.5, dA, K, dB, N, 0.5, dC, N, 3)
    dR = torch.from_numpy(C0).cuda()
    mm.gemm_run_config(mm.PATH_3XBF16, best, M, N, K, 1.5, dA, K, dB, N, 0.5, dR, N, n_products=3)
    torch.cuda.synchronize()
    assert np.array_equal(dC.cpu().numpy(), dR.cpu().numpy())


def test_grouped_autotune_variants_are_correct_and_become_the_default():
    import torch
    import paper_1902_10345_amd as mm
    probs = si.grouped_problems(96, seed=8, lo=32, hi=1024)
    dev = []
    for (M, N, K, A, B) in probs:
        dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
        dev.append((M, N, K, dA, K, dB, N, torch.empty((M, N), device="cuda"), N, 1.0, 0.0))
    arr = mm.problem_array(dev)
    n = len(probs)
    ws_bytes = mm.grouped_gemm_workspace_bytes(n)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    variants = mm.grouped_autotune(arr, n, mm.PATH_3XBF16, ws, ws_bytes, reps=2)
    assert len(variants) == n and set(variants) <= {0, 1}
    print("grouped_autotune: %d of %d problems on 64x64 tiles" % (sum(variants), n))
    # the winning rule is now the library's choice for these problems
    assert [mm.grouped_default_variant(M, N, K) for (M, N, K, _, _) in probs] == variants
    for d in dev:
        d[7].fill_(float("nan"))
    mm.grouped_gemm(arr, n, mm.PATH_3XBF16, variants, ws, ws_bytes)
    torch.cuda.synchronize()
    cfg_of = {v: [c for c in range(mm.gemm_num_configs(mm.PATH_3XBF16))
                  if mm.gemm_config_name(mm.PATH_3XBF16, c) == SOLO_CFG[v]][0] for v in (0, 1)}
    for t, ((M, N, K, A, B), d) in enumerate(zip(probs, dev)):
        C = d[7].cpu().numpy()
        check_split_result(oracle, A, B, None, C, 1.0, 0.0, 3)
        if t % 8 == 0:  # bitwise against the same tile body run alone
            solo = torch.empty((M, N), device="cuda")
            mm.gemm_run_config(mm.PATH_3XBF16, cfg_of[variants[t]], M, N, K, 1.0, d[3], K, d[5],
                               N, 0.0, solo, N, n_products=3)
            torch.cuda.synchronize()
            assert np.array_equal(solo.cpu().numpy(), C), (t, M, N, K)
