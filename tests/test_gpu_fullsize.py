"""Full-matrix parity at the paper-scale workloads: every element of C against
the binary64 oracle (all host threads), in the launch configuration the
benchmark times -- the 4096^3 and 8192x2048x4096 products (alpha 1.5,
beta 0.5) on the split-precision path (three and six products) and the
binary32 path (matrix-core default and the vector-ALU tile), the 4096^3 FP8
product for each outlier variant against the dequantised-input oracle and the
exact one, and every member of the 512-problem grouped batch.  The device
error norm (binary64 reduction on the GPU) is checked against the oracle's at
full size too.  Each test prints its errors, which the benchmark reports."""
import functools

import numpy as np
import pytest

import oracle
import seeded_inputs as si
from gpu_util import DROPPED, check_split_result, fp8_check, gamma

pytestmark = pytest.mark.gpu

WORKLOADS = [(4096, 4096, 4096, 2), (8192, 2048, 4096, 3)]


@functools.lru_cache(maxsize=2)
def _dense(M, N, K, seed):
    """Seeded operands (the benchmark's draws) and the oracle's Cref and
    componentwise denominator, alpha 1.5, beta 0.5."""
    A = si.uniform((M, K), seed)
    B = si.uniform((K, N), seed + 100)
    C0 = si.uniform((M, N), seed + 200)
    ref = oracle.gemm(A, B, alpha=1.5, beta=0.5, C0=C0)
    den = oracle.gemm_abs(A, B, alpha=1.5, beta=0.5, C0=C0)
    return A, B, C0, ref, den


def _run_dense(M, N, K, seed, call):
    import torch
    A, B, C0, ref, den = _dense(M, N, K, seed)
    dA, dB, dC = (torch.from_numpy(x).cuda() for x in (A, B, C0))
    call(dA, dB, dC)
    torch.cuda.synchronize()
    return dC, ref, den


def _device_norms(dC, ref, den):
    import torch
    import paper_1902_10345_amd as mm
    return mm.ops.err_norm(dC, torch.from_numpy(ref).cuda(), torch.from_numpy(den).cuda())


@pytest.mark.parametrize("n", [3, 6])
@pytest.mark.parametrize("M,N,K,seed", WORKLOADS)
def test_split_precision_full_matrix(M, N, K, seed, n):
    import paper_1902_10345_amd as mm
    dC, ref, den = _run_dense(M, N, K, seed, lambda dA, dB, dC: mm.gemm_f32_3xbf16(
        M, N, K, 1.5, dA, K, dB, N, 0.5, dC, N, n))
    C = dC.cpu().numpy()
    rel, _, _, cw = oracle.norms(C, ref, den)
    print("3xbf16 n=%d %dx%dx%d full matrix: rel_fro %.3e componentwise %.3e"
          % (n, M, N, K, rel, cw))
    assert rel <= 1e-5, rel
    assert cw <= DROPPED[n] + 2 * 1.01 * gamma(n * K), cw
    # the device norm agrees with the oracle's over all M*N elements
    drel, dnum, dref, dcw = _device_norms(dC, ref, den)
    assert abs(drel - rel) <= 1e-9 * rel and dcw == cw


@pytest.mark.parametrize("which", ["default", "valu"])
@pytest.mark.parametrize("M,N,K,seed", WORKLOADS)
def test_fp32_full_matrix(M, N, K, seed, which):
    """The binary32 path: the library's default (FP32 matrix-core tile at
    these shapes) and the vector-ALU tile the benchmark times beside it."""
    import paper_1902_10345_amd as mm
    if which == "default":
        call = lambda dA, dB, dC: mm.gemm_f32(M, N, K, 1.5, dA, K, dB, N, 0.5, dC, N)  # noqa: E731
    else:
        cfg = [c for c in range(mm.gemm_num_configs(mm.PATH_F32))
               if mm.gemm_config_name(mm.PATH_F32, c) == "f32_128x128x32_r8x8_u2"][0]
        call = lambda dA, dB, dC: mm.gemm_run_config(  # noqa: E731
            mm.PATH_F32, cfg, M, N, K, 1.5, dA, K, dB, N, 0.5, dC, N)
    dC, ref, den = _run_dense(M, N, K, seed, call)
    rel, _, _, cw = oracle.norms(dC.cpu().numpy(), ref, den)
    print("f32 %s %dx%dx%d full matrix: rel_fro %.3e componentwise %.3e (%.2f gamma_K)"
          % (which, M, N, K, rel, cw, cw / gamma(K)))
    assert rel <= 1e-5, rel
    assert cw <= gamma(K), cw


@pytest.mark.parametrize("outliers", ["none", "A", "B"])
def test_fp8_full_matrix(outliers):
    """gemm_fp8_scaled at 4096^3 on the seeded N(0,1) workload with 1 % of
    the columns of A (or of B) scaled by 1e3: the whole result against the
    dequantised-input oracle (codes and scales read back from the workspace,
    which the quantiser tests pin bit for bit) within the accumulation and
    group-truncation bound, and against the exact product within the
    quantisation error."""
    import torch
    import paper_1902_10345_amd as mm
    M = N = K = 4096
    A, B, C0 = si.fp8_workload(M, N, K, seed=4, outliers=outliers)
    dA, dB, dC = (torch.from_numpy(x).cuda() for x in (A, B, C0))
    nbytes = mm.gemm_fp8_workspace_bytes(M, N, K)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    mm.gemm_fp8_scaled(M, N, K, 1.5, dA, K, dB, N, 0.5, dC, N, ws, nbytes)
    torch.cuda.synchronize()
    L = mm.fp8_workspace_layout(M, N, K)
    h = ws.cpu().numpy()
    Kp = L["Kp"]
    qa = np.ascontiguousarray(h[L["qa"]:L["qa"] + M * Kp].reshape(M, Kp)[:, :K])
    qb = np.ascontiguousarray(h[L["qb"]:L["qb"] + N * Kp].reshape(N, Kp)[:, :K].T)
    sa = h[L["sa"]:L["sa"] + 4 * M].view(np.float32).copy()
    sb = h[L["sb"]:L["sb"] + 4 * N].view(np.float32).copy()
    C = dC.cpu().numpy()
    rel_q, ratio, cw_q = fp8_check(oracle, C, qa, qb, sa, sb, 1.5, 0.5, C0)
    ref = oracle.gemm(A, B, alpha=1.5, beta=0.5, C0=C0)
    den = oracle.gemm_abs(A, B, alpha=1.5, beta=0.5, C0=C0)
    rel, _, _, cw = oracle.norms(C, ref, den)
    print("fp8 outliers=%s 4096^3 full matrix: vs dequantised oracle rel_fro %.3e "
          "componentwise %.3e (%.3f of the bound); vs exact rel_fro %.3e componentwise %.3e"
          % (outliers, rel_q, cw_q, ratio, rel, cw))
    assert ratio <= 1.0, ratio
    assert rel <= 0.08 and cw <= 0.08, (rel, cw)


def test_grouped_all_512_members():
    """The 512-problem batch (M, N, K log-uniform in [32, 1024], multiples of
    16, seed 5: the benchmark's batch) in one launch; every member against the
    oracle."""
    import torch
    import paper_1902_10345_amd as mm
    probs = si.grouped_problems(512, seed=5)
    dev = []
    for (M, N, K, A, B) in probs:
        dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
        dC = torch.full((M, N), float("nan"), device="cuda")
        dev.append((M, N, K, dA, K, dB, N, dC, N, 1.0, 0.0))
    arr = mm.problem_array(dev)
    ws_bytes = mm.grouped_gemm_workspace_bytes(512)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    mm.grouped_gemm(arr, 512, mm.PATH_3XBF16, None, ws, ws_bytes)
    torch.cuda.synchronize()
    worst = 0.0
    for (M, N, K, A, B), d in zip(probs, dev):
        rel = check_split_result(oracle, A, B, None, d[7].cpu().numpy(), 1.0, 0.0, 3)
        worst = max(worst, rel)
    print("grouped 512 members: worst rel_fro %.3e" % worst)
