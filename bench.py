"""Benchmark of the MI355X GEMM library (one GPU).

Headline step: one FP32-accurate GEMM C <- 1.5*A*B + 0.5*C at M = N = K = 4096
(binary32 row-major operands, uniform[-1,1), inputs resident in HBM) on the
3xBF16 split-precision MFMA path.  The plain FP32 vector-ALU kernel, the
6-product variant, the rectangular 8192x2048x4096 case, the scaled FP8 path,
the grouped batch and the serving loop are measured beside it.

Prints ONE JSON line.  Throughput counts 2*M*N*K algorithmic flops per GEMM
(never padded tile work, never the extra split products).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
    python bench.py --profile     # a few headline launches + a 1 GiB copy, for rocprofv3
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published dense peaks (TFLOP/s) and HBM bandwidth (GB/s).
PEAK_BF16_MFMA = 2516.6
PEAK_FP8_MFMA = 5033.2
PEAK_FP32_VALU = 157.3
PEAK_FP64_MFMA = 78.6
PEAK_HBM_GBS = 8000.0


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def _dev_inputs(M, N, K, seed, torch):
    import seeded_inputs as si
    A = si.uniform((M, K), seed)
    B = si.uniform((K, N), seed + 100)
    C0 = si.uniform((M, N), seed + 200)
    return (A, B, C0), tuple(torch.from_numpy(x).cuda() for x in (A, B, C0))


def _sclk_mhz():
    """The engine clock's current DPM level from sysfs (None if unreadable).
    Under MFMA load the power limit holds the clock below its 2.4 GHz peak."""
    import glob
    for f in sorted(glob.glob("/sys/class/drm/card*/device/pp_dpm_sclk")):
        try:
            for line in open(f):
                if "*" in line:
                    return int("".join(ch for ch in line.split(":")[1] if ch.isdigit()))
        except (OSError, ValueError, IndexError):
            continue
    return None


def _settle(fn, seconds, torch):
    """Run fn untimed for about `seconds`: the engine clock ramps up over
    roughly a second of sustained load, longer than the warm-up steps."""
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(20):
            fn()
        torch.cuda.synchronize()


def _time_steps(fn, steps, warmup, torch):
    """Run `fn` warmup times, then time exactly `steps` calls on the current
    stream.  Returns (ms_per_step from the block, per-step list in ms)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record()
    for i in range(steps):
        fn()
        ev[i + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    block = ev[0].elapsed_time(ev[-1]) / steps
    return block, per, wall


def _time_graph(fn, launches, steps, torch):
    """Capture `launches` calls of `fn` in one graph and time `steps` replays
    with events; returns (ms per launch, per-replay list in ms per launch)."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(launches):
            fn()
    g.replay()
    torch.cuda.synchronize()
    per = []
    for _ in range(steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        g.replay()
        e1.record()
        torch.cuda.synchronize()
        per.append(e0.elapsed_time(e1) / launches)
    del g
    return statistics.median(per), per


def _stats(per):
    """Median and a 95% confidence interval of the median (order statistics)
    plus Tukey-fence outlier count, as in the paper's timing methodology."""
    s = sorted(per)
    n = len(s)
    med = statistics.median(s)
    # distribution-free CI for the median: ranks n/2 -+ 1.96 sqrt(n)/2
    half = 1.96 * math.sqrt(n) / 2
    lo = s[max(0, int(math.floor(n / 2 - half)))]
    hi = s[min(n - 1, int(math.ceil(n / 2 + half)) - 1)]
    q1, q3 = s[n // 4], s[(3 * n) // 4]
    iqr = q3 - q1
    out = sum(1 for v in s if v < q1 - 1.5 * iqr or v > q3 + 1.5 * iqr)
    return {"median_ms": round(med, 5), "ci95_ms": [round(lo, 5), round(hi, 5)],
            "tukey_outliers": out}


def _traffic(kernel):
    """HBM bytes per launch measured by rocprofv3 (FETCH_SIZE + WRITE_SIZE,
    calibrated against a copy of known size), read from profiles/; None when
    the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(kernel)
    except Exception:
        return None
    if not rec:
        return None
    if rec.get("source_sha") != _source_sha(rec.get("sources", [])):
        return None
    return rec.get("bytes_per_launch")


def _source_sha(files):
    h = hashlib.sha256()
    for f in files:
        p = os.path.join(ROOT, f)
        if not os.path.exists(p):
            return None
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def run_grouped(torch, mm, steps, warmup):
    """512 problems, M, N, K log-uniform in [32, 1024] (multiples of 16), one
    persistent launch captured in a HIP graph, tile shapes from the autotuner."""
    import numpy as np
    import seeded_inputs as si
    probs = si.grouped_problems(512, seed=5)
    dev, flops, min_bytes = [], 0.0, 0.0
    for (M, N, K, A, B) in probs:
        dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
        dC = torch.empty((M, N), dtype=torch.float32, device="cuda")
        dev.append((M, N, K, dA, K, dB, N, dC, N, 1.0, 0.0))
        flops += 2.0 * M * N * K
        min_bytes += 4.0 * (M * K + K * N + M * N)
    arr = mm.problem_array(dev)
    ws_bytes = mm.grouped_gemm_workspace_bytes(len(dev))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    variants = mm.grouped_autotune(arr, len(dev), mm.PATH_3XBF16, ws, ws_bytes, reps=3)
    g = mm.grouped_graph_create(arr, len(dev), mm.PATH_3XBF16, variants, ws, ws_bytes)
    try:
        ms, per, _ = _time_steps(lambda: mm.grouped_graph_launch(g), steps, warmup, torch)
    finally:
        mm.grouped_graph_destroy(g)
    tf = flops / (ms * 1e-3) / 1e12
    gbs = min_bytes / (ms * 1e-3) / 1e9
    n128 = int(sum(1 for v in variants if v == 0))
    torch.cuda.synchronize()
    outputs = [d[7].cpu().numpy() for d in dev]   # the last replay's results
    return probs, outputs, {"problems": len(dev), "gflop": round(flops / 1e9, 3),
            "min_hbm_mb": round(min_bytes / 1e6, 1), "ms": round(ms, 4),
            "tflops": round(tf, 1), "frac_3product_ceiling": round(tf * 3 / PEAK_BF16_MFMA, 4),
            "hbm_gbs_of_min_bytes": round(gbs, 1), "frac_hbm": round(gbs / PEAK_HBM_GBS, 4),
            "tiles_128x128": n128, "tiles_64x64": len(dev) - n128,
            "launch": "hipGraph replay (counter clear + persistent kernel)", **_stats(per)}


def run_serving(torch, mm, seconds, rate=2000.0):
    """Poisson arrivals at `rate` req/s for `seconds`; each request an
    FP32-accurate GEMM with M, N, K log-uniform in [64, 2048]; admission by a
    16 GB HBM operand budget; operands from a pinned host pool."""
    import collections
    import seeded_inputs as si
    t_arr, sizes = si.serving_requests(rate, seconds, seed=6)
    pool_n = 1 << 26                                 # 256 MB of uniform values
    pool = torch.from_numpy(si.uniform((1, pool_n), 61).reshape(-1)).pin_memory()
    ring_n = 1 << 27                                 # 512 MB pinned output ring
    ring = torch.empty(ring_n, dtype=torch.float32, pin_memory=True)
    budget = 16 << 30
    arena = torch.empty(budget, dtype=torch.uint8, device="cuda")
    srv = mm.server_create(arena, budget, 1024, mm.PATH_3XBF16, 4)
    outstanding = collections.deque()                 # (ticket, ring_off, n, index)
    head = 0
    lat = []
    sample_every = 100                                # every 100th request is kept
    kept = {}                                         # index -> result copy

    def reap():
        """Collect completed requests in submission order."""
        while outstanding:
            r = mm.server_poll(srv, outstanding[0][0])
            if r is None:
                return
            lat.append(r)
            _, off, n, idx = outstanding.popleft()
            if idx % sample_every == 0:
                kept[idx] = ring[off:off + n].numpy().copy()

    def overlaps_oldest(lo, hi):
        return bool(outstanding) and outstanding[0][1] < hi and outstanding[0][1] + outstanding[0][2] > lo

    try:
        time.sleep(0.05)
        base = mm.server_now(srv) + 0.05
        for i, (ta, (M, N, K)) in enumerate(zip(t_arr, sizes)):
            M, N, K = int(M), int(N), int(K)
            due = base + float(ta)
            while mm.server_now(srv) < due:
                pass
            n = M * N
            if head + n > ring_n:
                head = 0
            # ring slots are reused in order: wait for the oldest result that
            # still occupies [head, head + n)
            while overlaps_oldest(head, head + n):
                reap()
                if overlaps_oldest(head, head + n):
                    time.sleep(20e-6)
            offA = (i * 2654435761) % (pool_n - M * K)
            offB = (i * 40503 + 12345) % (pool_n - K * N)
            hA = pool[offA:offA + M * K]
            hB = pool[offB:offB + K * N]
            hC = ring[head:head + n]
            t = mm.server_submit(srv, M, N, K, 1.0, hA, hB, 0.0, None, hC, due)
            outstanding.append((t, head, n, i))
            head += n
            if i % 8 == 0:
                reap()
        mm.server_drain(srv, 120.0)
        reap()
        st = mm.server_stats(srv)
    finally:
        mm.server_destroy(srv)
    del arena
    offered = sum(2.0 * float(m) * float(n_) * float(k) for (m, n_, k) in sizes) / seconds
    # the kept 1 % sample, with the operands each request read from the pool
    sample = []
    for idx in sorted(kept):
        M, N, K = (int(v) for v in sizes[idx])
        offA = (idx * 2654435761) % (pool_n - M * K)
        offB = (idx * 40503 + 12345) % (pool_n - K * N)
        A = pool[offA:offA + M * K].numpy().reshape(M, K)
        B = pool[offB:offB + K * N].numpy().reshape(K, N)
        sample.append((A, B, kept[idx].reshape(M, N)))
    return sample, {"rate_req_s": rate, "seconds": seconds, "requests": int(len(t_arr)),
            "p50_ms": round(st["p50_ms"], 4), "p99_ms": round(st["p99_ms"], 4),
            "result_p50_ms": round(st["result_p50_ms"], 4),
            "result_p99_ms": round(st["result_p99_ms"], 4),
            "tflops": round(st["tflops"], 3), "offered_tflops": round(offered / 1e12, 3),
            "completed": st["completed"], "failed": st["failed"],
            "max_in_flight": st["max_in_flight"],
            "max_concurrent_steps": st["max_concurrent_steps"],
            "arena_high_water_mb": round(st["arena_high_water_bytes"] / 1e6, 1),
            "budget_gb": budget / (1 << 30), "streams": 4, "slots": 1024}


def run_profile(torch, mm):
    """Launches of every timed kernel and a 1 GiB copy (the calibration of the
    byte counters), for rocprofv3 counter runs."""
    M = N = K = 4096
    _, (A, B, C) = _dev_inputs(M, N, K, 2, torch)
    valu = [c for c in range(mm.gemm_num_configs(mm.PATH_F32))
            if mm.gemm_config_name(mm.PATH_F32, c) == "f32_128x128x32_r8x8_u2"][0]
    for i in range(5):
        mm.gemm_f32_3xbf16(M, N, K, 1.5, A, K, B, N, 0.5, C, N, 3)
        mm.gemm_f32(M, N, K, 1.5, A, K, B, N, 0.5, C, N)
        mm.gemm_run_config(mm.PATH_F32, valu, M, N, K, 1.5, A, K, B, N, 0.5, C, N)
    nbytes = mm.gemm_fp8_workspace_bytes(M, N, K)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    import seeded_inputs as si
    fA, fB, _ = si.fp8_workload(M, N, K, seed=4, outliers="A")
    An, Bn = torch.from_numpy(fA).cuda(), torch.from_numpy(fB).cuda()
    del fA, fB
    for i in range(5):
        mm.fp8_quantize(M, N, K, An, K, Bn, N, ws, nbytes)
    for i in range(5):
        mm.gemm_fp8_prequantized(M, N, K, 1.5, ws, nbytes, 0.5, C, N)
    del An, Bn, ws
    dev = []
    for (Mg, Ng, Kg, Ag, Bg) in si.grouped_problems(512, seed=5):
        dC = torch.empty((Mg, Ng), dtype=torch.float32, device="cuda")
        dev.append((Mg, Ng, Kg, torch.from_numpy(Ag).cuda(), Kg, torch.from_numpy(Bg).cuda(), Ng,
                    dC, Ng, 1.0, 0.0))
    arr = mm.problem_array(dev)
    gws_bytes = mm.grouped_gemm_workspace_bytes(len(dev))
    gws = torch.empty(gws_bytes, dtype=torch.uint8, device="cuda")
    for i in range(5):
        mm.grouped_gemm(arr, len(dev), mm.PATH_3XBF16, None, gws, gws_bytes)
    del dev, arr, gws
    Ad, Bd, Cd = (x.double() for x in (A, B, C))
    for i in range(5):
        mm.gemm_f64(M, N, K, 1.5, Ad, K, Bd, N, 0.5, Cd, N)
    del Ad, Bd, Cd
    ms_, nb_ = 32, 29297
    sz = ms_ * ms_
    Ab, Bb, Cb = (torch.rand(nb_ * sz, device="cuda", dtype=torch.float64) for _ in range(3))
    for i in range(5):
        mm.gemm_f64_strided_batched(ms_, ms_, ms_, 1.0, Ab, ms_, sz, Bb, ms_, sz, 0.0, Cb, ms_, sz,
                                    nb_)
    del Ab, Bb, Cb
    Ab, Bb, Cb = (torch.rand(nb_ * sz, device="cuda") for _ in range(3))
    for path in (mm.PATH_3XBF16, mm.PATH_F32):
        for i in range(5):
            mm.gemm_strided_batched(path, ms_, ms_, ms_, 1.0, Ab, ms_, sz, Bb, ms_, sz, 0.0, Cb, ms_,
                                    sz, nb_, 3)
    del Ab, Bb, Cb
    src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    _log("profile run done: 5 x gemm_bx3, gemm_f32 (matrix cores and the vector-ALU tile), "
         "fp8_quantize, gemm_fp8, gemm_f64 (4096^3), "
         "5 x grouped 512, "
         "5 x batched 32^3 x 29297 (binary64, then split precision and binary32), "
         "5 x copy of 1 GiB")


def _threads():
    return int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)


def _err(oracle, C, ref, den):
    rel, _, _, cw = oracle.norms(C, ref, den)
    return {"rel_fro": float("%.4g" % rel), "componentwise_max": float("%.4g" % cw)}


def run_accuracy(torch, mm, head_inputs, grouped_run, serving_sample):
    """Each path's error against the binary64 oracle over the whole result:
    relative Frobenius and componentwise max |dC| / (|alpha||A||B| +
    |beta||C0|).  The oracle runs on all host threads; its times are the CPU
    baseline (the whole 4096^3 headline product) and the per-workload
    detail (all threads, and one thread on a row sample)."""
    import numpy as np
    import oracle
    import seeded_inputs as si
    T = _threads()
    acc, detail = {}, {"threads": T}

    def timed(fn):
        t0 = time.perf_counter()
        r = fn()
        return r, time.perf_counter() - t0

    def one_thread(A, B, C0, alpha, beta, rows):
        sel = np.linspace(0, A.shape[0] - 1, rows).astype(np.int64)
        _, dt = timed(lambda: oracle.gemm(A[sel], B, alpha=alpha, beta=beta,
                                          C0=None if C0 is None else C0[sel], nthreads=1))
        return {"rows": rows, "s": round(dt, 3),
                "gflops": round(2.0 * rows * A.shape[1] * B.shape[1] / dt / 1e9, 3)}

    def dense(tag, M, N, K, seed, alpha, beta, runs, hin=None):
        if hin is None:
            hin = (si.uniform((M, K), seed), si.uniform((K, N), seed + 100),
                   si.uniform((M, N), seed + 200))
        A, B, C0 = hin
        _log("accuracy: oracle %s (%d threads)" % (tag, T))
        ref, dt = timed(lambda: oracle.gemm(A, B, alpha=alpha, beta=beta, C0=C0, nthreads=T))
        den = oracle.gemm_abs(A, B, alpha=alpha, beta=beta, C0=C0, nthreads=T)
        detail[tag] = {"all_threads_s": round(dt, 3),
                       "all_threads_gflops": round(2.0 * M * N * K / dt / 1e9, 2),
                       "one_thread": one_thread(A, B, C0, alpha, beta, min(M, 64))}
        dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
        for name, call in runs:
            dC = torch.from_numpy(C0).cuda()
            call(dA, dB, dC)
            torch.cuda.synchronize()
            acc[name] = _err(oracle, dC.cpu().numpy(), ref, den)
        return dt

    valu = [c for c in range(mm.gemm_num_configs(mm.PATH_F32))
            if mm.gemm_config_name(mm.PATH_F32, c) == "f32_128x128x32_r8x8_u2"][0]

    def runs_for(tag, M, N, K, alpha, beta, valu_too):
        r = [("3xbf16_n3_" + tag, lambda a, b, c: mm.gemm_f32_3xbf16(M, N, K, alpha, a, K, b, N,
                                                                     beta, c, N, 3)),
             ("3xbf16_n6_" + tag, lambda a, b, c: mm.gemm_f32_3xbf16(M, N, K, alpha, a, K, b, N,
                                                                     beta, c, N, 6)),
             ("f32_" + tag, lambda a, b, c: mm.gemm_f32(M, N, K, alpha, a, K, b, N, beta, c, N))]
        if valu_too:
            r.append(("f32_valu_" + tag, lambda a, b, c: mm.gemm_run_config(
                mm.PATH_F32, valu, M, N, K, alpha, a, K, b, N, beta, c, N)))
        return r

    t_head = dense("4096^3", 4096, 4096, 4096, 2, 1.5, 0.5,
                   runs_for("4096^3", 4096, 4096, 4096, 1.5, 0.5, True), head_inputs)
    dense("8192x2048x4096", 8192, 2048, 4096, 3, 1.5, 0.5,
          runs_for("8192x2048x4096", 8192, 2048, 4096, 1.5, 0.5, True))
    dense("256^3", 256, 256, 256, 1, 1.0, 0.0, runs_for("256^3", 256, 256, 256, 1.0, 0.0, False))
    cpu = {"value": round(2.0 * 4096 ** 3 / t_head / 1e12, 6), "unit": "TFLOP/s", "cores": T,
           "kind": "oracle",
           "sample": "the whole 4096^3 headline product (alpha=1.5, beta=0.5), FP64 i-k-j "
                     "loop over all rows, %.1f s on %d threads" % (t_head, T)}

    # FP8 at 4096^3 for the three outlier variants: against the dequantised
    # oracle (codes and scales read back) and against the exact product
    M = N = K = 4096
    nbytes = mm.gemm_fp8_workspace_bytes(M, N, K)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    L = mm.fp8_workspace_layout(M, N, K)
    for outl in ("none", "A", "B"):
        A, B, C0 = si.fp8_workload(M, N, K, seed=4, outliers=outl)
        dA, dB, dC = (torch.from_numpy(x).cuda() for x in (A, B, C0))
        mm.gemm_fp8_scaled(M, N, K, 1.5, dA, K, dB, N, 0.5, dC, N, ws, nbytes)
        torch.cuda.synchronize()
        C = dC.cpu().numpy()
        h = ws.cpu().numpy()
        Kp = L["Kp"]
        qa = np.ascontiguousarray(h[L["qa"]:L["qa"] + M * Kp].reshape(M, Kp)[:, :K])
        qb = np.ascontiguousarray(h[L["qb"]:L["qb"] + N * Kp].reshape(N, Kp)[:, :K].T)
        sa = h[L["sa"]:L["sa"] + 4 * M].view(np.float32).copy()
        sb = h[L["sb"]:L["sb"] + 4 * N].view(np.float32).copy()
        _log("accuracy: oracle fp8 outliers=%s" % outl)
        refq, dtq = timed(lambda: oracle.gemm_fp8_dequant(qa, sa, qb, sb, alpha=1.5, beta=0.5,
                                                          C0=C0, nthreads=T))
        denq = oracle.gemm_fp8_dequant(qa & 0x7F, sa, qb & 0x7F, sb, alpha=1.5, beta=0.5,
                                       C0=np.abs(C0), nthreads=T)
        ref = oracle.gemm(A, B, alpha=1.5, beta=0.5, C0=C0, nthreads=T)
        den = oracle.gemm_abs(A, B, alpha=1.5, beta=0.5, C0=C0, nthreads=T)
        acc["fp8_4096^3_outliers_" + outl] = {"vs_exact": _err(oracle, C, ref, den),
                                              "vs_dequantised": _err(oracle, C, refq, denq)}
        if outl == "A":
            detail["fp8_dequant_4096^3"] = {"all_threads_s": round(dtq, 3)}
        del A, B, C0, dA, dB, dC, refq, denq, ref, den
    del ws

    if grouped_run is not None:
        probs, outputs = grouped_run
        _log("accuracy: oracle on all 512 grouped problems")
        worst_rel = worst_cw = 0.0
        t0 = time.perf_counter()
        for (Mg, Ng, Kg, A, B), C in zip(probs, outputs):
            ref = oracle.gemm(A, B, nthreads=T)
            den = oracle.gemm_abs(A, B, nthreads=T)
            rel, _, _, cw = oracle.norms(C, ref, den)
            worst_rel, worst_cw = max(worst_rel, rel), max(worst_cw, cw)
        acc["grouped_512_max_over_members"] = {"rel_fro": float("%.4g" % worst_rel),
                                               "componentwise_max": float("%.4g" % worst_cw)}
        gfl = sum(2.0 * p[0] * p[1] * p[2] for p in probs) / 1e9
        detail["grouped_512_all_problems"] = {
            "s_including_abs_pass": round(time.perf_counter() - t0, 3), "gflop": round(gfl, 2)}

    if serving_sample:
        _log("accuracy: oracle on the %d-request serving sample" % len(serving_sample))
        worst_rel = worst_cw = 0.0
        t0 = time.perf_counter()
        fl = 0.0
        for (A, B, C) in serving_sample:
            ref = oracle.gemm(A, B, nthreads=T)
            fl += 2.0 * A.shape[0] * A.shape[1] * B.shape[1]
            den = oracle.gemm_abs(A, B, nthreads=T)
            rel, _, _, cw = oracle.norms(C, ref, den)
            worst_rel, worst_cw = max(worst_rel, rel), max(worst_cw, cw)
        acc["serving_1pct_sample_max"] = {"requests": len(serving_sample),
                                          "rel_fro": float("%.4g" % worst_rel),
                                          "componentwise_max": float("%.4g" % worst_cw)}
        detail["serving_1pct_sample"] = {"s_including_abs_pass": round(time.perf_counter() - t0, 3),
                                         "gflop": round(fl / 1e9, 2)}
    return cpu, detail, acc


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-grouped", action="store_true")
    ap.add_argument("--settle-seconds", type=float, default=1.0,
                    help="untimed run of the headline GEMM before its warm-up (clock ramp)")
    ap.add_argument("--headline-only", action="store_true",
                    help="time only the headline GEMM (for kernel-trace profiles)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(sharding is a design note). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1902_10345_amd as mm
    torch.cuda.set_device(0)
    if args.profile:
        run_profile(torch, mm)
        return

    K_, W_ = args.steps, args.warmup
    paths = {}

    # ---------------- headline: 4096^3 FP32-accurate on 3xBF16 MFMA --------
    M = N = K = 4096
    flops = 2.0 * M * N * K
    (hA, hB, hC0), (A, B, C) = _dev_inputs(M, N, K, 2, torch)
    _log("headline: gemm_f32_3xbf16 %dx%dx%d n_products=3" % (M, N, K))
    head = lambda: mm.gemm_f32_3xbf16(M, N, K, 1.5, A, K, B, N, 0.5, C, N, 3)  # noqa: E731
    _settle(head, args.settle_seconds, torch)
    ms, per, wall = _time_steps(head, K_, W_, torch)
    sclk = _sclk_mhz()
    head_tflops = flops / (ms * 1e-3) / 1e12
    paths["3xbf16_n3_4096^3"] = {"ms": round(ms, 4), "tflops": round(head_tflops, 1),
                                "frac_bf16_peak": round(head_tflops / PEAK_BF16_MFMA, 4),
                                "frac_3product_ceiling": round(head_tflops * 3 / PEAK_BF16_MFMA, 4),
                                "frac_fp32_peak": round(head_tflops / PEAK_FP32_VALU, 3),
                                **_stats(per)}

    if args.headline_only:
        args.no_grouped = args.no_serving = args.no_cpu_baseline = True

    # ---------------- the other paths --------------------------------------
    def one(name, fn, fl, peak, peak_name, graph=False):
        _log("path: " + name)
        extra = {}
        if graph:
            # launches shorter than the host's per-call cost: time a captured
            # graph of 20 launches (device time per launch), and report the
            # per-call time of host-issued launches beside it
            host_ms, _, _ = _time_steps(fn, K_, W_, torch)
            ms_, per_ = _time_graph(fn, 20, K_, torch)
            extra = {"timing": "hipGraph replay of 20 launches, per launch",
                     "host_issued_ms": round(host_ms, 4)}
        else:
            ms_, per_, _ = _time_steps(fn, K_, W_, torch)
        tf = fl / (ms_ * 1e-3) / 1e12
        paths[name] = {"ms": round(ms_, 4), "tflops": round(tf, 1),
                       "frac_" + peak_name: round(tf / peak, 4), **_stats(per_), **extra}

    if not args.headline_only:
        Cf = C.clone()
        one("f32_4096^3", lambda: mm.gemm_f32(M, N, K, 1.5, A, K, B, N, 0.5, Cf, N),
            flops, PEAK_FP32_VALU, "fp32_peak")
        valu = [c for c in range(mm.gemm_num_configs(mm.PATH_F32))
                if mm.gemm_config_name(mm.PATH_F32, c) == "f32_128x128x32_r8x8_u2"][0]
        one("f32_valu_4096^3",
            lambda: mm.gemm_run_config(mm.PATH_F32, valu, M, N, K, 1.5, A, K, B, N, 0.5, Cf, N),
            flops, PEAK_FP32_VALU, "fp32_valu_peak")
        one("3xbf16_n6_4096^3", lambda: mm.gemm_f32_3xbf16(M, N, K, 1.5, A, K, B, N, 0.5, Cf, N, 6),
            flops, PEAK_BF16_MFMA, "bf16_peak")
        # transposed operands (the square buffers read as A^T stored K x M, B^T stored N x K)
        for tag, ta, tb in (("TN", mm.TRANS, mm.NO_TRANS), ("NT", mm.NO_TRANS, mm.TRANS),
                            ("TT", mm.TRANS, mm.TRANS)):
            one("3xbf16_n3_4096^3_" + tag,
                lambda ta=ta, tb=tb: mm.gemm_ex(mm.ROW_MAJOR, ta, tb, M, N, K, 1.5, A, M, B, K, 0.5,
                                                Cf, N, mm.PATH_3XBF16, 3),
                flops, PEAK_BF16_MFMA, "bf16_peak")
        one("f32_4096^3_TN",
            lambda: mm.gemm_ex(mm.ROW_MAJOR, mm.TRANS, mm.NO_TRANS, M, N, K, 1.5, A, M, B, N, 0.5,
                               Cf, N, mm.PATH_F32, 3),
            flops, PEAK_FP32_VALU, "fp32_peak")
        nbytes = mm.gemm_fp8_workspace_bytes(M, N, K)
        ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        import seeded_inputs as si
        fA, fB, _ = si.fp8_workload(M, N, K, seed=4, outliers="A")
        An, Bn = torch.from_numpy(fA).cuda(), torch.from_numpy(fB).cuda()
        del fA, fB
        one("fp8_scaled_4096^3_with_quantize",
            lambda: mm.gemm_fp8_scaled(M, N, K, 1.5, An, K, Bn, N, 0.5, Cf, N, ws, nbytes),
            flops, PEAK_FP8_MFMA, "fp8_peak")
        one("fp8_prequantized_4096^3",
            lambda: mm.gemm_fp8_prequantized(M, N, K, 1.5, ws, nbytes, 0.5, Cf, N),
            flops, PEAK_FP8_MFMA, "fp8_peak")
        # beta = 0 (C write-only), the form a scaled-FP8 library GEMM computes
        one("fp8_prequantized_4096^3_beta0",
            lambda: mm.gemm_fp8_prequantized(M, N, K, 1.5, ws, nbytes, 0.0, Cf, N),
            flops, PEAK_FP8_MFMA, "fp8_peak")
        del An, Bn, ws, Cf
        # binary64 on the FP64 matrix cores, and a batched-strided small-matrix
        # workload (2.0 GFLOP useful: 29 297 products of 32 x 32 x 32)
        Ad, Bd, Cd = (x.double() for x in (A, B, C))
        one("f64_4096^3", lambda: mm.gemm_f64(M, N, K, 1.5, Ad, K, Bd, N, 0.5, Cd, N),
            flops, PEAK_FP64_MFMA, "fp64_peak")
        del Ad, Bd, Cd
        ms_, nb_ = 32, 29297
        gs = torch.Generator(device="cuda").manual_seed(11)
        Ab = torch.rand(nb_ * ms_ * ms_, device="cuda", dtype=torch.float64, generator=gs)
        Bb = torch.rand(nb_ * ms_ * ms_, device="cuda", dtype=torch.float64, generator=gs)
        Cb = torch.rand(nb_ * ms_ * ms_, device="cuda", dtype=torch.float64, generator=gs)
        sz = ms_ * ms_
        one("f64_sbsmm_32x32x32_x%d" % nb_,
            lambda: mm.gemm_f64_strided_batched(ms_, ms_, ms_, 1.0, Ab, ms_, sz, Bb, ms_, sz, 0.0,
                                                Cb, ms_, sz, nb_),
            2.0 * ms_ ** 3 * nb_, PEAK_FP64_MFMA, "fp64_peak")
        paths["f64_sbsmm_32x32x32_x%d" % nb_]["hbm_gbs"] = round(
            3 * 8 * sz * nb_ / (paths["f64_sbsmm_32x32x32_x%d" % nb_]["ms"] * 1e-3) / 1e9, 1)
        del Ab, Bb, Cb
        # the same batch in binary32 on the FP32-accurate split path
        Ab, Bb, Cb = (torch.rand(nb_ * sz, device="cuda", generator=gs) for _ in range(3))
        key = "3xbf16_n3_sbsmm_32x32x32_x%d" % nb_
        one(key, lambda: mm.gemm_strided_batched(mm.PATH_3XBF16, ms_, ms_, ms_, 1.0, Ab, ms_, sz, Bb,
                                                 ms_, sz, 0.0, Cb, ms_, sz, nb_, 3),
            2.0 * ms_ ** 3 * nb_, PEAK_BF16_MFMA, "bf16_peak")
        paths[key]["hbm_gbs"] = round(3 * 4 * sz * nb_ / (paths[key]["ms"] * 1e-3) / 1e9, 1)
        key = "f32_sbsmm_32x32x32_x%d" % nb_
        one(key, lambda: mm.gemm_strided_batched(mm.PATH_F32, ms_, ms_, ms_, 1.0, Ab, ms_, sz, Bb,
                                                 ms_, sz, 0.0, Cb, ms_, sz, nb_, 3),
            2.0 * ms_ ** 3 * nb_, PEAK_FP32_VALU, "fp32_peak")
        paths[key]["hbm_gbs"] = round(3 * 4 * sz * nb_ / (paths[key]["ms"] * 1e-3) / 1e9, 1)
        del Ab, Bb, Cb
        M2, N2, K2 = 8192, 2048, 4096
        _, (A2, B2, C2) = _dev_inputs(M2, N2, K2, 3, torch)
        fl2 = 2.0 * M2 * N2 * K2
        one("f32_8192x2048x4096", lambda: mm.gemm_f32(M2, N2, K2, 1.5, A2, K2, B2, N2, 0.5, C2, N2),
            fl2, PEAK_FP32_VALU, "fp32_peak")
        one("3xbf16_n3_8192x2048x4096",
            lambda: mm.gemm_f32_3xbf16(M2, N2, K2, 1.5, A2, K2, B2, N2, 0.5, C2, N2, 3),
            fl2, PEAK_BF16_MFMA, "bf16_peak")
        del A2, B2, C2
        M3 = 2048
        _, (A3, B3, C3) = _dev_inputs(M3, M3, M3, 7, torch)
        fl3 = 2.0 * M3 ** 3
        one("f32_2048^3", lambda: mm.gemm_f32(M3, M3, M3, 1.0, A3, M3, B3, M3, 0.0, C3, M3),
            fl3, PEAK_FP32_VALU, "fp32_peak")
        one("3xbf16_n3_2048^3",
            lambda: mm.gemm_f32_3xbf16(M3, M3, M3, 1.0, A3, M3, B3, M3, 0.0, C3, M3, 3),
            fl3, PEAK_BF16_MFMA, "bf16_peak")
        del A3, B3, C3
        M4 = 256
        _, (A4, B4, C4) = _dev_inputs(M4, M4, M4, 1, torch)
        one("f32_256^3", lambda: mm.gemm_f32(M4, M4, M4, 1.0, A4, M4, B4, M4, 0.0, C4, M4),
            2.0 * M4 ** 3, PEAK_FP32_VALU, "fp32_peak", graph=True)
        one("3xbf16_n3_256^3",
            lambda: mm.gemm_f32_3xbf16(M4, M4, M4, 1.0, A4, M4, B4, M4, 0.0, C4, M4, 3),
            2.0 * M4 ** 3, PEAK_BF16_MFMA, "bf16_peak", graph=True)
        del A4, B4, C4
        # one GPU's share of the 4096^3 product under eight-way row sharding
        M5 = 512
        _, (A5, B5, C5) = _dev_inputs(M5, N, K, 8, torch)
        one("3xbf16_n3_512x4096x4096_row_shard",
            lambda: mm.gemm_f32_3xbf16(M5, N, K, 1.5, A5, K, B5, N, 0.5, C5, N, 3),
            2.0 * M5 * N * K, PEAK_BF16_MFMA, "bf16_peak")
        nb5 = mm.gemm_splitk_workspace_bytes(M5, N, K, 0)
        ws5 = torch.empty(max(nb5, 256), dtype=torch.uint8, device="cuda")
        one("3xbf16_n3_512x4096x4096_row_shard_splitk%d" % mm.gemm_splitk_default_splits(M5, N, K),
            lambda: mm.gemm_f32_3xbf16_splitk(M5, N, K, 1.5, A5, K, B5, N, 0.5, C5, N, 3, 0, ws5, nb5),
            2.0 * M5 * N * K, PEAK_BF16_MFMA, "bf16_peak")
        del A5, B5, C5
        # a skinny product (64 rows): one pass on the small-product tiles, and split-K
        M6 = 64
        _, (A6, B6, C6) = _dev_inputs(M6, N, K, 9, torch)
        one("3xbf16_n3_64x4096x4096",
            lambda: mm.gemm_f32_3xbf16(M6, N, K, 1.5, A6, K, B6, N, 0.5, C6, N, 3),
            2.0 * M6 * N * K, PEAK_BF16_MFMA, "bf16_peak", graph=True)
        nb6 = mm.gemm_splitk_workspace_bytes(M6, N, K, 0)
        ws6 = torch.empty(max(nb6, 256), dtype=torch.uint8, device="cuda")
        one("3xbf16_n3_64x4096x4096_splitk%d" % mm.gemm_splitk_default_splits(M6, N, K),
            lambda: mm.gemm_f32_3xbf16_splitk(M6, N, K, 1.5, A6, K, B6, N, 0.5, C6, N, 3, 0, ws6, nb6),
            2.0 * M6 * N * K, PEAK_BF16_MFMA, "bf16_peak")
        del A6, B6, C6, ws5, ws6

    grouped = grouped_run = None
    if not args.no_grouped:
        _log("grouped: 512 problems, autotuned tiles, graph replay")
        *grouped_run, grouped = run_grouped(torch, mm, K_, W_)
    serving = serving_sample = None
    if not args.no_serving:
        _log("serving: Poisson 2000 req/s for %.0f s" % args.serve_seconds)
        serving_sample, serving = run_serving(torch, mm, args.serve_seconds)

    # ---------------- accuracy of every path and the CPU baseline -----------
    cpu = cpu_detail = accuracy = None
    if not args.no_cpu_baseline:
        cpu, cpu_detail, accuracy = run_accuracy(torch, mm, (hA, hB, hC0), grouped_run,
                                                 serving_sample)
    achieved = head_tflops
    line = {
        "metric": "FP32-accurate GEMM TFLOP/s & % peak: plain vs 3xBF16 MFMA; serve p50/p99 ms",
        "value": round(head_tflops, 2),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": K_,
        "warmup": W_,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "3xbf16 (bf16 split products, f32 accumulate)",
        "data": "synthetic",
        "config": {"workload": "gemm 4096x4096x4096 fp32 row-major, alpha=1.5 beta=0.5, "
                               "FP32-accurate via 3 bf16 split products on MFMA (fp32 accumulate)",
                   "M": M, "N": N, "K": K, "path": "3xbf16", "n_products": 3,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK_BF16_MFMA,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_BF16_MFMA, 4),
                     "traffic": _traffic("gemm_bx3_kernel_4096")},
        "cpu_baseline": cpu,
        "paths": paths,
        "grouped": grouped,
        "serving": serving,
        "accuracy": accuracy,
        "cpu_baseline_detail": cpu_detail,
        "wall_s_timed_region": round(wall, 3),
        "settle_s_before_warmup": args.settle_seconds,
        "sclk_dpm_mhz_after_timed": sclk,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
