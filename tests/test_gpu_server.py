"""Serving loop: results alone vs in the mix (bitwise), against the oracle,
admission under a small HBM budget, FIFO without starvation, rejection of a
request larger than the budget, and latency accounting."""
import time

import numpy as np
import pytest

import oracle
import seeded_inputs as si
from gpu_util import check_split_result

pytestmark = pytest.mark.gpu

SOLO_CFG = {0: "bx3_128x128x32_4w64x64_p3", 1: "bx3_64x64x32_4w32x32_p3"}


def _cfg_index(mm, name):
    for c in range(mm.gemm_num_configs(mm.PATH_3XBF16)):
        if mm.gemm_config_name(mm.PATH_3XBF16, c) == name:
            return c
    raise KeyError(name)


def _pinned(x):
    import torch
    t = torch.empty(x.shape, dtype=torch.float32, pin_memory=True)
    t.copy_(torch.from_numpy(x))
    return t


def _server(mm, arena_bytes, slots=64, streams=4):
    import torch
    arena = torch.empty(arena_bytes, dtype=torch.uint8, device="cuda")
    return arena, mm.server_create(arena, arena_bytes, slots, mm.PATH_3XBF16, streams)


def _wait(mm, srv, tickets, timeout=60.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets) and time.time() - t0 < timeout:
        for t in tickets:
            if t not in out:
                r = mm.server_poll(srv, t)
                if r is not None:
                    out[t] = r
        time.sleep(0.001)
    assert len(out) == len(tickets), "requests did not complete"
    return out


def _requests(n, seed, lo=17, hi=700):
    sizes = si.log_uniform_sizes(n, lo, hi, seed, 1)
    reqs = []
    for t, (M, N, K) in enumerate(sizes):
        M, N, K = int(M), int(N), int(K)
        A = si.uniform((M, K), seed * 7919 + 3 * t)
        B = si.uniform((K, N), seed * 7919 + 3 * t + 1)
        C0 = si.uniform((M, N), seed * 7919 + 3 * t + 2)
        reqs.append((M, N, K, A, B, C0))
    return reqs


def test_alone_and_in_the_mix_are_bitwise_equal_and_correct():
    import torch
    import paper_1902_10345_amd as mm
    # a large request first (its step copies 48 MB of operands, milliseconds
    # of work), then 40 small ones submitted while that step is on the device:
    # they are admitted into further steps on the other streams
    n = 2048
    big = (n, n, n, si.uniform((n, n), 91), si.uniform((n, n), 92), si.uniform((n, n), 93))
    reqs = [big] + _requests(40, seed=9)
    arena, srv = _server(mm, 1 << 30)
    try:
        bufs = []
        for (M, N, K, A, B, C0) in reqs:
            hA, hB, hC0 = _pinned(A), _pinned(B), _pinned(C0)
            hC = torch.empty((M, N), dtype=torch.float32, pin_memory=True)
            bufs.append((hA, hB, hC0, hC))
        tickets = []
        for i, ((M, N, K, _, _, _), (hA, hB, hC0, hC)) in enumerate(zip(reqs, bufs)):
            tickets.append(mm.server_submit(srv, M, N, K, 1.5, hA, hB, 0.5, hC0, hC))
            if i == 0:
                time.sleep(0.001)  # the large request's step is launched first
        _wait(mm, srv, tickets)
        st = mm.server_stats(srv)
        assert st["completed"] == len(reqs)
        # the requests really were in a mix: several admitted at once, and
        # steps on different streams in flight together
        assert st["max_in_flight"] > 1, st
        assert st["max_concurrent_steps"] > 1, st
    finally:
        mm.server_destroy(srv)
    for (M, N, K, A, B, C0), (hA, hB, hC0, hC) in zip(reqs, bufs):
        C = hC.numpy()
        check_split_result(oracle, A, B, C0, C, 1.5, 0.5, 3)
        v = mm.grouped_default_variant(M, N, K)
        solo = torch.from_numpy(C0).cuda()
        dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
        mm.gemm_run_config(mm.PATH_3XBF16, _cfg_index(mm, SOLO_CFG[v]), M, N, K, 1.5, dA, K, dB,
                           N, 0.5, solo, N, n_products=3)
        torch.cuda.synchronize()
        assert np.array_equal(solo.cpu().numpy(), C), (M, N, K)


def test_pageable_host_buffers_work():
    import paper_1902_10345_amd as mm
    reqs = _requests(6, seed=10)
    arena, srv = _server(mm, 1 << 28)
    try:
        outs, tickets = [], []
        for (M, N, K, A, B, C0) in reqs:
            C = np.empty((M, N), dtype=np.float32)
            outs.append(C)
            tickets.append(mm.server_submit(srv, M, N, K, 1.0, A, B, 0.0, None, C))
        _wait(mm, srv, tickets)
    finally:
        mm.server_destroy(srv)
    for (M, N, K, A, B, C0), C in zip(reqs, outs):
        check_split_result(oracle, A, B, None, C, 1.0, 0.0, 3)


def test_small_budget_limits_admission_and_fifo_has_no_starvation():
    import torch
    import paper_1902_10345_amd as mm
    # operand footprint of a 500^3 request: 3 * 1 MB; a 1000^3 one: 12 MB
    big = (1000, 1000, 1000)
    small = (500, 500, 500)
    budget = 16 << 20   # 16 MB arena (minus the per-stream workspaces)
    arena, srv = _server(mm, budget, slots=64, streams=2)
    try:
        g = np.random.default_rng(1)
        keep, tickets = [], []
        order = [small, big] + [small] * 12
        for (M, N, K) in order:
            hA = torch.from_numpy(g.uniform(-1, 1, (M, K)).astype(np.float32)).pin_memory()
            hB = torch.from_numpy(g.uniform(-1, 1, (K, N)).astype(np.float32)).pin_memory()
            hC = torch.empty((M, N), dtype=torch.float32, pin_memory=True)
            keep.append((hA, hB, hC))
            tickets.append(mm.server_submit(srv, M, N, K, 1.0, hA, hB, 0.0, None, hC))
        res = _wait(mm, srv, tickets)
        st = mm.server_stats(srv)
        assert st["completed"] == len(order)
        # never more resident than the budget allows
        assert st["arena_high_water_bytes"] <= budget
        assert st["max_in_flight"] <= 5
        # the big request is served (FIFO: later small ones cannot overtake it)
        assert tickets[1] in res
        # a request larger than the whole arena is rejected
        with pytest.raises(mm.GemmError) as e:
            mm.server_submit(srv, 4000, 4000, 4000, 1.0, 16, 16, 0.0, None, 16)
        assert e.value.status == mm.STATUS_REJECTED
        assert mm.server_stats(srv)["rejected"] == 1
    finally:
        mm.server_destroy(srv)


def test_latency_is_measured_from_the_arrival_stamp():
    import torch
    import paper_1902_10345_amd as mm
    arena, srv = _server(mm, 1 << 26)
    try:
        A = torch.ones((64, 64), pin_memory=True)
        hC = torch.empty((64, 64), pin_memory=True)
        time.sleep(0.1)                         # the server clock starts at 0
        arrival = mm.server_now(srv) - 0.050   # arrived 50 ms ago
        t = mm.server_submit(srv, 64, 64, 64, 1.0, A, A, 0.0, None, hC, arrival)
        lat, res_lat = _wait(mm, srv, [t])[t]
        assert lat >= 50.0 and res_lat >= lat
        assert np.all(hC.numpy() == 64.0)
    finally:
        mm.server_destroy(srv)


def test_drain_and_stats():
    import torch
    import paper_1902_10345_amd as mm
    arena, srv = _server(mm, 1 << 28)
    try:
        A = torch.ones((128, 128), pin_memory=True)
        outs = [torch.empty((128, 128), pin_memory=True) for _ in range(20)]
        for o in outs:
            mm.server_submit(srv, 128, 128, 128, 2.0, A, A, 0.0, None, o)
        mm.server_drain(srv, 30.0)
        st = mm.server_stats(srv)
        assert st["completed"] == 20 and st["p99_ms"] >= st["p50_ms"] > 0
        assert all(np.all(o.numpy() == 256.0) for o in outs)
    finally:
        mm.server_destroy(srv)


def test_injected_step_failure_is_reported_per_request():
    """A step that cannot be enqueued (forced from the host) ends its requests
    with GEMM_STATUS_HIP_ERROR -- never with OK and an unwritten result --
    gives their slots and arena ranges back, and later requests run."""
    import os
    import torch
    import paper_1902_10345_amd as mm
    os.environ["GEMM_SERVER_INJECT_STEP_FAILURES"] = "1"
    try:
        arena, srv = _server(mm, 1 << 26, slots=8, streams=2)
    finally:
        del os.environ["GEMM_SERVER_INJECT_STEP_FAILURES"]
    try:
        A = torch.ones((64, 64), pin_memory=True)
        hC = torch.full((64, 64), -1.0, pin_memory=True)
        t = mm.server_submit(srv, 64, 64, 64, 1.0, A, A, 0.0, None, hC)
        t0 = time.time()
        status = None
        while time.time() - t0 < 30:
            try:
                if mm.server_poll(srv, t) is not None:
                    status = mm.STATUS_OK
                    break
            except mm.GemmError as e:
                status = e.status
                break
            time.sleep(0.001)
        assert status == mm.STATUS_HIP_ERROR
        assert np.all(hC.numpy() == -1.0)           # nothing was written
        st = mm.server_stats(srv)
        assert st["failed"] == 1 and st["completed"] == 0
        # the ticket is forgotten after it was reported
        with pytest.raises(mm.GemmError) as e:
            mm.server_poll(srv, t)
        assert e.value.status == mm.STATUS_UNKNOWN
        # the server keeps serving
        hC2 = torch.empty((64, 64), pin_memory=True)
        t2 = mm.server_submit(srv, 64, 64, 64, 1.0, A, A, 0.0, None, hC2)
        _wait(mm, srv, [t2])
        assert np.all(hC2.numpy() == 64.0)
        mm.server_drain(srv, 30.0)
    finally:
        mm.server_destroy(srv)


def _poll_status(mm, srv, t, timeout=30.0):
    t0 = time.time()
    while time.time() - t0 < timeout:
        try:
            if mm.server_poll(srv, t) is not None:
                return mm.STATUS_OK
        except mm.GemmError as e:
            return e.status
        time.sleep(0.001)
    raise AssertionError("request did not end")


def test_queue_timeout_drops_stale_requests():
    """A request whose arrival stamp is older than the queue timeout is
    dropped before admission (the timeout check precedes admission in every
    scheduler pass) and reported as GEMM_STATUS_TIMED_OUT; fresh requests
    are served."""
    import torch
    import paper_1902_10345_amd as mm
    arena, srv = _server(mm, 1 << 26, slots=4, streams=2)
    try:
        mm.server_set_queue_timeout(srv, 0.2)
        A = torch.ones((32, 32), pin_memory=True)
        hC = torch.full((32, 32), -1.0, pin_memory=True)
        hC2 = torch.empty((32, 32), pin_memory=True)
        # the server clock starts at 0 when the server is created and a
        # negative stamp means "now": wait until a stamp 0.5 s in the past is
        # a valid (non-negative) one
        time.sleep(0.6)
        stamp = mm.server_now(srv) - 0.5
        assert stamp >= 0
        stale = mm.server_submit(srv, 32, 32, 32, 1.0, A, A, 0.0, None, hC, stamp)
        fresh = mm.server_submit(srv, 32, 32, 32, 1.0, A, A, 0.0, None, hC2)
        assert _poll_status(mm, srv, stale) == mm.STATUS_TIMED_OUT
        assert _poll_status(mm, srv, fresh) == mm.STATUS_OK
        assert np.all(hC.numpy() == -1.0) and np.all(hC2.numpy() == 32.0)
        with pytest.raises(mm.GemmError):
            mm.server_set_queue_timeout(srv, -1.0)
    finally:
        mm.server_destroy(srv)


def test_cancel_a_queued_request():
    """With one slot, a request submitted right behind a large one waits in
    the queue; cancelling it reports GEMM_STATUS_CANCELLED and its result
    buffer is never written.  (Should the large request finish before the
    cancel lands, the second one is admitted and the cancel is refused with
    NOT_READY; the pair is then tried again.)"""
    import torch
    import paper_1902_10345_amd as mm
    arena, srv = _server(mm, 1 << 28, slots=1, streams=2)
    try:
        n = 1536
        big = torch.rand((n, n), pin_memory=True)
        hbig = torch.empty((n, n), pin_memory=True)
        A = torch.ones((16, 16), pin_memory=True)
        cancelled = False
        for _ in range(3):
            hC = torch.full((16, 16), -1.0, pin_memory=True)
            t1 = mm.server_submit(srv, n, n, n, 1.0, big, big, 0.0, None, hbig)
            t2 = mm.server_submit(srv, 16, 16, 16, 1.0, A, A, 0.0, None, hC)
            try:
                mm.server_cancel(srv, t2)
                cancelled = True
            except mm.GemmError as err:
                assert err.status == mm.STATUS_NOT_READY
            _wait(mm, srv, [t1])
            if cancelled:
                assert _poll_status(mm, srv, t2) == mm.STATUS_CANCELLED
                assert np.all(hC.numpy() == -1.0)
                break
            assert _poll_status(mm, srv, t2) == mm.STATUS_OK
        assert cancelled
        with pytest.raises(mm.GemmError) as e:
            mm.server_cancel(srv, 123456789)
        assert e.value.status == mm.STATUS_UNKNOWN
        mm.server_drain(srv, 30.0)
    finally:
        mm.server_destroy(srv)


def test_offsets_beyond_32_bits_are_refused_at_submit():
    """K (or N) so large that the grouped tile body's 32-bit offsets would
    wrap is refused with GEMM_STATUS_UNSUPPORTED before anything is copied,
    even when the operands would fit the arena, and counts as rejected."""
    import paper_1902_10345_amd as mm
    arena, srv = _server(mm, 1 << 26, slots=4, streams=1)
    try:
        for (M, N, K) in [(1, 1, 5_000_000), (1, 20_000_000, 1)]:
            with pytest.raises(mm.GemmError) as e:
                mm.server_submit(srv, M, N, K, 1.0, 16, 16, 0.0, None, 16)
            assert e.value.status == mm.STATUS_UNSUPPORTED
        assert mm.server_stats(srv)["rejected"] == 2
    finally:
        mm.server_destroy(srv)
