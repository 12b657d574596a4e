"""Host-side logic that needs no GPU: the autotuner's JSON cache, workspace
layouts, tile-shape heuristics, argument checks of the grouped / FP8 /
serving entry points, and the seeded workload generators."""
import json
import math
import os

import numpy as np
import pytest

import seeded_inputs as si

F = 16  # non-null dummy device address; never dereferenced on rejection


def test_tuner_json_round_trip(tmp_path):
    import paper_1902_10345_amd as mm
    src = tmp_path / "in.json"
    name = mm.gemm_config_name(mm.PATH_3XBF16, 1)
    src.write_text(
        '{"arch": "gfx950", "grouped_small_cost": 2.5, "entries": [\n'
        '{"path": 1, "n_products": 3, "log2_m": 12, "log2_n": 12, "log2_k": 12, "config": "%s"},\n'
        '{"path": 1, "n_products": 3, "log2_m": 5, "log2_n": 5, "log2_k": 5, "config": "no_such_config"}\n'
        ']}\n' % name)
    mm.gemm_tuner_load(str(src))
    try:
        # the tuned choice replaces the heuristic for every shape in the bucket
        assert mm.gemm_default_config(mm.PATH_3XBF16, 4096, 4000, 3000) == 1
        out = tmp_path / "out.json"
        mm.gemm_tuner_save(str(out))
        doc = json.loads(out.read_text())
        assert doc["grouped_small_cost"] == 2.5
        assert doc["entries"] == [{"path": 1, "n_products": 3, "log2_m": 12, "log2_n": 12,
                                   "log2_k": 12, "config": name}]
    finally:
        mm.gemm_tuner_clear()
    assert mm.gemm_default_config(mm.PATH_3XBF16, 4096, 4096, 4096) != -1


def test_tuner_load_missing_file_is_an_error():
    import paper_1902_10345_amd as mm
    with pytest.raises(mm.GemmError):
        mm.gemm_tuner_load("/nonexistent/dir/tuner.json")


def test_fp8_workspace_layout_matches_library():
    import paper_1902_10345_amd as mm
    for (M, N, K) in [(1, 1, 1), (4096, 4096, 4096), (300, 77, 129), (8, 3000, 1000)]:
        L = mm.fp8_workspace_layout(M, N, K)
        total = mm.gemm_fp8_workspace_bytes(M, N, K)
        assert L["Kp"] % 128 == 0 and L["Kp"] >= K and L["Kp"] - K < 128
        assert L["qb"] >= M * L["Kp"] and L["sa"] >= L["qb"] + N * L["Kp"]
        assert all(L[k] % 256 == 0 for k in ("qa", "qb", "sa", "sb"))
        assert total >= L["sb"] + 4 * N


def test_grouped_workspace_and_variant_heuristic():
    import paper_1902_10345_amd as mm
    assert mm.grouped_gemm_workspace_bytes(0) >= 256
    assert mm.grouped_gemm_workspace_bytes(512) >= 512 * 80 + 513 * 4
    # small problems take the 64 x 64 tile, large ones the 128 x 128 tile
    assert mm.grouped_default_variant(32, 32, 100) == 1
    assert mm.grouped_default_variant(1024, 1024, 100) == 0
    assert mm.grouped_default_variant(48, 1024, 100) == 1   # half the 128-row tile wasted


def test_default_configs_are_valid_indices():
    import paper_1902_10345_amd as mm
    for path in (mm.PATH_F32, mm.PATH_3XBF16):
        n = mm.gemm_num_configs(path)
        for shape in [(256, 256, 256), (4096, 4096, 4096), (8192, 2048, 4096), (17, 5000, 3)]:
            c = mm.gemm_default_config(path, *shape)
            assert 0 <= c < n, (path, shape, c)


def test_grouped_argument_codes():
    import paper_1902_10345_amd as mm
    ws_bytes = mm.grouped_gemm_workspace_bytes(2)
    good = (64, 64, 64, F, 64, F, 64, F, 64, 1.0, 0.0)
    arr = mm.problem_array([good, good])
    lib = mm.lib
    assert lib.grouped_gemm(arr, -1, mm.PATH_3XBF16, None, F, ws_bytes, None) == -2
    assert lib.grouped_gemm(None, 2, mm.PATH_3XBF16, None, F, ws_bytes, None) == -1
    assert lib.grouped_gemm(arr, 2, mm.PATH_F32, None, F, ws_bytes, None) == -3
    assert lib.grouped_gemm(arr, 2, mm.PATH_3XBF16, None, None, ws_bytes, None) == -5
    assert lib.grouped_gemm(arr, 2, mm.PATH_3XBF16, None, 256, ws_bytes - 1, None) == -6
    assert lib.grouped_gemm(arr, 2, mm.PATH_3XBF16, None, 8, ws_bytes, None) == -5  # unaligned
    bad = mm.problem_array([good, (64, 64, 64, F, 63, F, 64, F, 64, 1.0, 0.0)])
    assert lib.grouped_gemm(bad, 2, mm.PATH_3XBF16, None, 256, ws_bytes, None) == -1
    assert "problems[1]" in mm.last_error()
    import ctypes
    v = (ctypes.c_int * 2)(0, 7)
    assert lib.grouped_gemm(arr, 2, mm.PATH_3XBF16, v, 256, ws_bytes, None) == -4


def test_fp8_argument_codes():
    import paper_1902_10345_amd as mm
    lib = mm.lib
    nb = mm.gemm_fp8_workspace_bytes(64, 64, 64)
    args = (64, 64, 64, 1.0, F, 64, F, 64, 0.0, F, 64)
    assert lib.gemm_fp8_scaled(*args, None, nb, None) == -12
    assert lib.gemm_fp8_scaled(*args, 256, nb - 1, None) == -13
    assert lib.gemm_fp8_scaled(*args, 8, nb, None) == -12
    assert lib.fp8_quantize(64, 64, 64, F, 63, F, 64, 256, nb, None) == -5
    assert lib.gemm_fp8_prequantized(64, 64, 64, 1.0, 256, nb, 0.0, F, 63, None) == -9
    assert lib.fp8_e4m3_encode(-1, F, F, None) == -1
    assert lib.split_bf16x3(-1, F, F, F, None, None) == -1
    # the split and encoder accept n == 0 without touching the device
    assert lib.split_bf16x3(0, None, None, None, None, None) == 0


def test_3xbf16_argument_codes():
    import paper_1902_10345_amd as mm
    lib = mm.lib
    assert lib.gemm_f32_3xbf16(4, 4, 4, 1.0, F, 4, F, 4, 0.0, F, 4, 5, None) == -12
    assert lib.gemm_f32_3xbf16(4, 4, 4, 1.0, F, 3, F, 4, 0.0, F, 4, 3, None) == -6
    assert lib.gemm_f32_3xbf16(0, 4, 4, 1.0, None, 4, None, 4, 0.0, None, 4, 3, None) == 0


def test_server_argument_codes():
    import ctypes
    import paper_1902_10345_amd as mm
    lib = mm.lib
    out = ctypes.c_void_p()
    assert lib.server_create(None, 1 << 20, 8, mm.PATH_3XBF16, 2, ctypes.byref(out)) == -1
    assert lib.server_create(8, 1 << 20, 8, mm.PATH_3XBF16, 2, ctypes.byref(out)) == -1
    assert lib.server_create(256, 1 << 20, 0, mm.PATH_3XBF16, 2, ctypes.byref(out)) == -3
    assert lib.server_create(256, 1 << 20, 8, mm.PATH_F32, 2, ctypes.byref(out)) == -4
    assert lib.server_create(256, 1 << 20, 8, mm.PATH_3XBF16, 0, ctypes.byref(out)) == -5
    assert lib.server_create(256, 1024, 8, mm.PATH_3XBF16, 2, ctypes.byref(out)) == -2
    t = ctypes.c_uint64()
    assert lib.server_submit(None, 1, 1, 1, 1.0, F, F, 0.0, None, F, -1.0, ctypes.byref(t)) == -1


# ------------------------------------------------------------- generators ---

def test_log_uniform_sizes_are_in_range_and_rounded():
    s = si.log_uniform_sizes(5000, 32, 1024, seed=5, multiple=16)
    assert s.min() >= 32 and s.max() <= 1024 and np.all(s % 16 == 0)
    # log-uniform: the median of exp(U[ln 32, ln 1024]) is sqrt(32*1024) = 181
    assert abs(np.median(s) - math.sqrt(32 * 1024)) < 20
    r = si.log_uniform_sizes(5000, 64, 2048, seed=6, multiple=1)
    assert r.min() >= 64 and r.max() <= 2048 and np.any(r % 16 != 0)


def test_poisson_arrivals_rate():
    t = si.poisson_arrivals(2000.0, 10.0, seed=6)
    assert np.all(np.diff(t) >= 0) and t[-1] < 10.0
    assert abs(len(t) - 20000) < 5 * math.sqrt(20000)
    gaps = np.diff(t)
    assert abs(gaps.mean() - 1 / 2000.0) < 0.05 / 2000.0


def test_fp8_workload_outliers():
    A, B, C0 = si.fp8_workload(64, 200, 300, seed=4, outliers="A")
    big = np.abs(A).max(axis=0) > 100
    assert big.sum() == math.ceil(0.01 * 300)
    A2, B2, _ = si.fp8_workload(64, 200, 300, seed=4, outliers="B")
    assert (np.abs(B2).max(axis=0) > 100).sum() == math.ceil(0.01 * 200)


def test_uniform_is_seeded_and_in_range():
    a = si.uniform((100, 100), 3)
    b = si.uniform((100, 100), 3)
    assert np.array_equal(a, b) and a.dtype == np.float32
    assert a.min() >= -1.0 and a.max() < 1.0
    p = si.uniform((10, 7), 3, ld=9, pad_value=np.nan)
    assert p.shape == (10, 7) and p.strides[0] == 9 * 4


def test_splitk_argument_codes_and_sizes():
    import paper_1902_10345_amd as mm
    lib = mm.lib
    args = (512, 512, 4096, 1.0, F, 4096, F, 512, 0.0, F, 512)
    nb = mm.gemm_splitk_workspace_bytes(512, 512, 4096, 4)
    assert nb == 4 * 512 * 512 * 4
    assert lib.gemm_f32_3xbf16_splitk(*args, 5, 4, 256, nb, None) == -12
    assert lib.gemm_f32_3xbf16_splitk(*args, 3, 65, 256, nb, None) == -13
    assert lib.gemm_f32_3xbf16_splitk(*args, 3, -1, 256, nb, None) == -13
    assert lib.gemm_f32_3xbf16_splitk(*args, 3, 4, None, nb, None) == -14
    assert lib.gemm_f32_3xbf16_splitk(*args, 3, 4, 8, nb, None) == -14
    assert lib.gemm_f32_3xbf16_splitk(*args, 3, 4, 256, nb - 1, None) == -15
    assert lib.gemm_f32_3xbf16_splitk(0, 4, 4, 1.0, None, 4, None, 4, 0.0, None, 4, 3, 4, None, 0,
                                      None) == 0
    # one chunk needs no workspace
    assert mm.gemm_splitk_workspace_bytes(512, 512, 4096, 1) == 0
    # the default fills the machine with 128 x 128 tiles, chunks >= 256 deep, at most 64
    for (M, N, K) in [(512, 4096, 4096), (64, 4096, 4096), (4096, 4096, 4096), (256, 256, 256),
                      (128, 128, 100000)]:
        s = mm.gemm_splitk_default_splits(M, N, K)
        assert 1 <= s <= 64 and (s == 1 or K // s >= 256)
        assert mm.gemm_splitk_workspace_bytes(M, N, K, 0) == mm.gemm_splitk_workspace_bytes(M, N, K, s)
    assert mm.gemm_splitk_default_splits(4096, 4096, 4096) == 1
    assert mm.gemm_splitk_default_splits(64, 4096, 4096) == 16


def test_gemm_ex_argument_codes():
    """Storage order, transpose flags and leading dimensions are checked
    before anything is enqueued (these calls never reach the device)."""
    import paper_1902_10345_amd as mm
    lib = mm.lib
    R, Cm, Nt, T = mm.ROW_MAJOR, mm.COL_MAJOR, mm.NO_TRANS, mm.TRANS
    M, N, K = 4, 8, 16

    def call(order=R, ta=Nt, tb=Nt, M=M, N=N, K=K, A=F, lda=None, B=F, ldb=None, C=F, ldc=None,
             path=mm.PATH_3XBF16, n=3, ws=None, nb=0, alpha=1.0):
        row = order == R
        lda = lda if lda is not None else ((M if ta == T else K) if row else (K if ta == T else M))
        ldb = ldb if ldb is not None else ((K if tb == T else N) if row else (N if tb == T else K))
        ldc = ldc if ldc is not None else (N if row else M)
        return lib.gemm_ex(order, ta, tb, M, N, K, alpha, A, lda, B, ldb, 0.0, C, ldc, path, n, ws,
                           nb, None)

    assert call(order=100) == -1
    assert call(ta=110) == -2
    assert call(tb=114) == -3
    assert call(M=-1) == -4 and call(N=-1) == -5 and call(K=-1) == -6
    # row-major: lda >= K (no trans) or M (trans); ldb >= N or K; ldc >= N
    assert call(lda=K - 1) == -9 and call(ta=T, lda=M - 1) == -9
    assert call(ldb=N - 1) == -11 and call(tb=T, ldb=K - 1) == -11
    assert call(ldc=N - 1) == -14
    # column-major: lda >= M or K; ldb >= K or N; ldc >= M
    assert call(order=Cm, lda=M - 1) == -9 and call(order=Cm, ta=T, lda=K - 1) == -9
    assert call(order=Cm, ldb=K - 1) == -11 and call(order=Cm, tb=T, ldb=N - 1) == -11
    assert call(order=Cm, ldc=M - 1) == -14
    # strides that are only valid for the other order or flag are accepted where they fit
    assert call(order=Cm, lda=M, ldb=K, ldc=M, A=None) == -8
    assert call(path=mm.PATH_FP8_PREQUANTIZED) == -15 and call(path=9) == -15
    assert call(n=5) == -16
    assert call(C=None) == -13
    assert call(A=None) == -8 and call(B=None) == -10
    nb = mm.gemm_fp8_workspace_bytes(M, N, K)
    assert call(path=mm.PATH_FP8) == -17
    assert call(path=mm.PATH_FP8, ws=8, nb=nb) == -17          # unaligned
    assert call(path=mm.PATH_FP8, ws=256, nb=nb - 1) == -18
    # empty output: nothing to do, pointers may be NULL
    assert call(M=0, A=None, B=None, C=None) == 0
    assert call(order=Cm, N=0, A=None, B=None, C=None) == 0
    assert mm.gemm_last_error() == ""


def test_fp8_workspace_is_symmetric_in_m_and_n():
    """A column-major FP8 call runs the row-major product with M and N
    exchanged; the workspace size must not depend on which is which."""
    import paper_1902_10345_amd as mm
    for (M, N, K) in [(1, 3000, 7), (4096, 64, 4096), (300, 77, 129)]:
        assert mm.gemm_fp8_workspace_bytes(M, N, K) == mm.gemm_fp8_workspace_bytes(N, M, K)


def test_f64_argument_codes_and_configs():
    import paper_1902_10345_amd as mm
    lib = mm.lib
    assert mm.gemm_num_configs(mm.PATH_F64) >= 2
    names = [mm.gemm_config_name(mm.PATH_F64, c) for c in range(mm.gemm_num_configs(mm.PATH_F64))]
    assert all(n.startswith("f64_") for n in names) and len(set(names)) == len(names)
    assert 0 <= mm.gemm_default_config(mm.PATH_F64, 4096, 4096, 4096) < len(names)
    assert lib.gemm_f64(-1, 4, 4, 1.0, F, 4, F, 4, 0.0, F, 4, None) == -1
    assert lib.gemm_f64(4, 4, 4, 1.0, F, 3, F, 4, 0.0, F, 4, None) == -6
    assert lib.gemm_f64(4, 4, 4, 1.0, F, 4, F, 3, 0.0, F, 4, None) == -8
    assert lib.gemm_f64(4, 4, 4, 1.0, F, 4, F, 4, 0.0, F, 3, None) == -11
    assert lib.gemm_f64(4, 4, 4, 1.0, None, 4, F, 4, 0.0, F, 4, None) == -5
    assert lib.gemm_f64(4, 4, 4, 1.0, F, 4, None, 4, 0.0, F, 4, None) == -7
    assert lib.gemm_f64(4, 4, 4, 1.0, F, 4, F, 4, 0.0, None, 4, None) == -10
    assert lib.gemm_f64(0, 4, 4, 1.0, None, 4, None, 4, 0.0, None, 4, None) == 0
    assert lib.gemm_f64_run_config(99, 4, 4, 4, 1.0, F, 4, F, 4, 0.0, F, 4, None) == -1
    assert lib.gemm_f64_run_config(0, 4, 4, 4, 1.0, F, 3, F, 4, 0.0, F, 4, None) == -7
    # the binary32 per-configuration entry point refuses binary64 operands
    assert lib.gemm_run_config(mm.PATH_F64, 0, 4, 4, 4, 1.0, F, 4, F, 4, 0.0, F, 4, 3, None, 0,
                               None) == -1
    sb = lib.gemm_f64_strided_batched
    args = lambda **kw: [kw.get(k, v) for k, v in (  # noqa: E731
        ("M", 4), ("N", 4), ("K", 4), ("alpha", 1.0), ("A", F), ("lda", 4), ("sa", 16), ("B", F),
        ("ldb", 4), ("sb", 16), ("beta", 0.0), ("C", F), ("ldc", 4), ("sc", 16), ("batch", 3))] + [None]
    assert sb(*args(M=-1)) == -1
    assert sb(*args(lda=3)) == -6
    assert sb(*args(sa=-1)) == -7
    assert sb(*args(ldb=3)) == -9
    assert sb(*args(sb=-4)) == -10
    assert sb(*args(ldc=3)) == -13
    assert sb(*args(sc=15)) == -14          # outputs would overlap
    assert sb(*args(batch=-1)) == -15
    assert sb(*args(C=None)) == -12
    assert sb(*args(A=None)) == -5 and sb(*args(B=None)) == -8
    assert sb(*args(batch=0, A=None, B=None, C=None)) == 0
    assert sb(*args(sc=0, batch=1, A=None)) == -5   # one problem: any output stride


def test_strided_batched_argument_codes():
    import paper_1902_10345_amd as mm
    sb = mm.lib.gemm_strided_batched
    base = dict(path=mm.PATH_3XBF16, M=4, N=4, K=4, alpha=1.0, A=F, lda=4, sa=16, B=F, ldb=4,
                sb=16, beta=0.0, C=F, ldc=4, sc=16, batch=3, n=3)

    def call(**kw):
        a = dict(base, **kw)
        return sb(a["path"], a["M"], a["N"], a["K"], a["alpha"], a["A"], a["lda"], a["sa"], a["B"],
                  a["ldb"], a["sb"], a["beta"], a["C"], a["ldc"], a["sc"], a["batch"], a["n"], None)

    assert call(path=mm.PATH_FP8) == -1 and call(path=mm.PATH_F64) == -1
    assert call(M=-1) == -2 and call(N=-1) == -3 and call(K=-1) == -4
    assert call(lda=3) == -7 and call(sa=-1) == -8
    assert call(ldb=3) == -10 and call(sb=-1) == -11
    assert call(ldc=3) == -14 and call(sc=15) == -15 and call(batch=-1) == -16
    assert call(n=5) == -17
    assert call(path=mm.PATH_F32, n=5, C=None) == -13   # n_products ignored on the FP32 path
    assert call(A=None) == -6 and call(B=None) == -9
    assert call(batch=0, A=None, B=None, C=None) == 0


def test_strides_beyond_32_bit_tile_offsets_are_refused_before_launch():
    """Leading dimensions whose tile panels exceed 2^31 bytes cannot be
    addressed with the kernels' 32-bit buffer offsets: the launchers refuse
    them (GEMM_STATUS_UNSUPPORTED) before anything is enqueued -- these calls
    never touch the (dummy) pointers."""
    import paper_1902_10345_amd as mm
    lib = mm.lib
    big = 1 << 24   # 64-row tiles: 64 x 2^24 floats x 4 B = 2^32 bytes
    assert lib.gemm_f32_3xbf16(300, 300, 300, 1.0, F, big, F, 300, 0.0, F, 300, 3, None) == \
        mm.STATUS_UNSUPPORTED
    assert "32-bit" in mm.gemm_last_error()
    assert lib.gemm_f32_3xbf16(300, 300, 300, 1.0, F, 300, F, big * 8, 0.0, F, 300, 3, None) == \
        mm.STATUS_UNSUPPORTED
    assert lib.gemm_f64(300, 300, 300, 1.0, F, big, F, 300, 0.0, F, 300, None) == mm.STATUS_UNSUPPORTED
    assert lib.gemm_ex(mm.ROW_MAJOR, mm.TRANS, mm.NO_TRANS, 300, 300, 300, 1.0, F, big * 8, F, 300,
                       0.0, F, 300, mm.PATH_3XBF16, 3, None, 0, None) == mm.STATUS_UNSUPPORTED
    assert lib.gemm_strided_batched(mm.PATH_3XBF16, 300, 300, 300, 1.0, F, big, 0, F, 300, 0, 0.0,
                                    F, 300, 90000, 2, 3, None) == mm.STATUS_UNSUPPORTED
    # small problems (one wave per problem) refuse the same way on every path
    # when neither their kernel nor the tile they fall back to can address the
    # operands (ldb 2^25: a 16-deep slab of B spans 2^31 bytes)
    for path, n in ((mm.PATH_3XBF16, 3), (mm.PATH_3XBF16, 6), (mm.PATH_F32, 3)):
        assert lib.gemm_strided_batched(path, 32, 32, 32, 1.0, F, big, 0, F, 32, 0, 0.0, F, 32,
                                        1024, 2, n, None) == mm.STATUS_UNSUPPORTED, (path, n)
        assert lib.gemm_strided_batched(path, 32, 32, 32, 1.0, F, 32, 0, F, 2 * big, 0, 0.0, F,
                                        32, 1024, 2, n, None) == mm.STATUS_UNSUPPORTED, (path, n)


def test_default_config_of_empty_shapes():
    import paper_1902_10345_amd as mm
    for path in (mm.PATH_F32, mm.PATH_3XBF16, mm.PATH_FP8, mm.PATH_F64):
        for shape in [(0, 5, 5), (5, 0, 5), (5, 5, 0), (0, 0, 0)]:
            c = mm.gemm_default_config(path, *shape)
            assert 0 <= c < mm.gemm_num_configs(path), (path, shape, c)


def test_default_tile_rules_for_underfilled_shapes():
    """Shapes whose 128 x 128 tiles leave compute units idle take the small-
    product tiles (k range split over a workgroup's waves); machine-filling
    shapes keep the LDS-staged matrix-core tiles (256 compute units)."""
    import paper_1902_10345_amd as mm

    def name(path, M, N, K):
        return mm.gemm_config_name(path, mm.gemm_default_config(path, M, N, K))
    assert name(mm.PATH_F32, 256, 256, 256) == "f32_small_32x32_8wk"
    assert name(mm.PATH_3XBF16, 256, 256, 256) == "bx3_small_32x32_8wk_p3"
    assert name(mm.PATH_F32, 1024, 1024, 1024) == "f32_small_64x64_8wk"
    assert name(mm.PATH_3XBF16, 1024, 1024, 1024) == "bx3_small_64x64_8wk_p3"
    assert name(mm.PATH_3XBF16, 64, 4096, 4096) == "bx3_small_32x32_8wk_p3"
    assert name(mm.PATH_3XBF16, 1536, 1536, 512) == "bx3_128x128x16_2x4w64x64_p3_kg2"
    assert name(mm.PATH_3XBF16, 2048, 2048, 2048) == "bx3_128x128x16_2x4w64x64_p3_kg2"
    assert name(mm.PATH_3XBF16, 2048, 2048, 2047) == "bx3_128x128x16_4w64x64_p3"  # odd K
    assert name(mm.PATH_3XBF16, 2048, 1024, 4096) == "bx3_64x64x32_4w32x32_p3"
    assert name(mm.PATH_F32, 2048, 2048, 2048) == "f32mfma_128x128x16_2x4w64x64_kg2"
    assert name(mm.PATH_F32, 2048, 1536, 2048) == "f32_small_64x64_8wk"
    assert name(mm.PATH_F32, 2560, 2048, 2048) == "f32mfma_128x128x16_4w64x64"
    assert name(mm.PATH_F32, 4096, 4096, 4096) == "f32mfma_256x256x16_8w128x64"
    assert name(mm.PATH_3XBF16, 4096, 4096, 4096) == "bx3_256x256x16_8w128x64_p3"
