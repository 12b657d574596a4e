"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/*.h, and rejects invalid arguments with the documented
BLAS-style codes before touching the device."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = []
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*"
                             r"([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M):
            names.append(m.group(1))
    return sorted(set(names))


def test_header_declares_functions():
    names = _declared_functions()
    assert "gemm_f32" in names and "err_norm_f64" in names and "gemm_last_error" in names


def test_library_exports_every_declared_symbol():
    import paper_1902_10345_amd as mm
    missing = [n for n in _declared_functions() if not hasattr(mm.lib, n)]
    assert not missing, missing


def test_binding_has_same_names():
    import paper_1902_10345_amd as mm
    missing = [n for n in _declared_functions() if not callable(getattr(mm, n, None))]
    assert not missing, missing


F = ctypes.c_void_p(16)  # a non-null dummy pointer; never dereferenced on rejection


@pytest.mark.parametrize("args,code", [
    ((-1, 4, 4, 1.0, F, 4, F, 4, 0.0, F, 4), -1),
    ((4, -1, 4, 1.0, F, 4, F, 4, 0.0, F, 4), -2),
    ((4, 4, -1, 1.0, F, 4, F, 4, 0.0, F, 4), -3),
    ((4, 4, 8, 1.0, F, 7, F, 4, 0.0, F, 4), -6),
    ((4, 4, 4, 1.0, F, 4, F, 3, 0.0, F, 4), -8),
    ((4, 4, 4, 1.0, F, 4, F, 4, 0.0, F, 3), -11),
    ((4, 4, 4, 1.0, None, 4, F, 4, 0.0, F, 4), -5),
    ((4, 4, 4, 1.0, F, 4, None, 4, 0.0, F, 4), -7),
    ((4, 4, 4, 1.0, F, 4, F, 4, 0.0, None, 4), -10),
    # quick return: M == 0 or N == 0 is a no-op even with NULL pointers
    ((0, 4, 4, 1.0, None, 4, None, 4, 0.0, None, 4), 0),
    ((4, 0, 4, 1.0, None, 4, None, 4, 0.0, None, 1), 0),
    # lda is checked before the quick return (BLAS order)
    ((0, 4, 4, 1.0, None, 1, None, 4, 0.0, None, 4), -6),
])
def test_gemm_f32_argument_codes(args, code):
    import paper_1902_10345_amd as mm
    st = mm.lib.gemm_f32(*args, None)
    assert st == code
    if code < 0:
        assert ("argument %d" % -code) in mm.last_error()


def test_gemm_run_config_argument_codes():
    import paper_1902_10345_amd as mm
    base = (4, 4, 4, 1.0, F, 4, F, 4, 0.0, F, 4, 3, None, 0, None)
    assert mm.lib.gemm_run_config(99, 0, *base) == -1
    assert mm.lib.gemm_run_config(0, 99, *base) == -2
    bad = (-1,) + base[1:]
    assert mm.lib.gemm_run_config(0, 0, *bad) == -3
    badlda = (4, 4, 8, 1.0, F, 7, F, 4, 0.0, F, 4, 3, None, 0, None)
    assert mm.lib.gemm_run_config(0, 0, *badlda) == -8


def test_err_norm_argument_codes():
    import paper_1902_10345_amd as mm
    ws = mm.err_norm_workspace_bytes()
    assert ws > 0
    assert mm.lib.err_norm_f64(-1, 4, F, 4, F, None, F, F, ws, None) == -1
    assert mm.lib.err_norm_f64(4, 4, F, 3, F, None, F, F, ws, None) == -4
    assert mm.lib.err_norm_f64(4, 4, F, 4, F, None, None, F, ws, None) == -7
    assert mm.lib.err_norm_f64(4, 4, F, 4, F, None, F, F, ws - 1, None) == -9


def test_configs_have_names():
    import paper_1902_10345_amd as mm
    for path in (mm.PATH_F32, mm.PATH_3XBF16, mm.PATH_FP8, mm.PATH_FP8_PREQUANTIZED):
        n = mm.gemm_num_configs(path)
        assert n >= 1
        names = [mm.gemm_config_name(path, i) for i in range(n)]
        assert all(names) and len(set(names)) == n
    # the two FP8 paths run the same kernels
    assert [mm.gemm_config_name(mm.PATH_FP8, i) for i in range(mm.gemm_num_configs(mm.PATH_FP8))] == \
        [mm.gemm_config_name(mm.PATH_FP8_PREQUANTIZED, i)
         for i in range(mm.gemm_num_configs(mm.PATH_FP8_PREQUANTIZED))]
    assert mm.gemm_num_configs(5) == 0 and mm.gemm_config_name(5, 0) == ""


def test_prequantized_run_config_argument_codes():
    """GEMM_PATH_FP8_PREQUANTIZED ignores A, B, lda and ldb."""
    import paper_1902_10345_amd as mm
    lib, P = mm.lib, mm.PATH_FP8_PREQUANTIZED
    nb = mm.gemm_fp8_workspace_bytes(4, 4, 4)
    assert lib.gemm_run_config(P, 0, 4, 4, 4, 1.0, None, 0, None, 0, 0.0, F, 4, 3, None, nb, None) == -15
    assert lib.gemm_run_config(P, 0, 4, 4, 4, 1.0, None, 0, None, 0, 0.0, F, 4, 3, 8, nb, None) == -15
    assert lib.gemm_run_config(P, 0, 4, 4, 4, 1.0, None, 0, None, 0, 0.0, F, 4, 3, 256, nb - 1, None) == -16
    assert lib.gemm_run_config(P, 0, 4, 4, 4, 1.0, None, 0, None, 0, 0.0, F, 3, 3, 256, nb, None) == -13
    assert lib.gemm_run_config(P, 0, 4, 4, 4, 1.0, None, 0, None, 0, 0.0, None, 4, 3, 256, nb, None) == -12
    assert lib.gemm_run_config(P, 0, -1, 4, 4, 1.0, None, 0, None, 0, 0.0, F, 4, 3, 256, nb, None) == -3
    n = mm.gemm_num_configs(P)
    assert lib.gemm_run_config(P, n, 4, 4, 4, 1.0, None, 0, None, 0, 0.0, F, 4, 3, 256, nb, None) == -2
    # M == 0: nothing to do, nothing touched
    assert lib.gemm_run_config(P, 0, 0, 4, 4, 1.0, None, 0, None, 0, 0.0, None, 4, 3, 256,
                               mm.gemm_fp8_workspace_bytes(0, 4, 4), None) == 0
