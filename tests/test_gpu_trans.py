"""Storage order and transposed operands (gemm_ex): C <- alpha*op(A)op(B) +
beta*C with each operand in row- or column-major storage, op(X) = X or X^T,
as the BLAS-style external-code call of the paper passes them (Sec. 2.1).

Operands are placed in memory by numpy (C or Fortran order, padded leading
dimensions, NaN padding that must never be read); results are checked against
the FP64 oracle with the bounds of each path, and -- since a transposed
operand changes only how a tile is staged into LDS -- bit for bit against the
untransposed call wherever both run the same tile configuration."""
import itertools

import numpy as np
import pytest

import oracle
import seeded_inputs as si
from gpu_util import check_split_result, gamma, sample_rows

pytestmark = pytest.mark.gpu

FLAGS = list(itertools.product((False, True), (False, True)))
ORDERS = ("C", "F")


def _flags(mm, ta, tb):
    return mm.TRANS if ta else mm.NO_TRANS, mm.TRANS if tb else mm.NO_TRANS


def _order(mm, o):
    return mm.ROW_MAJOR if o == "C" else mm.COL_MAJOR


def _ld(x, o, pad):
    return (x.shape[1] if o == "C" else x.shape[0]) + pad


class Problem:
    """Logical op(A) (M x K), op(B) (K x N), C0 (M x N), and their storage
    buffers on the device for one (order, ta, tb)."""

    def __init__(self, opA, opB, C0, o, ta, tb, pad=3):
        import torch
        self.opA, self.opB, self.C0, self.o, self.ta, self.tb = opA, opB, C0, o, ta, tb
        self.M, self.K = opA.shape
        self.N = opB.shape[1]
        a_st = np.ascontiguousarray(opA.T) if ta else opA
        b_st = np.ascontiguousarray(opB.T) if tb else opB
        self.lda, self.ldb, self.ldc = _ld(a_st, o, pad), _ld(b_st, o, pad + 1), _ld(C0, o, pad + 2)
        self.hA = si.storage(a_st, o, self.lda)
        self.hB = si.storage(b_st, o, self.ldb)
        self.hC = si.storage(C0, o, self.ldc, pad_value=-7.0)
        self.dA = torch.from_numpy(self.hA).cuda()
        self.dB = torch.from_numpy(self.hB).cuda()
        self.dC = torch.from_numpy(self.hC).cuda()

    def run(self, mm, alpha, beta, path, n=3):
        import torch
        ta, tb = _flags(mm, self.ta, self.tb)
        ws, nb = None, 0
        if path == mm.PATH_FP8:
            nb = mm.gemm_fp8_workspace_bytes(self.M, self.N, self.K)
            ws = torch.zeros(nb, dtype=torch.uint8, device="cuda")
        mm.gemm_ex(_order(mm, self.o), ta, tb, self.M, self.N, self.K, alpha, self.dA, self.lda,
                   self.dB, self.ldb, beta, self.dC, self.ldc, path, n, ws, nb)
        torch.cuda.synchronize()
        buf = self.dC.cpu().numpy()
        # every element outside the M x N matrix keeps its padding value
        idx = np.arange(buf.size)
        if self.o == "C":
            r, c = idx // self.ldc, idx % self.ldc
            mask = (r < self.M) & (c < self.N)
        else:
            c, r = idx // self.ldc, idx % self.ldc
            mask = (r < self.M) & (c < self.N)
        assert np.all(buf[~mask] == -7.0)
        return si.unstorage(buf, self.o, self.M, self.N, self.ldc)

    def oracle_ref(self, alpha, beta):
        ta = oracle.TRANS if self.ta else oracle.NO_TRANS
        tb = oracle.TRANS if self.tb else oracle.NO_TRANS
        order = oracle.ROW_MAJOR if self.o == "C" else oracle.COL_MAJOR
        return oracle.gemm_op(order, ta, tb, self.M, self.N, self.K, alpha, self.hA, self.lda,
                              self.hB, self.ldb, beta, self.hC, self.ldc)


def _operands(M, N, K, seed, kind="uniform"):
    if kind == "integers":
        return si.integers((M, K), seed), si.integers((K, N), seed + 1), si.integers((M, N), seed + 2)
    return si.uniform((M, K), seed), si.uniform((K, N), seed + 1), si.uniform((M, N), seed + 2)


# Ragged shapes spanning several tiles; the library picks the 64 x 64 tile
# (three products) / 128 x 128 x 32 (six) / 128 x 128 FP32 matrix-core tile.
SMALL = [(300, 260, 333), (129, 67, 1001), (1, 130, 64), (77, 1, 257)]


@pytest.mark.parametrize("o", ORDERS)
@pytest.mark.parametrize("ta,tb", FLAGS)
@pytest.mark.parametrize("M,N,K", SMALL)
@pytest.mark.parametrize("n", [3, 6])
def test_split_path_parity(o, ta, tb, M, N, K, n):
    import paper_1902_10345_amd as mm
    opA, opB, C0 = _operands(M, N, K, M + 3 * N + 7 * K)
    p = Problem(opA, opB, C0, o, ta, tb)
    C = p.run(mm, 1.5, 0.5, mm.PATH_3XBF16, n)
    check_split_result(oracle, opA, opB, C0, C, 1.5, 0.5, n)


@pytest.mark.parametrize("o", ORDERS)
@pytest.mark.parametrize("ta,tb", FLAGS)
@pytest.mark.parametrize("M,N,K", SMALL)
def test_f32_path_parity(o, ta, tb, M, N, K):
    import paper_1902_10345_amd as mm
    opA, opB, C0 = _operands(M, N, K, 5 * M + N + K)
    p = Problem(opA, opB, C0, o, ta, tb)
    C = p.run(mm, 1.5, 0.5, mm.PATH_F32)
    ref = p.oracle_ref(1.5, 0.5)
    den = oracle.gemm_abs(opA, opB, alpha=1.5, beta=0.5, C0=C0)
    rel, _, _, cw = oracle.norms(C, ref, den)
    assert cw <= gamma(K), (cw, gamma(K))
    if M * N * K >= 32768:
        assert rel <= 1e-5, rel


@pytest.mark.parametrize("o", ORDERS)
@pytest.mark.parametrize("ta,tb", FLAGS)
def test_integer_inputs_are_exact_on_every_path(o, ta, tb):
    import torch
    import paper_1902_10345_amd as mm
    M, N, K = 200, 150, 700
    opA, opB, C0 = _operands(M, N, K, 91, kind="integers")
    p = Problem(opA, opB, C0, o, ta, tb)
    exact = oracle.gemm(opA, opB, alpha=2.0, beta=-1.0, C0=C0)
    for path, n in ((mm.PATH_F32, 3), (mm.PATH_3XBF16, 3), (mm.PATH_3XBF16, 6)):
        p.dC.copy_(torch.from_numpy(p.hC))
        C = p.run(mm, 2.0, -1.0, path, n)
        assert np.array_equal(C.astype(np.float64), exact), (path, n)


@pytest.mark.parametrize("o", ORDERS)
@pytest.mark.parametrize("n", [3, 6])
def test_flags_change_only_the_staging_bitwise(o, n):
    """Within one storage order, all four flag combinations of one logical
    problem return the same bits (same tile configuration, same LDS contents,
    same MFMA sequence)."""
    import paper_1902_10345_amd as mm
    M, N, K = 333, 270, 517
    opA, opB, C0 = _operands(M, N, K, 17)
    outs = [Problem(opA, opB, C0, o, ta, tb).run(mm, 1.5, 0.5, mm.PATH_3XBF16, n)
            for ta, tb in FLAGS]
    for C in outs[1:]:
        assert np.array_equal(C, outs[0])


def test_row_major_untransposed_equals_the_plain_entry_points():
    import torch
    import paper_1902_10345_amd as mm
    M, N, K = 300, 260, 333
    opA, opB, C0 = _operands(M, N, K, 23)
    for path, n in ((mm.PATH_3XBF16, 3), (mm.PATH_3XBF16, 6), (mm.PATH_F32, 3)):
        p = Problem(opA, opB, C0, "C", False, False, pad=0)
        C = p.run(mm, 1.5, 0.5, path, n)
        dA, dB, dC = (torch.from_numpy(x).cuda() for x in (opA, opB, C0))
        if path == mm.PATH_F32:
            mm.gemm_f32(M, N, K, 1.5, dA, K, dB, N, 0.5, dC, N)
        else:
            mm.gemm_f32_3xbf16(M, N, K, 1.5, dA, K, dB, N, 0.5, dC, N, n)
        torch.cuda.synchronize()
        assert np.array_equal(C, dC.cpu().numpy()), (path, n)


@pytest.mark.parametrize("ta,tb", FLAGS)
def test_fp8_row_major_flags_are_bitwise_the_untransposed_call(ta, tb):
    """A transposed operand is quantised by the other quantiser (rows of A^T
    as stored are columns of op(A)), giving the same codes and scales."""
    import paper_1902_10345_amd as mm
    M, N, K = 300, 260, 333
    A, B, C0 = si.fp8_workload(M, N, K, 61)
    base = Problem(A, B, C0, "C", False, False).run(mm, 1.5, 0.5, mm.PATH_FP8)
    got = Problem(A, B, C0, "C", ta, tb).run(mm, 1.5, 0.5, mm.PATH_FP8)
    assert np.array_equal(got, base)


@pytest.mark.parametrize("ta,tb", FLAGS)
@pytest.mark.parametrize("outliers", ["none", "A"])
def test_fp8_column_major_against_dequantised_oracle(ta, tb, outliers):
    """Column-major FP8 runs the row-major product C^T = op(B)^T op(A)^T:
    op(A)'s rows and op(B)'s columns keep their scales, so the result obeys
    the same dequantised-input bound as the row-major path."""
    from gpu_util import fp8_check
    import paper_1902_10345_amd as mm
    M, N, K = 260, 300, 1000
    A, B, C0 = si.fp8_workload(M, N, K, 71, outliers=outliers)
    C = Problem(A, B, C0, "F", ta, tb).run(mm, 1.5, 0.5, mm.PATH_FP8)
    sa, sb = oracle.fp8_scales_rows(A), oracle.fp8_scales_cols(B)
    qa, qb = oracle.fp8_quantize_rows(A, sa), oracle.fp8_quantize_cols(B, sb)
    ratio = fp8_check(oracle, C, qa, qb, sa, sb, 1.5, 0.5, C0)[1]
    assert ratio <= 1.0, ratio


# Shapes on which the library picks the larger tiles: 256 x 128 x 32 and
# 128 x 128 x 16 (three products), the 256 x 256 tiles (three and six
# products, FP32), and the 64 x 64 tile next to them.
@pytest.mark.parametrize("M,N,K", [(2085, 1998, 515), (4101, 4093, 300), (2560, 2560, 300),
                                   (3000, 3000, 300)])
@pytest.mark.parametrize("o", ORDERS)
@pytest.mark.parametrize("ta,tb", FLAGS[1:])
def test_large_tiles_sampled_rows(M, N, K, o, ta, tb):
    import torch
    import paper_1902_10345_amd as mm
    opA, opB, C0 = _operands(M, N, K, M + N)
    p = Problem(opA, opB, C0, o, ta, tb, pad=1)
    rows = sample_rows(M, 24, K)
    for path, n in ((mm.PATH_3XBF16, 3), (mm.PATH_3XBF16, 6), (mm.PATH_F32, 3)):
        p.dC.copy_(torch.from_numpy(p.hC))
        C = p.run(mm, 1.5, 0.5, path, n)
        if path == mm.PATH_3XBF16:
            check_split_result(oracle, opA[rows], opB, C0[rows], C[rows], 1.5, 0.5, n)
        else:
            ref = oracle.gemm(opA[rows], opB, alpha=1.5, beta=0.5, C0=C0[rows])
            den = oracle.gemm_abs(opA[rows], opB, alpha=1.5, beta=0.5, C0=C0[rows])
            rel, _, _, cw = oracle.norms(C[rows], ref, den)
            assert rel <= 1e-5 and cw <= gamma(K), (rel, cw)


@pytest.mark.parametrize("ta,tb", FLAGS[1:])
def test_full_size_4096_sampled_rows(ta, tb):
    """The benchmark's transposed 4096^3 products, default launch, 32 seeded
    rows against the oracle."""
    import paper_1902_10345_amd as mm
    M = N = K = 4096
    opA, opB, C0 = _operands(M, N, K, 2)
    p = Problem(opA, opB, C0, "C", ta, tb, pad=0)
    C = p.run(mm, 1.5, 0.5, mm.PATH_3XBF16, 3)
    rows = sample_rows(M, 32, 2)
    check_split_result(oracle, opA[rows], opB, C0[rows], C[rows], 1.5, 0.5, 3)


def test_quick_paths_and_empty_shapes():
    import torch
    import paper_1902_10345_amd as mm
    M, N = 70, 50
    C0 = si.uniform((M, N), 5)
    for o in ORDERS:
        ld = (N if o == "C" else M) + 2
        h = si.storage(C0, o, ld, pad_value=-7.0)
        d = torch.from_numpy(h).cuda()
        # K == 0: C <- beta*C, A and B unread (NULL)
        lda, ldb = (M, N) if o == "C" else (1, 1)
        mm.gemm_ex(_order(mm, o), mm.TRANS, mm.NO_TRANS, M, N, 0, 1.0, None, lda, None, ldb, 0.5,
                   d, ld, mm.PATH_3XBF16, 3)
        torch.cuda.synchronize()
        got = d.cpu().numpy()
        assert np.array_equal(si.unstorage(got, o, M, N, ld), (np.float32(0.5) * C0))
        assert np.all(got[si.storage(np.zeros((M, N), np.float32), o, ld, 1.0) == 1.0] == -7.0)


@pytest.mark.parametrize("path", ["f32", "3xbf16", "fp8"])
def test_tensor_helper_takes_transposed_views(path):
    """ops.gemm passes a column-contiguous view (A.t() of a row-major tensor)
    as a transposed operand: same bits as the call on materialised copies."""
    import torch
    import paper_1902_10345_amd as mm
    M, N, K = 150, 130, 170
    At = torch.from_numpy(si.uniform((K, M), 81)).cuda()   # stored K x M
    Bt = torch.from_numpy(si.uniform((N, K), 82)).cuda()   # stored N x K
    C0 = torch.from_numpy(si.uniform((M, N), 83)).cuda()
    got = mm.ops.gemm(At.t(), Bt.t(), C0.clone(), alpha=1.5, beta=0.5, path=path)
    ref = mm.ops.gemm(At.t().contiguous(), Bt.t().contiguous(), C0.clone(), alpha=1.5, beta=0.5,
                      path=path)
    torch.cuda.synchronize()
    if path == "f32":  # the untransposed call may pick the vector-ALU tile: tolerance
        d = (got - ref).abs().max().item()
        assert d <= 1e-4, d
    else:
        assert torch.equal(got, ref)


def test_tensor_helper_float64():
    import torch
    import paper_1902_10345_amd as mm
    from test_gpu_f64 import _check
    A, B, C0 = (si.uniform(s, 90 + i).astype(np.float64) for i, s in
                enumerate(((70, 90), (90, 60), (70, 60))))
    C = mm.ops.gemm(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(),
                    torch.from_numpy(C0).cuda(), alpha=1.5, beta=0.5)
    torch.cuda.synchronize()
    _check(A, B, C0, C.cpu().numpy(), 1.5, 0.5)
