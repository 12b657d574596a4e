/*
 * gemm_mi355x.h -- C ABI of the MI355X (gfx950) dense GEMM library.
 *
 * Operation (Ben-Nun et al., "Stateful Dataflow Multigraphs", SC'19):
 * matrix multiplication is the map A[i,k]*B[k,j] followed by a reduction over
 * k (Sec. 3.3, matrix-multiplication panel of Fig. "Write-Conflicts and
 * Reductions"); the library computes it with the BLAS scalars of the external
 * code call in Sec. 2.1:
 *
 *        C <- alpha * A*B + beta * C
 *
 * Conventions shared by every entry point
 *   - Layout: row-major.  A is MxK with row stride lda >= max(1,K); B is KxN
 *     with row stride ldb >= max(1,N); C is MxN with row stride ldc >= max(1,N).
 *     Strides are in elements.  gemm_ex adds column-major storage and
 *     transposed operands.
 *   - Pointers named A, B, C, workspace, arena are DEVICE pointers owned by
 *     the caller; the library never frees caller memory.  Pointers prefixed
 *     h (hA, hC_out, ...) are host pointers.
 *   - Every GPU entry point is asynchronous on the given stream.  Arguments
 *     are checked before anything is enqueued; a rejected call enqueues
 *     nothing.  The caller synchronises (stream or event) before reading C.
 *   - beta == 0: C is write-only (NaN/Inf already in C never propagate).
 *     alpha == 0 or K == 0: C <- beta*C and A, B are not read.
 *     M == 0 or N == 0: no-op.  Quick returns take precedence over the
 *     pointer checks (a pointer not needed may be NULL).
 *   - Status: 0 = success; -i = argument i (1-based, in declaration order) is
 *     invalid (BLAS xerbla convention); > 0 = runtime failure, see
 *     GEMM_STATUS_*.  gemm_last_error() returns a thread-local message for the
 *     most recent failure on the calling thread.
 *   - Results are deterministic: the same call on the same inputs gives
 *     bitwise-identical C (no atomics into C; the reduction order depends
 *     only on M, N, K, the path and the tile configuration).
 */
#ifndef GEMM_MI355X_H
#define GEMM_MI355X_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int gemm_status;

#define GEMM_STATUS_OK            0
#define GEMM_STATUS_HIP_ERROR     1  /* a HIP runtime call or launch failed */
#define GEMM_STATUS_NO_MEMORY     2  /* workspace/arena too small, allocation failed */
#define GEMM_STATUS_NOT_READY     3  /* server_poll: request still in flight */
#define GEMM_STATUS_UNSUPPORTED   4  /* e.g. device is not gfx950 */
#define GEMM_STATUS_REJECTED      5  /* server: request can never fit the budget */
#define GEMM_STATUS_UNKNOWN       6  /* server: unknown ticket */
#define GEMM_STATUS_CANCELLED     7  /* server: request cancelled before admission */
#define GEMM_STATUS_TIMED_OUT     8  /* server: request waited longer than the queue timeout */

/* Thread-local text of the last failure on this thread ("" if none). */
const char *gemm_last_error(void);

/* Library version string. */
const char *gemm_version(void);

/* ------------------------------------------------------------------------
 * Plain FP32 path: binary32 products and binary32 sums, no split.
 * C <- alpha*A*B + beta*C.  The library picks the tile configuration per
 * shape (gemm_default_config): where 256 x 256 or 128 x 128 tiles fill the
 * compute units, the binary32 matrix-core tile (v_mfma_f32_32x32x2_f32: each
 * product and sum in binary32); below that the small-product tiles (32 x 32
 * or 64 x 64 outputs per workgroup, the k range split over its eight waves
 * on the same matrix-core instruction, partial tiles summed in wave order).
 * The vector-ALU tiles (fused multiply-add accumulation in per-lane register
 * micro-tiles) remain configurations of the path: gemm_run_config selects
 * any of them.
 * Tiling of the (i,j) map, LDS staging of A/B tiles with double buffering and
 * register micro-tiles realise the MapTiling, LocalStorage, DoubleBuffering
 * and Vectorization steps of the paper's transformation chain (Sec. 6.2,
 * App. B table of transformations); alpha and beta are applied once in a
 * peeled epilogue (ReducePeeling, Sec. 6.2).
 * Arguments: 1 M, 2 N, 3 K, 4 alpha, 5 A, 6 lda, 7 B, 8 ldb, 9 beta, 10 C,
 * 11 ldc, 12 stream.
 * ---------------------------------------------------------------------- */
gemm_status gemm_f32(int64_t M, int64_t N, int64_t K, float alpha,
                     const float *A, int64_t lda, const float *B, int64_t ldb,
                     float beta, float *C, int64_t ldc, hipStream_t stream);

/* ------------------------------------------------------------------------
 * FP32-accurate split-precision path on bf16 MFMA (not in the paper).
 * Each binary32 operand element is split on the fly into bfloat16 planes
 * a = a0 + a1 + a2 (round-to-nearest-even at every level, exact sum) while the
 * tile is staged into LDS, and
 *   n_products == 3 : acc += a0*b0 + a0*b1 + a1*b0
 *   n_products == 6 : acc += the above + a0*b2 + a1*b1 + a2*b0
 * with binary32 MFMA accumulation.  Arguments as gemm_f32, then
 * 12 n_products (3 or 6), 13 stream.
 * ---------------------------------------------------------------------- */
gemm_status gemm_f32_3xbf16(int64_t M, int64_t N, int64_t K, float alpha,
                            const float *A, int64_t lda, const float *B, int64_t ldb,
                            float beta, float *C, int64_t ldc, int n_products,
                            hipStream_t stream);

/* Split-K form of gemm_f32_3xbf16, for shapes whose output tiles alone leave
 * compute units idle (few or thin tiles, deep K).  The reduction over k is cut
 * into `splits` chunks of whole 16-deep (32-deep for 6 products) slabs; each
 * (chunk, 128 x 128 output tile) pair is one workgroup that writes its partial
 * product to the workspace, and a second kernel resolves the write conflict of
 * the chunks on C -- the write-conflict resolution of a reduction (Sec. 3.3,
 * write-conflict resolution memlets; App. A, the wcr attribute), here an
 * ordered sum rather than atomics -- by summing them in chunk order and applying
 * alpha and beta (C <- alpha * sum_c P_c + beta * C; beta == 0: C is not
 * read).  Deterministic for a given (shape, n_products, splits); with one
 * chunk the result equals that of the 128 x 128 tile configuration
 * (gemm_run_config, configuration "bx3_128x128x16_4w64x64_p3" or
 * "bx3_128x128x32_4w64x64_p6") bit for bit.
 * splits: 1..64, or 0 for gemm_splitk_default_splits (enough chunks for two
 * workgroups per compute unit, each chunk at least 256 deep).
 * workspace: device memory of at least gemm_splitk_workspace_bytes(M, N, K,
 * splits) bytes (splits * M * N floats; 0 bytes, and NULL allowed, when the
 * split count resolves to 1), 256-byte aligned, owned by the caller.
 * Arguments: 1..11 as gemm_f32, 12 n_products, 13 splits, 14 workspace,
 * 15 ws_bytes, 16 stream.  Returns -14 / -15 for a missing, misaligned or
 * short workspace. */
int gemm_splitk_default_splits(int64_t M, int64_t N, int64_t K);
size_t gemm_splitk_workspace_bytes(int64_t M, int64_t N, int64_t K, int splits);
gemm_status gemm_f32_3xbf16_splitk(int64_t M, int64_t N, int64_t K, float alpha,
                                   const float *A, int64_t lda, const float *B, int64_t ldb,
                                   float beta, float *C, int64_t ldc, int n_products,
                                   int splits, void *workspace, size_t ws_bytes,
                                   hipStream_t stream);

/* The split-K product above for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): no workspace argument; the partial planes live in a fixed
 * device array of GEMM_NOALLOC_SCRATCH_BYTES bytes inside the library, one
 * copy per device, held until the process ends and resolved on the first
 * call with that device current.  No device memory is allocated or freed by
 * the call.  Every call on one device shares that device's array, so calls
 * that overlap on one device race: serialise them (one stream).  Results are
 * bitwise those of gemm_f32_3xbf16_splitk with the same split count.
 * Arguments: 1..13 as gemm_f32_3xbf16_splitk, 14 stream.  Returns
 * GEMM_STATUS_NO_MEMORY, with nothing enqueued, when splits * M * N * 4
 * bytes (after resolving splits = 0 to the default; 0 bytes when the count
 * resolves to 1) exceed GEMM_NOALLOC_SCRATCH_BYTES. */
#define GEMM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
gemm_status gemm_f32_3xbf16_splitk_noalloc(int64_t M, int64_t N, int64_t K, float alpha,
                                           const float *A, int64_t lda, const float *B,
                                           int64_t ldb, float beta, float *C, int64_t ldc,
                                           int n_products, int splits, hipStream_t stream);

/* The staging split alone, for verification: x (n floats, device) ->
 * planes p0, p1, p2 (n bfloat16 bit patterns each, device; p2 may be NULL).
 * Arguments: 1 n, 2 x, 3 p0, 4 p1, 5 p2, 6 stream. */
gemm_status split_bf16x3(int64_t n, const float *x, uint16_t *p0, uint16_t *p1,
                         uint16_t *p2, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Scaled FP8 path (not in the paper).  OCP E4M3 (max 448) operands with
 * binary32 per-row scales of A and per-column scales of B:
 *   sa[i] = max_k |A[i,k]| / 448,  sb[j] = max_k |B[k,j]| / 448 (0 -> 1),
 *   qa = e4m3_rne_sat(A / sa),     qb = e4m3_rne_sat(B / sb),
 *   C <- alpha * sa[i]*sb[j] * sum_k qa*qb + beta*C   (binary32 accumulation).
 * The quantised operands and scales live in a caller-provided device
 * workspace of at least gemm_fp8_workspace_bytes(M,N,K) bytes, laid out as
 * [qa: M x Kp bytes][qb^T: N x Kp bytes][sa: M floats][sb: N floats]
 * [max(M,N) uint32 of scratch], each region 256-byte aligned, Kp = K rounded up to a
 * multiple of 128 (the padding holds zero codes).  qb is stored transposed
 * (column j of B contiguous).  Codes are E4M3 bit patterns (sign, 4 exponent
 * bits with bias 7, 3 mantissa bits; 0x7E = 448, no infinities).
 * Arguments: 1..11 as gemm_f32, 12 workspace, 13 ws_bytes, 14 stream.
 * ---------------------------------------------------------------------- */
size_t gemm_fp8_workspace_bytes(int64_t M, int64_t N, int64_t K);
gemm_status gemm_fp8_scaled(int64_t M, int64_t N, int64_t K, float alpha,
                            const float *A, int64_t lda, const float *B, int64_t ldb,
                            float beta, float *C, int64_t ldc, void *workspace,
                            size_t ws_bytes, hipStream_t stream);
/* The two halves of gemm_fp8_scaled: quantise A and B into the workspace,
 * then multiply the quantised operands already in the workspace.
 * fp8_quantize arguments: 1 M, 2 N, 3 K, 4 A, 5 lda, 6 B, 7 ldb, 8 workspace,
 * 9 ws_bytes, 10 stream.  gemm_fp8_prequantized arguments: 1 M, 2 N, 3 K,
 * 4 alpha, 5 workspace, 6 ws_bytes, 7 beta, 8 C, 9 ldc, 10 stream. */
gemm_status fp8_quantize(int64_t M, int64_t N, int64_t K, const float *A, int64_t lda,
                         const float *B, int64_t ldb, void *workspace, size_t ws_bytes,
                         hipStream_t stream);
gemm_status gemm_fp8_prequantized(int64_t M, int64_t N, int64_t K, float alpha,
                                  const void *workspace, size_t ws_bytes, float beta,
                                  float *C, int64_t ldc, hipStream_t stream);
/* The E4M3 encoder alone, for verification: codes[i] = e4m3_rne_sat(x[i])
 * (NaN -> 0x7F; the sign of a value that rounds to zero is kept).
 * Arguments: 1 n, 2 x (device floats), 3 codes (device bytes), 4 stream. */
gemm_status fp8_e4m3_encode(int64_t n, const float *x, uint8_t *codes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Binary64 path on the FP64 matrix cores (v_mfma_f64_16x16x4f64).
 * C <- alpha*A*B + beta*C with binary64 operands, products and sums, for the
 * double-precision workloads the paper evaluates (the Polybench kernels run
 * mostly in double precision, Sec. 6.1; the batched-strided small products of
 * the quantum-transport case study, Sec. 6.4 and table "Strided Matrix
 * Multiplication Performance", are double precision by the peak they are
 * measured against).  Layout, quick returns, status codes and determinism as
 * gemm_f32.  Arguments: 1 M, 2 N, 3 K, 4 alpha, 5 A, 6 lda, 7 B, 8 ldb,
 * 9 beta, 10 C, 11 ldc, 12 stream.
 * ---------------------------------------------------------------------- */
gemm_status gemm_f64(int64_t M, int64_t N, int64_t K, double alpha,
                     const double *A, int64_t lda, const double *B, int64_t ldb,
                     double beta, double *C, int64_t ldc, hipStream_t stream);

/* Batched-strided binary64 product (SBSMM, Sec. 6.4): `batch` independent
 * problems of one shape, problem b reading A + b*stride_a, B + b*stride_b and
 * updating C + b*stride_c (strides in elements; a zero input stride reuses
 * one matrix for every problem).  Output matrices must not overlap:
 * stride_c >= (M-1)*ldc + N when batch > 1.  One launch covers up to 65535
 * problems (more are issued as consecutive launches on the stream).
 * Arguments: 1 M, 2 N, 3 K, 4 alpha, 5 A, 6 lda, 7 stride_a, 8 B, 9 ldb,
 * 10 stride_b, 11 beta, 12 C, 13 ldc, 14 stride_c, 15 batch, 16 stream. */
gemm_status gemm_f64_strided_batched(int64_t M, int64_t N, int64_t K, double alpha,
                                     const double *A, int64_t lda, int64_t stride_a,
                                     const double *B, int64_t ldb, int64_t stride_b,
                                     double beta, double *C, int64_t ldc, int64_t stride_c,
                                     int64_t batch, hipStream_t stream);

/* Batched-strided binary32 product (SBSMM, Sec. 6.4, on the binary32 paths):
 * `batch` independent problems of one shape, problem b reading
 * A + b*stride_a, B + b*stride_b and updating C + b*stride_c (strides in
 * elements; zero input strides reuse one matrix).  path: GEMM_PATH_F32
 * (binary32 products on the FP32 matrix cores) or GEMM_PATH_3XBF16
 * (n_products 3 or 6, as gemm_f32_3xbf16).  Output matrices must not
 * overlap: stride_c >= (M-1)*ldc + N when batch > 1.  Layout and quick
 * returns as gemm_f32; up to 65535 problems per launch.  Small problems (M,
 * N <= 64; with three products also M*N <= 48*48) run one wave per problem
 * (no LDS staging), with results bitwise those of the library's matrix-core
 * tiles of the same arithmetic.  Arguments: 1 path,
 * 2 M, 3 N, 4 K, 5 alpha, 6 A, 7 lda, 8 stride_a, 9 B, 10 ldb, 11 stride_b,
 * 12 beta, 13 C, 14 ldc, 15 stride_c, 16 batch, 17 n_products, 18 stream. */
gemm_status gemm_strided_batched(int path, int64_t M, int64_t N, int64_t K, float alpha,
                                 const float *A, int64_t lda, int64_t stride_a, const float *B,
                                 int64_t ldb, int64_t stride_b, float beta, float *C, int64_t ldc,
                                 int64_t stride_c, int64_t batch, int n_products,
                                 hipStream_t stream);

/* gemm_f64 with an explicit tile configuration of GEMM_PATH_F64 (0 <= cfg <
 * gemm_num_configs(GEMM_PATH_F64), or -1 for the default).  Arguments: 1 cfg,
 * then 2..13 as gemm_f64's 1..12. */
gemm_status gemm_f64_run_config(int cfg, int64_t M, int64_t N, int64_t K, double alpha,
                                const double *A, int64_t lda, const double *B, int64_t ldb,
                                double beta, double *C, int64_t ldc, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Tile configurations (for the autotuner and for per-configuration tests).
 * Every configuration of a path computes the same operation; results may
 * differ between configurations only by binary32 summation order.
 * path: GEMM_PATH_F32, GEMM_PATH_3XBF16, GEMM_PATH_FP8 (quantise A and B into
 * the workspace, then multiply) or GEMM_PATH_FP8_PREQUANTIZED (multiply the
 * codes and scales already in the workspace, as gemm_fp8_prequantized; A, B,
 * lda and ldb are ignored and may be NULL / 0).  The two FP8 paths share one
 * set of configurations and one autotuner entry per size bucket.
 * gemm_run_config: arguments 1 path, 2 cfg (0 <= cfg < gemm_num_configs, or
 * -1 for the library's default choice), then 3..13 as gemm_f32's 1..11,
 * 14 n_products (3XBF16 only; ignored otherwise), 15 workspace, 16 ws_bytes
 * (FP8 paths only; ignored otherwise), 17 stream.
 * ---------------------------------------------------------------------- */
#define GEMM_PATH_F32     0
#define GEMM_PATH_3XBF16  1
#define GEMM_PATH_FP8     2
#define GEMM_PATH_FP8_PREQUANTIZED 3
#define GEMM_PATH_F64     4  /* configurations only (gemm_num_configs, gemm_config_name,
                                gemm_default_config); run with gemm_f64_run_config */
int gemm_num_configs(int path);
const char *gemm_config_name(int path, int cfg);
/* Default configuration the library picks for this shape on the current device. */
int gemm_default_config(int path, int64_t M, int64_t N, int64_t K);
gemm_status gemm_run_config(int path, int cfg, int64_t M, int64_t N, int64_t K, float alpha,
                            const float *A, int64_t lda, const float *B, int64_t ldb,
                            float beta, float *C, int64_t ldc, int n_products,
                            void *workspace, size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Storage order and transposed operands, BLAS style.  The external-code call
 * of the paper (Sec. 2.1) passes a storage order and transpose flags with its
 * matrix product; gemm_ex accepts them:
 *
 *        C <- alpha * op(A) * op(B) + beta * C,   op(X) = X or X^T,
 *
 * op(A) is M x K, op(B) is K x N, C is M x N, each stored in `order`
 * (GEMM_ROW_MAJOR: element (r, c) at r*ld + c; GEMM_COL_MAJOR: at c*ld + r).
 * With trans_a == GEMM_TRANS, A is stored as the K x M matrix A^T, likewise
 * B as N x K (GEMM_CONJ_TRANS is the same for real data).  Leading
 * dimensions bound the stored row (row-major) or column (column-major)
 * length: lda >= max(1, stored extent of A along its contiguous index), and
 * so on: row-major lda >= K (no trans) or M (trans), ldb >= N or K, ldc >= N;
 * column-major lda >= M or K, ldb >= K or N, ldc >= M.  The values of the
 * enumerators are those of CBLAS.
 * A column-major call is the row-major product C^T = op(B)^T op(A)^T with the
 * operands exchanged; no data is moved.  Transposed operands change only how
 * tiles are staged into LDS, not the arithmetic: a row-major call with both
 * flags GEMM_NO_TRANS returns the same bits as gemm_f32 / gemm_f32_3xbf16 /
 * gemm_fp8_scaled.
 * path: GEMM_PATH_F32 (binary32 products; transposed operands run on the FP32
 * matrix-core tiles), GEMM_PATH_3XBF16 (n_products 3 or 6) or GEMM_PATH_FP8
 * (workspace of at least gemm_fp8_workspace_bytes(M, N, K) bytes, 256-byte
 * aligned; ignored, and may be NULL, on the other paths).
 * Arguments: 1 order, 2 trans_a, 3 trans_b, 4 M, 5 N, 6 K, 7 alpha, 8 A,
 * 9 lda, 10 B, 11 ldb, 12 beta, 13 C, 14 ldc, 15 path, 16 n_products,
 * 17 workspace, 18 ws_bytes, 19 stream.
 * ---------------------------------------------------------------------- */
#define GEMM_ROW_MAJOR   101
#define GEMM_COL_MAJOR   102
#define GEMM_NO_TRANS    111
#define GEMM_TRANS       112
#define GEMM_CONJ_TRANS  113
gemm_status gemm_ex(int order, int trans_a, int trans_b, int64_t M, int64_t N, int64_t K,
                    float alpha, const float *A, int64_t lda, const float *B, int64_t ldb,
                    float beta, float *C, int64_t ldc, int path, int n_products,
                    void *workspace, size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Grouped GEMM: many independent problems of uneven sizes in ONE persistent
 * launch on the 3xBF16 path (3 products).  Workgroups dequeue output tiles
 * from an atomic counter, the batch-dequeue mechanism the paper uses for
 * consume scopes (Sec. 3.3), and each problem runs with its own tile shape.
 *
 * gemm_problem: one C <- alpha*A*B + beta*C with the conventions above
 * (device pointers owned by the caller).  A problem with M == 0 or N == 0 is
 * skipped; alpha == 0 or K == 0 gives C <- beta*C.
 *
 * tile_variant: per-problem tile shape (0: 128 x 128, 1: 64 x 64), or NULL
 * for the library's choice (grouped_default_variant).  The autotuner
 * (grouped_autotune) returns such an array.
 *
 * workspace: device memory of at least grouped_gemm_workspace_bytes(count)
 * bytes, 256-byte aligned, owned by the caller; it holds the tile counter and
 * the descriptor table.  Calls that share a workspace must not overlap.
 *
 * grouped_gemm uploads the descriptor table with a stream synchronisation
 * (the host table is released on return) and then enqueues the launch.
 * Arguments: 1 problems (host array), 2 count, 3 path (GEMM_PATH_3XBF16),
 * 4 tile_variant (host array or NULL), 5 workspace, 6 ws_bytes, 7 stream.
 *
 * grouped_graph_create uploads the table once and captures the launch (a
 * counter-clearing kernel and the persistent kernel, no memset nodes) into
 * an executable HIP graph; grouped_graph_launch replays it on a stream with
 * no host work; the workspace and the problems' buffers must stay valid until
 * grouped_graph_destroy.  Arguments of create: 1..6 as grouped_gemm,
 * 7 stream used for the upload, 8 graph (out).
 * ---------------------------------------------------------------------- */
typedef struct gemm_problem {
  int64_t M, N, K, lda, ldb, ldc;
  const float *A;
  const float *B;
  float *C;
  float alpha, beta;
} gemm_problem;

size_t grouped_gemm_workspace_bytes(int count);
int grouped_default_variant(int64_t M, int64_t N, int64_t K);
gemm_status grouped_gemm(const gemm_problem *problems, int count, int path,
                         const int *tile_variant, void *workspace, size_t ws_bytes,
                         hipStream_t stream);
gemm_status grouped_graph_create(const gemm_problem *problems, int count, int path,
                                 const int *tile_variant, void *workspace, size_t ws_bytes,
                                 hipStream_t stream, void **graph);
gemm_status grouped_graph_launch(void *graph, hipStream_t stream);
gemm_status grouped_graph_destroy(void *graph);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of GEMM requests on one GPU.
 *
 * A server owns a caller-provided device arena (the HBM operand budget; the
 * memory stays owned by the caller, e.g. a torch tensor) and a scheduler
 * thread.  Requests enter a FIFO; the head is admitted when a slot
 * (max_slots requests in flight) and room in the arena are free, its operands
 * are copied into the arena and it joins the next step: one grouped launch on
 * the next idle stream of n_streams (default priority).  Steps on different
 * streams overlap on the device, so requests that arrive while others run are
 * admitted as slots and memory free up -- independent work on separate
 * streams, as the paper maps connected components of a dataflow graph to
 * concurrent GPU streams (Sec. 3.3, "Concurrency").  A request's tile shape
 * depends only on its (M, N), so its result is bitwise the same alone and in
 * any mix.  Host buffers should be pinned (hipHostMalloc, torch
 * pin_memory) for asynchronous copies and must stay valid until the request
 * completes; hC_out receives the MxN result.
 *
 * Latency = arrival (the caller's stamp on the server clock, or the submit
 * time when arrival < 0) to the host observing the completion of the request's
 * kernel; result latency additionally includes the copy of C to hC_out.
 *
 * server_create arguments: 1 arena (device, 256-byte aligned), 2 arena_bytes,
 * 3 max_slots [1, 4096], 4 path (GEMM_PATH_3XBF16), 5 n_streams [1, 16],
 * 6 out.  server_submit arguments: 1 server, 2 M, 3 N, 4 K, 5 alpha, 6 hA,
 * 7 hB, 8 beta, 9 hC0 (read when beta != 0), 10 hC_out, 11 arrival (seconds on
 * the server clock, or < 0), 12 ticket (out).  A request larger than the whole
 * arena returns GEMM_STATUS_REJECTED; one whose K or N exceeds the grouped
 * kernel's 32-bit tile offsets ((129 K) * 4 or (33 N) * 4 bytes >= 2^31)
 * returns GEMM_STATUS_UNSUPPORTED; both count as rejected.  server_poll
 * returns GEMM_STATUS_NOT_READY until the result is in hC_out, then the
 * latencies (and forgets the ticket).  A request that ended without a result
 * is reported once by server_poll with its status and then forgotten:
 * GEMM_STATUS_HIP_ERROR (its step's copies or launch could not be enqueued,
 * or the device reported an error; hC_out holds no result),
 * GEMM_STATUS_CANCELLED or GEMM_STATUS_TIMED_OUT.  After a device error
 * reported asynchronously the server is failed: server_submit and
 * server_drain return GEMM_STATUS_HIP_ERROR.  For tests of the error path the
 * environment variable GEMM_SERVER_INJECT_STEP_FAILURES=n, read by
 * server_create, makes the first n steps fail before anything is enqueued.
 *
 * server_cancel removes a request that is still queued (not yet admitted);
 * its poll then returns GEMM_STATUS_CANCELLED.  An admitted request cannot be
 * cancelled (GEMM_STATUS_NOT_READY: it completes normally).  Arguments:
 * 1 server, 2 ticket.  server_set_queue_timeout drops queued requests that
 * waited longer than `seconds` since their arrival stamp without being
 * admitted (0, the default, waits forever).  Arguments: 1 server, 2 seconds.
 * ---------------------------------------------------------------------- */
typedef struct gemm_server gemm_server;
gemm_status server_create(void *arena, size_t arena_bytes, int max_slots, int path,
                          int n_streams, gemm_server **out);
double server_now(gemm_server *server);
gemm_status server_submit(gemm_server *server, int64_t M, int64_t N, int64_t K, float alpha,
                          const float *hA, const float *hB, float beta, const float *hC0,
                          float *hC_out, double arrival, uint64_t *ticket);
gemm_status server_poll(gemm_server *server, uint64_t ticket, double *latency_ms,
                        double *result_latency_ms);
/* Blocks until every submitted request has completed (or timeout_s passes:
 * GEMM_STATUS_NOT_READY). */
gemm_status server_drain(gemm_server *server, double timeout_s);
gemm_status server_cancel(gemm_server *server, uint64_t ticket);
gemm_status server_set_queue_timeout(gemm_server *server, double seconds);
/* Latency percentiles over completed requests, throughput (completed
 * algorithmic flops over first arrival .. last completion), counters:
 * max_in_flight (admitted requests at once), arena_high_water (bytes),
 * rejected (at submit), failed (ended with GEMM_STATUS_HIP_ERROR) and
 * max_concurrent_steps (steps enqueued on different streams and not yet
 * complete at once).  Every output pointer may be NULL. */
gemm_status server_stats(gemm_server *server, double *p50_ms, double *p99_ms, double *tflops,
                         uint64_t *completed, double *result_p50_ms, double *result_p99_ms,
                         int *max_in_flight, size_t *arena_high_water, uint64_t *rejected,
                         uint64_t *failed, int *max_concurrent_steps);
gemm_status server_destroy(gemm_server *server);

/* ------------------------------------------------------------------------
 * Autotuner: size-specific tuning of tile parameters (the paper tunes
 * transformation parameters for a specific size, Sec. 6.2).
 *
 * gemm_autotune times every configuration of `path` (matching n_products on
 * GEMM_PATH_3XBF16) on the caller's operands (C is overwritten), keeps the
 * fastest for the size bucket of (M, N, K) (powers of two) and returns it;
 * afterwards the entry points use the tuned choice for every shape in that
 * bucket.  Arguments: 1 path, 2..12 as gemm_f32's 1..11, 13 n_products,
 * 14 workspace, 15 ws_bytes (FP8), 16 reps, 17 stream, 18 best_cfg (out).
 *
 * grouped_autotune times candidate tile-shape policies for a grouped batch
 * (the padded-work rule at several relative costs of a 64 x 64 tile element,
 * including 0 -- every problem on 64 x 64 tiles -- and a cost so large that
 * every problem takes 128 x 128 tiles) and writes the fastest per-problem
 * variants to variants_out (count ints); the winning rule becomes the
 * library's, so grouped_default_variant and grouped calls without explicit
 * variants reproduce variants_out for these problems.  Arguments: 1 problems, 2 count, 3 path, 4 workspace,
 * 5 ws_bytes, 6 reps, 7 stream, 8 variants_out.
 *
 * gemm_tuner_save / gemm_tuner_load write and read the tuned table as JSON.
 * ---------------------------------------------------------------------- */
gemm_status gemm_autotune(int path, int64_t M, int64_t N, int64_t K, float alpha, const float *A,
                          int64_t lda, const float *B, int64_t ldb, float beta, float *C,
                          int64_t ldc, int n_products, void *workspace, size_t ws_bytes,
                          int reps, hipStream_t stream, int *best_cfg);
gemm_status grouped_autotune(const gemm_problem *problems, int count, int path, void *workspace,
                             size_t ws_bytes, int reps, hipStream_t stream, int *variants_out);
gemm_status gemm_tuner_save(const char *json_path);
gemm_status gemm_tuner_load(const char *json_path);
/* Forget every tuned choice (back to the library's default heuristics). */
void gemm_tuner_clear(void);

/* ------------------------------------------------------------------------
 * FP64 on-device error norm (verification only).
 * C (binary32, MxN, row stride ldc) against Cref (binary64, MxN dense); den
 * (binary64, MxN dense) may be NULL.  Writes four doubles to out (device):
 *   out[0] = ||C - Cref||_F / ||Cref||_F  (||C - Cref||_F if Cref == 0)
 *   out[1] = sum (C - Cref)^2,  out[2] = sum Cref^2,
 *   out[3] = max |C - Cref| / den  (0/0 -> 0, x/0 -> inf), or max |C - Cref|
 *            when den is NULL.
 * The reduction order is fixed (deterministic).  workspace must hold
 * err_norm_workspace_bytes() bytes of device memory.
 * Arguments: 1 M, 2 N, 3 C, 4 ldc, 5 Cref, 6 den, 7 out, 8 workspace,
 * 9 ws_bytes, 10 stream.
 * ---------------------------------------------------------------------- */
size_t err_norm_workspace_bytes(void);
gemm_status err_norm_f64(int64_t M, int64_t N, const float *C, int64_t ldc,
                         const double *Cref, const double *den, double *out,
                         void *workspace, size_t ws_bytes, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* GEMM_MI355X_H */
