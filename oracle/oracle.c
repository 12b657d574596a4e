/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct CPU reference for everything the GPU GEMM
 * library computes.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load this file's shared object.  It shares no code,
 * header, table or constant with the HIP library: every function below is
 * written from the definition of the quantity it computes.
 *
 * Problem statement (Ben-Nun et al., "Stateful Dataflow Multigraphs", SC'19):
 *   - matrix multiplication as a map producing tmp[i,j,k] = A[i,k]*B[k,j]
 *     followed by a reduction over k (Sec. 3.3, Fig. "Write-Conflicts and
 *     Reductions", matrix multiplication panel);
 *   - the BLAS-style call with scalars alpha and beta (Sec. 2.1, Fig.
 *     "External Code in DaCe").
 *   The oracle therefore computes, in binary64,
 *       Cref[i,j] = alpha * sum_k A[i,k]*B[k,j] + (beta == 0 ? 0 : beta*C0[i,j]).
 *   Any summation order is a valid schedule (App. A, operational semantics:
 *   execution order inside a state is unconstrained beyond dependencies), so
 *   the k-loop runs in natural order in binary64.
 *
 * The precision variants (bf16 three-way split, e4m3 scaled quantisation) are
 * not in the paper; their definitions here follow the IEEE-754 round-to-
 * nearest-even rule and the OCP 8-bit floating point (OFP8) E4M3 format.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC (no -ffast-math: float division and
 * rounding must be IEEE-exact for the quantiser).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- GEMM --- */

/* Cref = alpha * A*B + beta*C0, all in binary64 (Sec. 3.3 map-reduce MM with
 * the BLAS scalars of Sec. 2.1).  A is MxK (row stride lda), B is KxN (row
 * stride ldb), C0 is MxN (row stride ldc0; never read when beta == 0, per the
 * BLAS convention), Cref is MxN dense (row stride N).
 * absolute != 0 computes the Higham denominator |alpha|*|A||B| + |beta|*|C0|
 * instead, used for componentwise error bounds. */
void orc_gemm(int64_t M, int64_t N, int64_t K, double alpha,
              const float *A, int64_t lda, const float *B, int64_t ldb,
              double beta, const float *C0, int64_t ldc0, double *Cref,
              int absolute, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < M; ++i) {
        double *row = Cref + i * N;
        for (int64_t j = 0; j < N; ++j) row[j] = 0.0;
        for (int64_t k = 0; k < K; ++k) {
            double a = (double)A[i * lda + k];
            if (absolute) a = fabs(a);
            const float *brow = B + k * ldb;
            for (int64_t j = 0; j < N; ++j) {
                double b = (double)brow[j];
                if (absolute) b = fabs(b);
                row[j] += a * b;
            }
        }
        for (int64_t j = 0; j < N; ++j) {
            double al = absolute ? fabs(alpha) : alpha;
            double v = al * row[j];
            if (beta != 0.0) {
                double c = (double)C0[i * ldc0 + j];
                v += absolute ? fabs(beta) * fabs(c) : beta * c;
            }
            row[j] = v;
        }
    }
}

/* -------------------------------------------------- bf16 RNE and split --- */

/* Round a finite binary32 value to the nearest bfloat16 value (8 significant
 * bits, same exponent range as binary32), ties to even.  Written from the
 * definition: find the quantum (spacing of bfloat16 values in the binade of
 * x; below the smallest normal binade the spacing is fixed at 2^-133), divide,
 * round to the nearest integer with ties to even (rint under the default
 * rounding mode), multiply back.  All steps are exact in binary64. */
static double bf16_rne(double x)
{
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    (void)frexp(x, &e);                /* |x| = m * 2^e, m in [0.5, 1) */
    if (e < -125) e = -125;            /* subnormal binade: fixed spacing */
    double quantum = ldexp(1.0, e - 8);/* 8 significant bits */
    return rint(x / quantum) * quantum;
}

float orc_bf16_rne(float x) { return (float)bf16_rne((double)x); }

/* Three-way split with round-to-nearest-even at every level:
 *   a0 = rne(a), r1 = a - a0 (exact), a1 = rne(r1), a2 = rne(r1 - a1).
 * For |a| >= 2^-100 the last rounding is exact (r1 - a1 needs at most 8
 * significant bits and lies in bfloat16's normal range), so a0 + a1 + a2 == a;
 * below that the last plane may fall on bfloat16's subnormal grid (spacing
 * 2^-133) and is rounded there.  Output planes hold the bfloat16 values as
 * floats. */
void orc_split_bf16x3(int64_t n, const float *x, float *p0, float *p1, float *p2)
{
    for (int64_t t = 0; t < n; ++t) {
        double a = (double)x[t];
        double a0 = bf16_rne(a);
        double r1 = a - a0;
        double a1 = bf16_rne(r1);
        double a2 = bf16_rne(r1 - a1);
        p0[t] = (float)a0;
        p1[t] = (float)a1;
        p2[t] = (float)a2;
    }
}

/* Sum of the selected split products in binary64:
 *   n_products == 3 : a0*b0 + a0*b1 + a1*b0
 *   n_products == 6 : the above + a0*b2 + a1*b1 + a2*b0
 *   n_products == 1 : a0*b0
 * Cref = alpha * sum + (beta == 0 ? 0 : beta*C0).  This is the exact value a
 * split-precision kernel approximates with binary32 accumulation. */
void orc_gemm_bf16_split(int64_t M, int64_t N, int64_t K, double alpha,
                         const float *A, int64_t lda, const float *B, int64_t ldb,
                         double beta, const float *C0, int64_t ldc0,
                         int n_products, double *Cref, int nthreads)
{
    float *a0 = malloc(sizeof(float) * (size_t)(M * K > 0 ? M * K : 1));
    float *a1 = malloc(sizeof(float) * (size_t)(M * K > 0 ? M * K : 1));
    float *a2 = malloc(sizeof(float) * (size_t)(M * K > 0 ? M * K : 1));
    float *b0 = malloc(sizeof(float) * (size_t)(K * N > 0 ? K * N : 1));
    float *b1 = malloc(sizeof(float) * (size_t)(K * N > 0 ? K * N : 1));
    float *b2 = malloc(sizeof(float) * (size_t)(K * N > 0 ? K * N : 1));
    for (int64_t i = 0; i < M; ++i)
        orc_split_bf16x3(K, A + i * lda, a0 + i * K, a1 + i * K, a2 + i * K);
    for (int64_t k = 0; k < K; ++k)
        orc_split_bf16x3(N, B + k * ldb, b0 + k * N, b1 + k * N, b2 + k * N);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < M; ++i) {
        double *row = Cref + i * N;
        for (int64_t j = 0; j < N; ++j) row[j] = 0.0;
        for (int64_t k = 0; k < K; ++k) {
            double x0 = a0[i * K + k], x1 = a1[i * K + k], x2 = a2[i * K + k];
            for (int64_t j = 0; j < N; ++j) {
                double y0 = b0[k * N + j], y1 = b1[k * N + j], y2 = b2[k * N + j];
                double s = x0 * y0;
                if (n_products >= 3) s += x0 * y1 + x1 * y0;
                if (n_products >= 6) s += x0 * y2 + x1 * y1 + x2 * y0;
                row[j] += s;
            }
        }
        for (int64_t j = 0; j < N; ++j) {
            double v = alpha * row[j];
            if (beta != 0.0) v += beta * (double)C0[i * ldc0 + j];
            row[j] = v;
        }
    }
    free(a0); free(a1); free(a2); free(b0); free(b1); free(b2);
}

/* ------------------------------------------------------ OFP8 E4M3 (fn) --- */

/* Value of an E4M3 code: sign bit, 4 exponent bits with bias 7, 3 mantissa
 * bits; exponent field 0 encodes subnormals m/8 * 2^-6; the single NaN
 * pattern per sign is exponent 1111 with mantissa 111; there is no infinity.
 * Largest finite magnitude: 1.75 * 2^8 = 448. */
double orc_e4m3_value(uint8_t code)
{
    int s = code >> 7, e = (code >> 3) & 15, m = code & 7;
    double v;
    if (e == 15 && m == 7) return NAN;
    if (e == 0) v = ldexp((double)m / 8.0, -6);
    else        v = ldexp(1.0 + (double)m / 8.0, e - 7);
    return s ? -v : v;
}

void orc_e4m3_decode(int64_t n, const uint8_t *codes, float *out)
{
    for (int64_t t = 0; t < n; ++t) out[t] = (float)orc_e4m3_value(codes[t]);
}

/* Encode a binary32 value to E4M3 by round-to-nearest, ties to the even code,
 * with saturation: the nearest code is found by scanning all 127 non-negative
 * finite codes in increasing order (their values increase with the code), so
 * any magnitude above 448 lands on 448.  The sign bit is copied from x, so a
 * negative value that rounds to zero gives the negative-zero code 0x80.
 * NaN encodes to 0x7F (positive NaN pattern). */
uint8_t orc_e4m3_encode1(float x)
{
    if (isnan(x)) return 0x7F;
    double ax = fabs((double)x);
    int best = 0;
    double bestd = ax;                 /* distance to code 0 (value 0) */
    for (int c = 1; c <= 126; ++c) {
        double d = fabs(ax - orc_e4m3_value((uint8_t)c));
        if (d < bestd || (d == bestd && (c & 1) == 0)) { best = c; bestd = d; }
    }
    return (uint8_t)(best | (signbit(x) ? 0x80 : 0));
}

void orc_e4m3_encode(int64_t n, const float *x, uint8_t *codes)
{
    for (int64_t t = 0; t < n; ++t) codes[t] = orc_e4m3_encode1(x[t]);
}

/* Per-row scales of A (MxK): s[i] = max_k |A[i,k]| / 448 in binary32
 * (correctly rounded division); an all-zero row gets scale 1. */
void orc_fp8_scales_rows(int64_t M, int64_t K, const float *A, int64_t lda, float *s)
{
    for (int64_t i = 0; i < M; ++i) {
        float amax = 0.0f;
        for (int64_t k = 0; k < K; ++k) {
            float v = fabsf(A[i * lda + k]);
            if (v > amax) amax = v;
        }
        s[i] = (amax == 0.0f) ? 1.0f : amax / 448.0f;
    }
}

/* Per-column scales of B (KxN): s[j] = max_k |B[k,j]| / 448, zero column -> 1. */
void orc_fp8_scales_cols(int64_t K, int64_t N, const float *B, int64_t ldb, float *s)
{
    for (int64_t j = 0; j < N; ++j) {
        float amax = 0.0f;
        for (int64_t k = 0; k < K; ++k) {
            float v = fabsf(B[k * ldb + j]);
            if (v > amax) amax = v;
        }
        s[j] = (amax == 0.0f) ? 1.0f : amax / 448.0f;
    }
}

/* q[i,k] = e4m3(A[i,k] / s[i]), the division in binary32 (correctly rounded);
 * q is MxK dense. */
void orc_fp8_quantize_rows(int64_t M, int64_t K, const float *A, int64_t lda,
                           const float *s, uint8_t *q)
{
#pragma omp parallel for
    for (int64_t i = 0; i < M; ++i)
        for (int64_t k = 0; k < K; ++k)
            q[i * K + k] = orc_e4m3_encode1(A[i * lda + k] / s[i]);
}

/* q[k,j] = e4m3(B[k,j] / s[j]); q is KxN dense. */
void orc_fp8_quantize_cols(int64_t K, int64_t N, const float *B, int64_t ldb,
                           const float *s, uint8_t *q)
{
#pragma omp parallel for
    for (int64_t k = 0; k < K; ++k)
        for (int64_t j = 0; j < N; ++j)
            q[k * N + j] = orc_e4m3_encode1(B[k * ldb + j] / s[j]);
}

/* Dequantised-input product in binary64:
 *   Cref[i,j] = alpha * sa[i]*sb[j] * sum_k val(qa[i,k])*val(qb[k,j])
 *               + (beta == 0 ? 0 : beta*C0[i,j]).
 * qa is MxK dense, qb is KxN dense.  This is what a scaled FP8 kernel computes
 * exactly up to its binary32 accumulation and epilogue rounding. */
void orc_gemm_fp8_dequant(int64_t M, int64_t N, int64_t K, double alpha,
                          const uint8_t *qa, const float *sa,
                          const uint8_t *qb, const float *sb,
                          double beta, const float *C0, int64_t ldc0,
                          double *Cref, int nthreads)
{
    double lut[256];
    for (int c = 0; c < 256; ++c) lut[c] = orc_e4m3_value((uint8_t)c);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < M; ++i) {
        double *row = Cref + i * N;
        for (int64_t j = 0; j < N; ++j) row[j] = 0.0;
        for (int64_t k = 0; k < K; ++k) {
            double a = lut[qa[i * K + k]];
            for (int64_t j = 0; j < N; ++j) row[j] += a * lut[qb[k * N + j]];
        }
        for (int64_t j = 0; j < N; ++j) {
            double v = alpha * (double)sa[i] * (double)sb[j] * row[j];
            if (beta != 0.0) v += beta * (double)C0[i * ldc0 + j];
            row[j] = v;
        }
    }
}

/* ------------------------------------------------------------- norms --- */

/* out[0] = ||C - Cref||_F / ||Cref||_F (or ||C - Cref||_F if Cref == 0)
 * out[1] = sum (C - Cref)^2,  out[2] = sum Cref^2
 * out[3] = max_ij |C - Cref| / den[i,j] when den != NULL (0/0 -> 0, x/0 -> inf),
 *          otherwise max_ij |C - Cref|.
 * C is MxN with row stride ldc (binary32); Cref and den are MxN dense. */
void orc_norms(int64_t M, int64_t N, const float *C, int64_t ldc,
               const double *Cref, const double *den, double *out)
{
    double num = 0.0, ref = 0.0, mx = 0.0;
    for (int64_t i = 0; i < M; ++i)
        for (int64_t j = 0; j < N; ++j) {
            double r = Cref[i * N + j];
            double d = (double)C[i * ldc + j] - r;
            num += d * d;
            ref += r * r;
            double q = fabs(d);
            if (den) {
                double dd = den[i * N + j];
                if (dd == 0.0) q = (d == 0.0) ? 0.0 : INFINITY;
                else q = q / dd;
            }
            if (q > mx || isnan(q)) mx = q;
        }
    out[0] = (ref > 0.0) ? sqrt(num / ref) : sqrt(num);
    out[1] = num;
    out[2] = ref;
    out[3] = mx;
}

/* ------------------------------------------------------------ FP64 GEMM --- */

/* Error-free transformations in binary64 (no fast-math, no contraction):
 * two_sum: a + b = s + e exactly (Knuth); two_prod: a * b = p + e exactly,
 * the error term from one fused multiply-add. */
static void two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    double z = x - a;
    *e = (a - (x - z)) + (b - z);
    *s = x;
}

static void two_prod(double a, double b, double *p, double *e)
{
    double x = a * b;
    *e = fma(a, b, -x);
    *p = x;
}

/* Cref = alpha * A*B + beta*C0 for binary64 operands (the same map-reduce MM,
 * Sec. 3.3, with the scalars of Sec. 2.1).  Because the result under test is
 * itself binary64, the reference is evaluated in double-double: each sum over
 * k is the compensated dot product "Dot2" of Ogita, Rump and Oishi (Accurate
 * Sum and Dot Product, SIAM J. Sci. Comput. 26(6), 2005) -- every product split
 * exactly into p + e, p added error-free into the running high part, all
 * error terms collected in a low part -- and alpha*s + beta*c is formed from
 * exact products and sums before one final rounding.  Natural k order.
 * A is MxK (row stride lda), B is KxN (ldb), C0 is MxN (ldc0; unread when
 * beta == 0); Cref is MxN dense.  absolute != 0 computes the Higham
 * denominator |alpha||A||B| + |beta||C0| (plain binary64 sums) instead. */
void orc_dgemm(int64_t M, int64_t N, int64_t K, double alpha,
               const double *A, int64_t lda, const double *B, int64_t ldb,
               double beta, const double *C0, int64_t ldc0, double *Cref,
               int absolute, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        double *lo = (double *)calloc((size_t)(N > 0 ? N : 1), sizeof(double));
#pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < M; ++i) {
            double *hi = Cref + i * N;
            for (int64_t j = 0; j < N; ++j) { hi[j] = 0.0; lo[j] = 0.0; }
            for (int64_t k = 0; k < K; ++k) {
                const double a = A[i * lda + k];
                const double *brow = B + k * ldb;
                if (absolute) {
                    for (int64_t j = 0; j < N; ++j) hi[j] += fabs(a) * fabs(brow[j]);
                    continue;
                }
                for (int64_t j = 0; j < N; ++j) {
                    double p, pe, se;
                    two_prod(a, brow[j], &p, &pe);
                    two_sum(hi[j], p, &hi[j], &se);
                    lo[j] += pe + se;
                }
            }
            for (int64_t j = 0; j < N; ++j) {
                if (absolute) {
                    double v = fabs(alpha) * hi[j];
                    if (beta != 0.0) v += fabs(beta) * fabs(C0[i * ldc0 + j]);
                    hi[j] = v;
                    continue;
                }
                /* alpha * (hi + lo) as p1 + t */
                double p1, e1;
                two_prod(alpha, hi[j], &p1, &e1);
                double t = e1 + alpha * lo[j];
                if (beta != 0.0) {
                    double p2, e2, s, e3;
                    two_prod(beta, C0[i * ldc0 + j], &p2, &e2);
                    two_sum(p1, p2, &s, &e3);
                    hi[j] = s + (t + (e2 + e3));
                } else {
                    hi[j] = p1 + t;
                }
            }
        }
        free(lo);
    }
}
