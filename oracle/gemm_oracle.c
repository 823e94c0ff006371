/*
 * gemm_oracle.c -- plain CPU reference for batched small-matrix GEMM.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: it is used by tests/, by __graft_entry__.smoke() and by the
 * cpu_baseline leg of bench.py, and by nothing else.  It shares no source,
 * header, table or helper with the HIP library.
 *
 * What it computes (Jhurani & Mullowney, "A GEMM interface and implementation
 * on NVIDIA GPUs for multiple small matrices", Sec. 2, Eq. (1)):
 *
 *     C^p <- alpha * op(A^p) * op(B^p) + beta * C^p,     p = 0 .. batch-1,
 *
 * with C^p m x n, op(A^p) m x k, op(B^p) k x n, every matrix column-major with
 * its own leading dimension; element (i, j) of the p-th matrix of a batch sits
 * at  base[off[p] + i + ld * j]  (Sec. 5, the "second leading dimension" rule,
 * generalised to an explicit per-matrix element offset so that one routine
 * serves the strided form, the pointer-array form and the variable-size form).
 *
 * op() per Sec. 2 (and the conjugation functor of Sec. 6):
 *     'N' : op(X)(r, c) = X[r + ld*c]
 *     'T' : op(X)(r, c) = X[c + ld*r]
 *     'C' : op(X)(r, c) = conj(X[c + ld*r])         (== 'T' for real data)
 *     'R' : op(X)(r, c) = conj(X[r + ld*c])         (conjugate, no transpose;
 *           not in the paper -- needed to express gradients of complex
 *           products as one more call of the same routine)
 *
 * The a1b0 / general "axpby" functors of Sec. 6 fix two special cases that are
 * part of the definition here: when alpha == 0 the operands A and B are never
 * read; when beta == 0 the input C is never read (the functor y = x does not
 * look at y).
 *
 * Arithmetic: every element is promoted exactly to the accumulator type; the
 * inner sum runs over l = 0 .. k-1 in ascending order; products and sums are
 * separate roundings (compile with -ffp-contract=off).  Two accumulators:
 *     ext = 0 : IEEE binary64 ("FP64 accumulation");
 *     ext = 1 : x87 80-bit long double (64-bit significand), used as the
 *               reference for the binary64 (D/Z) GPU results, whose own
 *               rounding error is comparable to that of an FP64 oracle.
 * The result is returned unrounded to the working precision as a pair of
 * binary64 numbers hi + lo (lo may be NULL; with ext = 0 lo is 0).
 *
 * The companion routine oracle_gemm_bound() returns the denominator of the
 * acceptance test,  |alpha| * (|op(A)| |op(B)|)_ij + |beta| * |C_ij|,
 * with |.| the modulus taken elementwise.
 *
 * Storage type codes: 0 f32, 1 f64, 2 c64, 3 c128, 4 bf16, 5 f16,
 * 6 fp8 e4m3 (OCP "fn" variant: bias 7, no infinities, max 448).
 * Complex values are (re, im) pairs.  Optional per-matrix scales multiply every
 * decoded element of A^p (scaleA[p]) or B^p (scaleB[p]) exactly.
 *
 * Two further routines serve the precision modes:
 *   oracle_quant_e4m3   per-matrix absmax scaling s = max|X|/448 (1 when X = 0)
 *                       and rounding of X/s (binary32 division) to the nearest
 *                       OCP E4M3 value, ties to even, saturating to +-448;
 *   oracle_gemm_split3  the BF16x3 product: every binary32 operand x is split
 *                       into hi = bf16(x), lo = bf16(x - hi) (round to nearest
 *                       even) and sum_l hi_a hi_b + hi_a lo_b + lo_a hi_b is
 *                       accumulated exactly as in oracle_gemm.
 *
 * Parity status: pinned by tests/test_oracle_*.py (library cross-checks,
 * identities, closed forms, exact rational brute force, torch's float8 and
 * bfloat16 conversions).
 */
#include <stdint.h>
#include <stddef.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { T_F32 = 0, T_F64 = 1, T_C64 = 2, T_C128 = 3, T_BF16 = 4, T_F16 = 5, T_E4M3 = 6 };

static int is_complex(int t) { return t == T_C64 || t == T_C128; }

/* ---- exact decoders of the narrow storage formats ------------------------ */

/* bfloat16: the upper half of an IEEE binary32 word. */
static double dec_bf16(uint16_t h)
{
    uint32_t w = ((uint32_t)h) << 16;
    float f;
    memcpy(&f, &w, 4);
    return (double)f;
}

/* IEEE 754 binary16: 1 sign, 5 exponent (bias 15), 10 fraction bits. */
static double dec_f16(uint16_t h)
{
    int s = (h >> 15) & 1, e = (h >> 10) & 0x1f, f = h & 0x3ff;
    double v;
    if (e == 0)
        v = ldexp((double)f, -24);                 /* subnormal: f * 2^-14 * 2^-10 */
    else if (e == 31)
        v = f ? NAN : INFINITY;
    else
        v = ldexp((double)(1024 + f), e - 25);     /* (1 + f/2^10) * 2^(e-15) */
    return s ? -v : v;
}

/* OCP 8-bit floating point, E4M3 "fn": 1 sign, 4 exponent (bias 7), 3 fraction
 * bits; exponent field 15 with fraction 7 is NaN, there is no infinity. */
static double dec_e4m3(uint8_t b)
{
    int s = (b >> 7) & 1, e = (b >> 3) & 0xf, f = b & 7;
    double v;
    if (e == 15 && f == 7)
        v = NAN;
    else if (e == 0)
        v = ldexp((double)f, -9);                  /* f/8 * 2^-6 */
    else
        v = ldexp((double)(8 + f), e - 10);        /* (1 + f/8) * 2^(e-7) */
    return s ? -v : v;
}

/* Element idx (in elements of the storage type) promoted exactly to double. */
static void get(int t, const void* base, int64_t idx, double* re, double* im)
{
    switch (t) {
    case T_F32:  *re = ((const float*)base)[idx];              *im = 0; break;
    case T_F64:  *re = ((const double*)base)[idx];             *im = 0; break;
    case T_C64:  *re = ((const float*)base)[2 * idx];
                 *im = ((const float*)base)[2 * idx + 1];          break;
    case T_C128: *re = ((const double*)base)[2 * idx];
                 *im = ((const double*)base)[2 * idx + 1];         break;
    case T_BF16: *re = dec_bf16(((const uint16_t*)base)[idx]);  *im = 0; break;
    case T_F16:  *re = dec_f16(((const uint16_t*)base)[idx]);   *im = 0; break;
    case T_E4M3: *re = dec_e4m3(((const uint8_t*)base)[idx]);   *im = 0; break;
    default:     *re = NAN; *im = NAN;
    }
}

/* op(X)(r, c) of one matrix whose (0,0) element is at index off. */
static void op_elem(int t, char op, const void* X, int64_t off, int ld,
                    int r, int c, double* re, double* im)
{
    int64_t idx;
    int conj = 0;
    switch (op) {
    case 'N': case 'n': idx = off + r + (int64_t)ld * c;               break;
    case 'T': case 't': idx = off + c + (int64_t)ld * r;               break;
    case 'C': case 'c': idx = off + c + (int64_t)ld * r;   conj = 1;   break;
    case 'R': case 'r': idx = off + r + (int64_t)ld * c;   conj = 1;   break;
    default: *re = NAN; *im = NAN; return;
    }
    get(t, X, idx, re, im);
    if (conj && *im != 0)
        *im = -*im;
}

static int op_ok(char op)
{
    return op == 'N' || op == 'n' || op == 'T' || op == 't' ||
           op == 'C' || op == 'c' || op == 'R' || op == 'r';
}

/* One accumulator type per generated function: ACC is double or long double. */
#define DEFINE_ORACLE(NAME, ACC)                                                  \
static void NAME(int tA, int tB, int tC, char ta, char tb, int64_t p,             \
                 int m, int n, int k, const double* alpha, const double* beta,   \
                 const void* A, int64_t oA, int lda, double sA,                   \
                 const void* B, int64_t oB, int ldb, double sB,                   \
                 const void* C, int64_t oC, int ldc,                              \
                 double* hi, double* lo, int64_t oO)                              \
{                                                                                 \
    const int cplx = is_complex(tC);                                              \
    const int a_zero = alpha[0] == 0.0 && alpha[1] == 0.0;                        \
    const int b_zero = beta[0] == 0.0 && beta[1] == 0.0;                          \
    const ACC ar = alpha[0], ai = alpha[1], br = beta[0], bi = beta[1];           \
    (void)p;                                                                      \
    for (int j = 0; j < n; ++j)                                                   \
        for (int i = 0; i < m; ++i) {                                             \
            ACC sr = 0, si = 0;                       /* sum_l opA(i,l) opB(l,j) */\
            if (!a_zero)                                                          \
                for (int l = 0; l < k; ++l) {                                     \
                    double xr, xi, yr, yi;                                        \
                    op_elem(tA, ta, A, oA, lda, i, l, &xr, &xi);                   \
                    op_elem(tB, tb, B, oB, ldb, l, j, &yr, &yi);                   \
                    ACC Xr = (ACC)xr * (ACC)sA, Xi = (ACC)xi * (ACC)sA;           \
                    ACC Yr = (ACC)yr * (ACC)sB, Yi = (ACC)yi * (ACC)sB;           \
                    ACC pr = Xr * Yr;                                             \
                    ACC pi = Xr * Yi;                                             \
                    if (cplx) {                                                   \
                        ACC t1 = Xi * Yi;                                         \
                        ACC t2 = Xi * Yr;                                         \
                        pr = pr - t1;                                             \
                        pi = pi + t2;                                             \
                    }                                                             \
                    sr = sr + pr;                                                 \
                    if (cplx) si = si + pi;                                       \
                }                                                                 \
            ACC cr = 0, ci = 0;                                                   \
            if (!b_zero) {                                                        \
                double zr, zi;                                                    \
                get(tC, C, oC + i + (int64_t)ldc * j, &zr, &zi);                  \
                cr = zr; ci = zi;                                                 \
            }                                                                     \
            ACC rr, ri;                                                           \
            if (cplx) {                                                           \
                ACC ur = 0, ui = 0, vr = 0, vi = 0;                               \
                if (!a_zero) { ur = ar * sr - ai * si; ui = ar * si + ai * sr; }  \
                if (!b_zero) { vr = br * cr - bi * ci; vi = br * ci + bi * cr; }  \
                rr = ur + vr; ri = ui + vi;                                       \
            } else {                                                              \
                ACC u = 0, v = 0;                                                 \
                if (!a_zero) u = ar * sr;                                         \
                if (!b_zero) v = br * cr;                                         \
                rr = a_zero ? v : (b_zero ? u : u + v);                           \
                ri = 0;                                                           \
            }                                                                     \
            int64_t o = oO + (cplx ? 2 : 1) * ((int64_t)i + (int64_t)m * j);      \
            double h = (double)rr;                                                \
            hi[o] = h;                                                            \
            if (lo) lo[o] = (double)(rr - (ACC)h);                                \
            if (cplx) {                                                           \
                double hh = (double)ri;                                           \
                hi[o + 1] = hh;                                                   \
                if (lo) lo[o + 1] = (double)(ri - (ACC)hh);                       \
            }                                                                     \
        }                                                                         \
}

DEFINE_ORACLE(oracle_one_f64, double)
DEFINE_ORACLE(oracle_one_ext, long double)

void oracle_set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Batched reference.  All per-matrix arrays have `batch` entries.
 *   m, n, k, lda, ldb, ldc : sizes and leading dimensions (elements);
 *   offA, offB, offC       : element offset of matrix p's (0,0) entry;
 *   scaleA, scaleB         : per-matrix multipliers of the decoded operands, or NULL (1);
 *   alpha, beta            : (re, im) of the scalars;
 *   C may be NULL when beta == 0;  A, B may be NULL when alpha == 0;
 *   offO                   : offset (in doubles) of matrix p's m*n result block in
 *                            hi/lo, entries column-major, complex as (re, im);
 *   ext                    : 0 = binary64 accumulation, 1 = long double.
 * Returns 0, or -1 on an invalid op character / type code.
 */
int oracle_gemm(int tA, int tB, int tC, char transa, char transb, int64_t batch,
                const int32_t* m, const int32_t* n, const int32_t* k,
                const double* alpha, const double* beta,
                const void* A, const int64_t* offA, const int32_t* lda, const double* scaleA,
                const void* B, const int64_t* offB, const int32_t* ldb, const double* scaleB,
                const void* C, const int64_t* offC, const int32_t* ldc,
                const int64_t* offO, double* hi, double* lo, int ext)
{
    if (!op_ok(transa) || !op_ok(transb) || tA < 0 || tA > 6 || tB < 0 || tB > 6 ||
        tC < 0 || tC > 3)
        return -1;
    if (lo && !ext)
        for (int64_t p = 0; p < batch; ++p) {
            int64_t cnt = (is_complex(tC) ? 2 : 1) * (int64_t)m[p] * n[p];
            for (int64_t e = 0; e < cnt; ++e) lo[offO[p] + e] = 0.0;
        }
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t p = 0; p < batch; ++p) {
        double sA = scaleA ? scaleA[p] : 1.0, sB = scaleB ? scaleB[p] : 1.0;
        if (ext)
            oracle_one_ext(tA, tB, tC, transa, transb, p, m[p], n[p], k[p], alpha, beta,
                           A, offA ? offA[p] : 0, lda[p], sA, B, offB ? offB[p] : 0, ldb[p], sB,
                           C, offC ? offC[p] : 0, ldc[p], hi, ext ? lo : NULL, offO[p]);
        else
            oracle_one_f64(tA, tB, tC, transa, transb, p, m[p], n[p], k[p], alpha, beta,
                           A, offA ? offA[p] : 0, lda[p], sA, B, offB ? offB[p] : 0, ldb[p], sB,
                           C, offC ? offC[p] : 0, ldc[p], hi, NULL, offO[p]);
    }
    return 0;
}

/*
 * Denominator of the acceptance test for every output entry:
 *   |alpha| * sum_l |op(A)(i,l)| * |op(B)(l,j)|  +  |beta| * |C_in(i,j)|
 * (the first term is absent when alpha == 0, the second when beta == 0).
 * Same argument conventions as oracle_gemm; out holds one double per entry,
 * at offO[p] + i + m*j (real-valued also for complex data, so offO counts
 * entries, not doubles).
 */
int oracle_gemm_bound(int tA, int tB, int tC, char transa, char transb, int64_t batch,
                      const int32_t* m, const int32_t* n, const int32_t* k,
                      const double* alpha, const double* beta,
                      const void* A, const int64_t* offA, const int32_t* lda, const double* scaleA,
                      const void* B, const int64_t* offB, const int32_t* ldb, const double* scaleB,
                      const void* C, const int64_t* offC, const int32_t* ldc,
                      const int64_t* offO, double* out)
{
    if (!op_ok(transa) || !op_ok(transb)) return -1;
    const int a_zero = alpha[0] == 0.0 && alpha[1] == 0.0;
    const int b_zero = beta[0] == 0.0 && beta[1] == 0.0;
    const long double amod = hypotl(alpha[0], alpha[1]);
    const long double bmod = hypotl(beta[0], beta[1]);
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t p = 0; p < batch; ++p) {
        long double sA = scaleA ? fabsl(scaleA[p]) : 1.0L;
        long double sB = scaleB ? fabsl(scaleB[p]) : 1.0L;
        for (int j = 0; j < n[p]; ++j)
            for (int i = 0; i < m[p]; ++i) {
                long double s = 0;
                if (!a_zero)
                    for (int l = 0; l < k[p]; ++l) {
                        double xr, xi, yr, yi;
                        op_elem(tA, transa, A, offA ? offA[p] : 0, lda[p], i, l, &xr, &xi);
                        op_elem(tB, transb, B, offB ? offB[p] : 0, ldb[p], l, j, &yr, &yi);
                        s += hypotl(xr, xi) * sA * hypotl(yr, yi) * sB;
                    }
                long double c = 0;
                if (!b_zero) {
                    double zr, zi;
                    get(tC, C, (offC ? offC[p] : 0) + i + (int64_t)ldc[p] * j, &zr, &zi);
                    c = hypotl(zr, zi);
                }
                out[offO[p] + i + (int64_t)m[p] * j] =
                    (double)((a_zero ? 0.0L : amod * s) + (b_zero ? 0.0L : bmod * c));
            }
    }
    return 0;
}

/* ---- precision-mode helpers ------------------------------------------------ */

/* Nearest bfloat16 value (8 significant bits, binary32 exponent range with
 * subnormal spacing 2^-133), ties to even; exact in double. */
static double round_bf16(double x)
{
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    frexp(x, &e);                       /* x = f 2^e, 0.5 <= |f| < 1 */
    int q = e - 8;                      /* spacing 2^q of 8-bit significands */
    if (q < -133) q = -133;
    return ldexp(nearbyint(ldexp(x, -q)), q);
}

/* Nearest OCP E4M3 code of a binary32 value: 3 fraction bits, exponents
 * -6..8, subnormal spacing 2^-9, ties to even, saturation to 448 (0x7E). */
static uint8_t encode_e4m3(float v)
{
    uint8_t sign = signbit(v) ? 0x80 : 0x00;
    double a = fabs((double)v);
    if (isnan(v)) return (uint8_t)(sign | 0x7F);
    if (a >= 464.0) return (uint8_t)(sign | 0x7E);
    if (a < ldexp(1.0, -6)) {
        double m = nearbyint(a * 512.0);            /* units of 2^-9 */
        return (uint8_t)(sign | (uint8_t)m);        /* m == 8 is the code of 2^-6 */
    }
    int e;
    frexp(a, &e);
    e -= 1;                                         /* a = 1.f * 2^e */
    double m = nearbyint((ldexp(a, -e) - 1.0) * 8.0);
    if (m == 8.0) { m = 0.0; e += 1; }
    return (uint8_t)(sign | (uint8_t)((e + 7) << 3) | (uint8_t)m);
}

/*
 * Per-matrix absmax quantisation.  Matrix p: rows[p] x cols[p] binary32 values
 * at X[offX[p] + i + ldx[p] j]; writes codes column-major (leading dimension
 * rows[p]) at Q[offQ[p] ...] and the scale to scales[p].
 */
void oracle_quant_e4m3(int64_t batch, const int32_t* rows, const int32_t* cols, const float* X,
                       const int64_t* offX, const int32_t* ldx, uint8_t* Q, const int64_t* offQ,
                       float* scales)
{
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t p = 0; p < batch; ++p) {
        float amax = 0.0f;
        for (int j = 0; j < cols[p]; ++j)
            for (int i = 0; i < rows[p]; ++i) {
                float a = fabsf(X[offX[p] + i + (int64_t)ldx[p] * j]);
                if (a > amax) amax = a;
            }
        float s = amax > 0.0f ? amax / 448.0f : 1.0f;
        scales[p] = s;
        for (int j = 0; j < cols[p]; ++j)
            for (int i = 0; i < rows[p]; ++i) {
                float x = X[offX[p] + i + (int64_t)ldx[p] * j];
                Q[offQ[p] + i + (int64_t)rows[p] * j] = encode_e4m3(x / s);
            }
    }
}

/* op(X)(r, c) of a binary32 matrix split into bf16 hi and lo parts. */
static void op_split(char op, const float* X, int64_t off, int ld, int r, int c, double* hi, double* lo)
{
    int64_t idx = (op == 'N' || op == 'n' || op == 'R' || op == 'r') ? off + r + (int64_t)ld * c
                                                                     : off + c + (int64_t)ld * r;
    double x = X[idx];
    *hi = round_bf16(x);
    *lo = round_bf16(x - *hi);      /* x - hi is exact in double */
}

/*
 * BF16x3 reference (real binary32 inputs and C): per entry
 *   acc = sum_l hi_a hi_b + hi_a lo_b + lo_a hi_b   (long double, l ascending)
 *   out = alpha acc + beta C_in   (alpha == 0: A, B unread; beta == 0: C unread)
 * returned as hi + lo doubles; bound[] (may be NULL) receives
 *   |alpha| sum_l (|hi_a hi_b| + |hi_a lo_b| + |lo_a hi_b|) + |beta| |C_in|.
 * Same conventions as oracle_gemm (real types only: alpha, beta are doubles).
 */
int oracle_gemm_split3(char transa, char transb, int64_t batch, const int32_t* m, const int32_t* n,
                       const int32_t* k, double alpha, double beta, const float* A, const int64_t* offA,
                       const int32_t* lda, const float* B, const int64_t* offB, const int32_t* ldb,
                       const float* C, const int64_t* offC, const int32_t* ldc, const int64_t* offO,
                       double* hi, double* lo, double* bound)
{
    if (!op_ok(transa) || !op_ok(transb)) return -1;
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t p = 0; p < batch; ++p)
        for (int j = 0; j < n[p]; ++j)
            for (int i = 0; i < m[p]; ++i) {
                long double s = 0, sb = 0;
                if (alpha != 0.0)
                    for (int l = 0; l < k[p]; ++l) {
                        double ah, al, bh, bl;
                        op_split(transa, A, offA[p], lda[p], i, l, &ah, &al);
                        op_split(transb, B, offB[p], ldb[p], l, j, &bh, &bl);
                        long double t1 = (long double)ah * bh;
                        long double t2 = (long double)ah * bl;
                        long double t3 = (long double)al * bh;
                        s = s + t1;
                        s = s + t2;
                        s = s + t3;
                        sb += fabsl(t1) + fabsl(t2) + fabsl(t3);
                    }
                long double c = 0;
                if (beta != 0.0) c = C[offC[p] + i + (int64_t)ldc[p] * j];
                long double r;
                if (alpha == 0.0) r = beta == 0.0 ? 0.0L : (long double)beta * c;
                else if (beta == 0.0) r = (long double)alpha * s;
                else r = (long double)alpha * s + (long double)beta * c;
                int64_t o = offO[p] + i + (int64_t)m[p] * j;
                double h = (double)r;
                hi[o] = h;
                lo[o] = (double)(r - (long double)h);
                if (bound)
                    bound[o] = (double)(fabsl((long double)alpha) * sb + fabsl((long double)beta) * fabsl(c));
            }
    return 0;
}

/* Exposed for the pins: the encoder and the bf16 rounding on single values. */
uint8_t oracle_encode_e4m3(float v) { return encode_e4m3(v); }
double oracle_round_bf16(double x) { return round_bf16(x); }
double oracle_decode_e4m3(uint8_t b) { return dec_e4m3(b); }
double oracle_decode_f16(uint16_t h) { return dec_f16(h); }
double oracle_decode_bf16(uint16_t h) { return dec_bf16(h); }
