/*
 * sbg.h -- batched GEMM over many small matrices on AMD Instinct MI355X (gfx950).
 *
 * The operation (Jhurani & Mullowney, "A GEMM interface and implementation on
 * NVIDIA GPUs for multiple small matrices", Sec. 2, Eq. (1)):
 *
 *     C_p <- alpha * op(A_p) * op(B_p) + beta * C_p,      p = 0 .. batch_count-1,
 *
 * with C_p m x n, op(A_p) m x k, op(B_p) k x n.  The paper's kernels cover
 * 0 <= m, n, k <= 16; the plain S/D/C/Z forms here also take larger sizes
 * (cut into 16 x 16 output blocks and 16-wide k-chunks: the extension the
 * paper says its method allows, Sec. 1, by sub-block products, Sec. 7), while
 * the mixed-precision and variable-size forms keep the limit of 16.
 * op(X) is selected per operand by a character (Sec. 2; Sec. 5 argument list):
 *     'N'/'n'  X            'T'/'t'  X^T            'C'/'c'  X^H (conjugate transpose)
 *     'R'/'r'  conj(X), no transpose -- an extension not in the paper, used to
 *              express gradients of complex products as one more call.
 * For real types 'C' equals 'T' and 'R' equals 'N'.
 *
 * Storage: every matrix is column-major; leading dimensions and strides are in
 * ELEMENTS, never bytes (Sec. 5).  Element (i, j) of the p-th matrix of a
 * strided batch is X[i + ld * j + stride * p] (the paper's second leading
 * dimension, here 64-bit).
 *
 * Scalar types (suffix letter as in BLAS): s = float, d = double,
 * c = sbg_cfloat, z = sbg_cdouble (interleaved real, imaginary parts).
 *
 * Ownership and execution: all matrix, pointer-array and dimension memory is
 * DEVICE memory owned by the caller.  Calls are asynchronous on `stream` (a
 * hipStream_t; NULL = the legacy default stream) and never allocate, copy to
 * the host or synchronise.  alpha and beta are read at call time from HOST
 * memory (default) or, after sbg_set_scalar_mode(SBG_SCALAR_DEVICE), at kernel
 * time from DEVICE memory.  Invalid device pointers are undefined behaviour, as
 * in BLAS.  Calls on one stream are ordered; calls writing overlapping C on
 * different streams race.
 *
 * Errors: SBG_INVALID_VALUE with the 1-based position of the first rejected
 * argument recorded for sbg_last_invalid_arg() (checked in argument order, as
 * BLAS's xerbla does); SBG_NOT_SUPPORTED for m, n or k above 16 in the
 * mixed-precision, variable-size and quantiser entry points;
 * SBG_HIP_ERROR when the kernel launch fails.  Nothing is launched unless the
 * result is SBG_OK.
 *
 * Quick returns (no launch, SBG_OK): m == 0, n == 0, batch_count == 0, or
 * (alpha == 0 or k == 0) and beta == 1 (host scalar mode only).
 * Special cases of the definition (Sec. 6, the a1b0 and axpby functors):
 * when alpha == 0 neither A nor B is read; when beta == 0 C is not read, so
 * NaN or Inf there never reaches the result.
 */
#ifndef SBG_H
#define SBG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SBG_OK = 0,
    SBG_INVALID_VALUE = 1,
    SBG_NOT_SUPPORTED = 2,
    SBG_HIP_ERROR = 3,
    SBG_WORKSPACE_TOO_SMALL = 4
} sbg_status_t;

typedef enum { SBG_SCALAR_HOST = 0, SBG_SCALAR_DEVICE = 1 } sbg_scalar_mode_t;

typedef struct { float re, im; } sbg_cfloat;
typedef struct { double re, im; } sbg_cdouble;

/* Stored type of A and B in the mixed-precision (_ex) forms; C and the
 * accumulation are binary32. */
typedef enum {
    SBG_R_32F = 0,       /* binary32 */
    SBG_R_16BF = 1,      /* bfloat16 */
    SBG_R_16F = 2,       /* IEEE binary16 */
    SBG_R_8F_E4M3 = 3    /* OCP FP8 E4M3 ("fn": max 448, no infinities), per-matrix scales */
} sbg_datatype_t;

/* SBG_MODE_BF16X3: binary32 A and B are split into bfloat16 hi + lo on the fly
 * and hi*hi + hi*lo + lo*hi is accumulated in binary32 (the lo*lo term is
 * dropped; accuracy is about 2^-16 relative, not binary32). */
typedef enum { SBG_MODE_PLAIN = 0, SBG_MODE_BF16X3 = 1 } sbg_compute_mode_t;

/* ---- strided form: the paper's TGEMM_multi_uniform (Sec. 5) --------------
 * Arguments, in order (positions used by sbg_last_invalid_arg):
 *   1 transa, 2 transb   op characters (see above)
 *   3 m, 4 n, 5 k        sizes, >= 0 (above 16: the sub-blocked kernel)
 *   6 alpha              pointer to the scalar (host or device, see mode)
 *   7 A                  device pointer to the (0,0) element of A_0
 *   8 lda                >= max(1, m) for op N/R, >= max(1, k) for T/C
 *   9 strideA            elements between A_p and A_{p+1}; >= 0 (0 = one A
 *                        shared by the whole batch)
 *  10 B, 11 ldb (>= max(1, k) for N/R, >= max(1, n) for T/C), 12 strideB (>= 0)
 *  13 beta
 *  14 C, 15 ldc (>= max(1, m)), 16 strideC (>= ldc * n when batch_count > 1:
 *     output matrices may not overlap, cf. the layout figure of Sec. 5)
 *  17 batch_count (>= 0)
 *  18 stream
 */
sbg_status_t sbg_sgemm_strided_batched(char transa, char transb, int m, int n, int k,
    const float* alpha, const float* A, int lda, int64_t strideA,
    const float* B, int ldb, int64_t strideB, const float* beta,
    float* C, int ldc, int64_t strideC, int64_t batch_count, void* stream);
sbg_status_t sbg_dgemm_strided_batched(char transa, char transb, int m, int n, int k,
    const double* alpha, const double* A, int lda, int64_t strideA,
    const double* B, int ldb, int64_t strideB, const double* beta,
    double* C, int ldc, int64_t strideC, int64_t batch_count, void* stream);
sbg_status_t sbg_cgemm_strided_batched(char transa, char transb, int m, int n, int k,
    const sbg_cfloat* alpha, const sbg_cfloat* A, int lda, int64_t strideA,
    const sbg_cfloat* B, int ldb, int64_t strideB, const sbg_cfloat* beta,
    sbg_cfloat* C, int ldc, int64_t strideC, int64_t batch_count, void* stream);
sbg_status_t sbg_zgemm_strided_batched(char transa, char transb, int m, int n, int k,
    const sbg_cdouble* alpha, const sbg_cdouble* A, int lda, int64_t strideA,
    const sbg_cdouble* B, int ldb, int64_t strideB, const sbg_cdouble* beta,
    sbg_cdouble* C, int ldc, int64_t strideC, int64_t batch_count, void* stream);

/* ---- pointer-array form: the paper's TGEMM_multi_nounif (Sec. 3-5) --------
 * Same semantics with per-matrix device pointers instead of strides: A_p is
 * Aarray[p] etc.  Aarray, Barray, Carray are device arrays of batch_count
 * device pointers.  Positions: 1 transa, 2 transb, 3 m, 4 n, 5 k, 6 alpha,
 * 7 Aarray, 8 lda, 9 Barray, 10 ldb, 11 beta, 12 Carray, 13 ldc,
 * 14 batch_count, 15 stream.  Distinct Carray entries must not overlap
 * (not checked: the pointers live on the device). */
sbg_status_t sbg_sgemm_batched(char transa, char transb, int m, int n, int k,
    const float* alpha, const float* const* Aarray, int lda,
    const float* const* Barray, int ldb, const float* beta,
    float* const* Carray, int ldc, int64_t batch_count, void* stream);
sbg_status_t sbg_dgemm_batched(char transa, char transb, int m, int n, int k,
    const double* alpha, const double* const* Aarray, int lda,
    const double* const* Barray, int ldb, const double* beta,
    double* const* Carray, int ldc, int64_t batch_count, void* stream);
sbg_status_t sbg_cgemm_batched(char transa, char transb, int m, int n, int k,
    const sbg_cfloat* alpha, const sbg_cfloat* const* Aarray, int lda,
    const sbg_cfloat* const* Barray, int ldb, const sbg_cfloat* beta,
    sbg_cfloat* const* Carray, int ldc, int64_t batch_count, void* stream);
sbg_status_t sbg_zgemm_batched(char transa, char transb, int m, int n, int k,
    const sbg_cdouble* alpha, const sbg_cdouble* const* Aarray, int lda,
    const sbg_cdouble* const* Barray, int ldb, const sbg_cdouble* beta,
    sbg_cdouble* const* Carray, int ldc, int64_t batch_count, void* stream);

/* ---- variable-size form (one call for a batch of unequal sizes) ------------
 * Matrix p has its own sizes d_m[p], d_n[p], d_k[p] and leading dimensions
 * d_lda[p], d_ldb[p], d_ldc[p] (device int arrays) and its own pointers, as in
 * the pointer-array form; ops, alpha and beta are shared.  This generalises the
 * paper's remark that unequal sizes can be partitioned into sets of equal size
 * (Sec. 1): the partition is done on the device (size classes by max(m, n, k))
 * and the whole batch runs as one persistent launch, so a call can be captured
 * in a HIP graph and replayed.
 *   max_m, max_n, max_k: host-side upper bounds of the sizes (<= 16; larger
 *     gives SBG_NOT_SUPPORTED).  A matrix whose sizes exceed them, are
 *     negative, or whose leading dimensions are too small is SKIPPED (its C is
 *     untouched) and counted in the int at word 3 of the workspace.
 *   workspace: caller-owned, 16-byte aligned device memory of at least
 *     sbg_vbatched_workspace_size(batch_count) bytes (64 + 144 per matrix);
 *     it is overwritten on every call, so concurrent calls need distinct
 *     workspaces.
 * Positions: 1 transa, 2 transb, 3 d_m, 4 d_n, 5 d_k, 6 max_m, 7 max_n,
 * 8 max_k, 9 alpha, 10 Aarray, 11 d_lda, 12 Barray, 13 d_ldb, 14 beta,
 * 15 Carray, 16 d_ldc, 17 batch_count (<= 2^31 - 1), 18 workspace,
 * 19 workspace_bytes (SBG_WORKSPACE_TOO_SMALL when short), 20 stream. */
size_t sbg_vbatched_workspace_size(int64_t batch_count);
sbg_status_t sbg_sgemm_vbatched(char transa, char transb, const int* d_m, const int* d_n, const int* d_k,
    int max_m, int max_n, int max_k, const float* alpha, const float* const* Aarray, const int* d_lda,
    const float* const* Barray, const int* d_ldb, const float* beta, float* const* Carray, const int* d_ldc,
    int64_t batch_count, void* workspace, size_t workspace_bytes, void* stream);
sbg_status_t sbg_dgemm_vbatched(char transa, char transb, const int* d_m, const int* d_n, const int* d_k,
    int max_m, int max_n, int max_k, const double* alpha, const double* const* Aarray, const int* d_lda,
    const double* const* Barray, const int* d_ldb, const double* beta, double* const* Carray, const int* d_ldc,
    int64_t batch_count, void* workspace, size_t workspace_bytes, void* stream);
sbg_status_t sbg_cgemm_vbatched(char transa, char transb, const int* d_m, const int* d_n, const int* d_k,
    int max_m, int max_n, int max_k, const sbg_cfloat* alpha, const sbg_cfloat* const* Aarray, const int* d_lda,
    const sbg_cfloat* const* Barray, const int* d_ldb, const sbg_cfloat* beta, sbg_cfloat* const* Carray,
    const int* d_ldc, int64_t batch_count, void* workspace, size_t workspace_bytes, void* stream);
sbg_status_t sbg_zgemm_vbatched(char transa, char transb, const int* d_m, const int* d_n, const int* d_k,
    int max_m, int max_n, int max_k, const sbg_cdouble* alpha, const sbg_cdouble* const* Aarray, const int* d_lda,
    const sbg_cdouble* const* Barray, const int* d_ldb, const sbg_cdouble* beta, sbg_cdouble* const* Carray,
    const int* d_ldc, int64_t batch_count, void* workspace, size_t workspace_bytes, void* stream);

/* ---- mixed precision (binary32 accumulation and C) --------------------------
 * A and B are stored as ab_type; with scaleA/scaleB (device float arrays of
 * batch_count entries, both or neither; required for SBG_R_8F_E4M3) the
 * operands are sA[p] * A_p and sB[p] * B_p, so
 *     C_p <- alpha * sA[p] * sB[p] * op(A_p) op(B_p) + beta * C_p.
 * Narrow inputs are decoded exactly to binary32; products of bf16, fp16 and
 * e4m3 values are exact in binary32.  mode SBG_MODE_BF16X3 needs ab_type
 * SBG_R_32F.  Positions of the strided form: 1 transa, 2 transb, 3 m, 4 n, 5 k,
 * 6 alpha, 7 A, 8 lda, 9 strideA, 10 scaleA, 11 B, 12 ldb, 13 strideB,
 * 14 scaleB, 15 beta, 16 C, 17 ldc, 18 strideC, 19 batch_count, 20 ab_type,
 * 21 mode; of the variable-size form: as sbg_sgemm_vbatched with scaleA at 12,
 * scaleB at 15 (B, d_ldb at 13, 14), beta 16, Carray 17, d_ldc 18,
 * batch_count 19, ab_type 20, mode 21, workspace 22, workspace_bytes 23.
 * Scales, type and mode are checked after the other arguments. */
sbg_status_t sbg_gemm_strided_batched_ex(char transa, char transb, int m, int n, int k, const float* alpha,
    const void* A, int lda, int64_t strideA, const float* scaleA,
    const void* B, int ldb, int64_t strideB, const float* scaleB,
    const float* beta, float* C, int ldc, int64_t strideC, int64_t batch_count,
    sbg_datatype_t ab_type, sbg_compute_mode_t mode, void* stream);
sbg_status_t sbg_gemm_vbatched_ex(char transa, char transb, const int* d_m, const int* d_n, const int* d_k,
    int max_m, int max_n, int max_k, const float* alpha, const void* const* Aarray, const int* d_lda,
    const float* scaleA, const void* const* Barray, const int* d_ldb, const float* scaleB, const float* beta,
    float* const* Carray, const int* d_ldc, int64_t batch_count, sbg_datatype_t ab_type,
    sbg_compute_mode_t mode, void* workspace, size_t workspace_bytes, void* stream);

/* ---- variable-size mixed precision without a workspace argument ------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, and harnesses that forbid allocation.  Same
 * arguments, semantics and positions 1-21 as sbg_gemm_vbatched_ex, with the
 * workspace taken from a scratch array the library keeps in device memory
 * (one copy per GPU, resident until the process ends), so the call performs
 * no allocation of any kind.
 *   batch_count above SBG_NOALLOC_MAX_BATCH gives SBG_WORKSPACE_TOO_SMALL.
 *   The scratch is shared by every call on a GPU and keeps the last call's
 *   contents (its counters are cleared by each call): calls that overlap on
 *   one GPU (other streams, other threads) race and must be serialised by
 *   the caller.  The rejected-matrix count is not returned (it lives in the
 *   shared scratch).  Position 22 is the stream. */
#define SBG_NOALLOC_MAX_BATCH 262144
sbg_status_t sbg_gemm_vbatched_ex_noalloc(char transa, char transb, const int* d_m, const int* d_n,
    const int* d_k, int max_m, int max_n, int max_k, const float* alpha, const void* const* Aarray,
    const int* d_lda, const float* scaleA, const void* const* Barray, const int* d_ldb, const float* scaleB,
    const float* beta, float* const* Carray, const int* d_ldc, int64_t batch_count, sbg_datatype_t ab_type,
    sbg_compute_mode_t mode, void* stream);

/* ---- per-matrix absmax quantisation to FP8 E4M3 -----------------------------
 * For each binary32 matrix X_p (rows x cols <= 16 x 16): s_p = max|X_p| / 448
 * (1 for an all-zero matrix), Q_p = e4m3(X_p / s_p) rounded to nearest even and
 * saturated to +-448; scales[p] = s_p.  The outputs feed the _ex forms with
 * ab_type SBG_R_8F_E4M3.  Strided positions: 1 rows, 2 cols, 3 X, 4 ldx,
 * 5 strideX, 6 Q, 7 ldq, 8 strideQ, 9 scales, 10 batch_count.  Variable-size
 * positions: 1 d_rows, 2 d_cols, 3 max_rows, 4 max_cols, 5 Xarray, 6 d_ldx,
 * 7 Qarray, 8 d_ldq, 9 scales, 10 batch_count; matrices with invalid sizes are
 * skipped (scale not written). */
sbg_status_t sbg_quantize_e4m3_strided_batched(int rows, int cols, const float* X, int ldx, int64_t strideX,
    unsigned char* Q, int ldq, int64_t strideQ, float* scales, int64_t batch_count, void* stream);
sbg_status_t sbg_quantize_e4m3_vbatched(const int* d_rows, const int* d_cols, int max_rows, int max_cols,
    const float* const* Xarray, const int* d_ldx, unsigned char* const* Qarray, const int* d_ldq, float* scales,
    int64_t batch_count, void* stream);

/* ---- other BLAS routines in the same strided interface ----------------------
 * The paper proposes its second-leading-dimension interface for other BLAS
 * routines, formulated in terms of batched GEMM (Sec. 9).  Both routines
 * below follow reference-BLAS semantics per matrix, on column-major storage
 * with 64-bit strides between consecutive matrices / vectors of the batch.
 *
 * GEMV: y_p <- alpha op(A_p) x_p + beta y_p, A_p m x n, op in N, T, C (R is
 * rejected); x_p has n entries for N (m for T, C), y_p the other count.
 * Vector entry i of x_p is x[stridex p + incx i] (likewise y).  Runs as one
 * batched GEMM call: y as an m' x 1 matrix for op N with incy == 1,
 * otherwise y^T = alpha x^T op(A)^T + beta y^T with y^T a 1 x m' matrix of
 * leading dimension incy.  Positions: 1 trans, 2 m, 3 n, 4 alpha, 5 A, 6 lda
 * (>= max(1, m)), 7 strideA (>= 0), 8 x, 9 incx (>= 1; negative increments
 * are not supported), 10 stridex (>= 0), 11 beta, 12 y, 13 incy (>= 1),
 * 14 stridey (>= 0, and >= (len_y - 1) incy + 1 when batch_count > 1: output
 * vectors may not overlap), 15 batch_count, 16 stream.  Quick returns as in
 * BLAS: m == 0 or n == 0 leaves y unchanged; alpha == 0 and beta == 1 (host
 * mode) too.  alpha == 0 does not read A or x; beta == 0 does not read y.
 *
 * TRSM: side 'L' solves op(A_p) X_p = alpha B_p (A_p m x m), side 'R'
 * X_p op(A_p) = alpha B_p (A_p n x n); B_p is m x n and is overwritten by X_p.
 * uplo 'U'/'L' selects the triangle of A_p that is read; diag 'U' takes the
 * diagonal as ones without reading it, 'N' reads it.  The triangular order
 * s (m for L, n for R) may be any size: up to 16 one substitution kernel
 * (one 16-lane row of a wave per matrix); above 16, B is scaled by alpha,
 * then 16 x 16 diagonal blocks are solved by that kernel and the rest of B is
 * updated by batched GEMM calls (several launches on `stream`).  alpha == 0
 * sets B to zero without reading A (host mode; in device mode with s > 16 A
 * is still read).  No singularity check: a zero diagonal entry gives Inf/NaN
 * as in BLAS.  Positions: 1 side, 2 uplo, 3 transa (N, T, C), 4 diag, 5 m,
 * 6 n, 7 alpha, 8 A, 9 lda (>= max(1, s)), 10 strideA (>= 0), 11 B, 12 ldb
 * (>= max(1, m)), 13 strideB (>= ldb * n when batch_count > 1),
 * 14 batch_count, 15 stream.  Quick return: m == 0, n == 0 or
 * batch_count == 0. */
sbg_status_t sbg_sgemv_strided_batched(char trans, int m, int n, const float* alpha, const float* A, int lda,
    int64_t strideA, const float* x, int incx, int64_t stridex, const float* beta, float* y, int incy,
    int64_t stridey, int64_t batch_count, void* stream);
sbg_status_t sbg_dgemv_strided_batched(char trans, int m, int n, const double* alpha, const double* A, int lda,
    int64_t strideA, const double* x, int incx, int64_t stridex, const double* beta, double* y, int incy,
    int64_t stridey, int64_t batch_count, void* stream);
sbg_status_t sbg_cgemv_strided_batched(char trans, int m, int n, const sbg_cfloat* alpha, const sbg_cfloat* A,
    int lda, int64_t strideA, const sbg_cfloat* x, int incx, int64_t stridex, const sbg_cfloat* beta,
    sbg_cfloat* y, int incy, int64_t stridey, int64_t batch_count, void* stream);
sbg_status_t sbg_zgemv_strided_batched(char trans, int m, int n, const sbg_cdouble* alpha, const sbg_cdouble* A,
    int lda, int64_t strideA, const sbg_cdouble* x, int incx, int64_t stridex, const sbg_cdouble* beta,
    sbg_cdouble* y, int incy, int64_t stridey, int64_t batch_count, void* stream);
sbg_status_t sbg_strsm_strided_batched(char side, char uplo, char transa, char diag, int m, int n,
    const float* alpha, const float* A, int lda, int64_t strideA, float* B, int ldb, int64_t strideB,
    int64_t batch_count, void* stream);
sbg_status_t sbg_dtrsm_strided_batched(char side, char uplo, char transa, char diag, int m, int n,
    const double* alpha, const double* A, int lda, int64_t strideA, double* B, int ldb, int64_t strideB,
    int64_t batch_count, void* stream);
sbg_status_t sbg_ctrsm_strided_batched(char side, char uplo, char transa, char diag, int m, int n,
    const sbg_cfloat* alpha, const sbg_cfloat* A, int lda, int64_t strideA, sbg_cfloat* B, int ldb,
    int64_t strideB, int64_t batch_count, void* stream);
sbg_status_t sbg_ztrsm_strided_batched(char side, char uplo, char transa, char diag, int m, int n,
    const sbg_cdouble* alpha, const sbg_cdouble* A, int lda, int64_t strideA, sbg_cdouble* B, int ldb,
    int64_t strideB, int64_t batch_count, void* stream);

/* ---- library state ----------------------------------------------------------
 * sbg_set_scalar_mode: where alpha/beta live for calls made later by the
 *   calling thread (thread-local; default SBG_SCALAR_HOST).  In DEVICE mode the
 *   kernels read the scalars when they run, so a captured graph can be replayed
 *   with new values; the host-side quick returns on alpha/beta are skipped.
 * sbg_last_invalid_arg: 1-based position of the argument rejected by the
 *   calling thread's last SBG_INVALID_VALUE (0 if none).
 * sbg_status_string: static text for a status code.
 * sbg_version: library version as major*10000 + minor*100 + patch. */
void sbg_set_scalar_mode(sbg_scalar_mode_t mode);
sbg_scalar_mode_t sbg_get_scalar_mode(void);
int sbg_last_invalid_arg(void);
const char* sbg_status_string(sbg_status_t status);
int sbg_version(void);

/* ---- launch tuning ----------------------------------------------------------
 * Each call's kernel and launch shape come, in this order, from: knobs set to
 * a non-automatic value; the tuned table (one entry per type, batch form, op
 * pair and size max(m, n, k) <= 16, measured by the autotuner
 * paper_1304_7053_amd/tune.py and read once per process from SBG_TUNE_FILE or
 * from tuned.json beside the library); built-in rules.
 * Knobs are process-wide, for tuning sweeps and A/B comparisons (not
 * thread-safe against concurrent calls; set them before launching).  Keys
 * (0 = automatic unless stated):
 *   "wg_per_cu"   persistent grids: work-groups per CU, 0..32 (automatic: 4,
 *                 capped by the kernel's residency; a set value is taken as
 *                 given and may exceed it);
 *   "xcd_chunk"   consecutive work units per XCD run, >= 0 (automatic: 16);
 *   "staged"      packed strided batches through the LDS-staged kernel:
 *                 0 never, 1 always, 2 automatic (default);
 *   "path"        0 automatic, 1 MFMA tile kernels only, 2 team kernel for
 *                 sizes <= 8, 3 team kernel also up to 16 (real types);
 *   "unroll"      tiles per wave step of the direct kernel, 0..8 (a power of
 *                 two, capped per size class);
 *   "grid"        work-groups of persistent grids, 0..2^20 (the launch-shape
 *                 sweep; 0: CUs times wg_per_cu);
 *   "table"       1 (default) use the tuned table, 0 ignore it;
 *   "tile_bytes", "tile_bytes16"  per-wave bytes in flight that choose the
 *                 direct kernel's unroll when neither the knob nor the table
 *                 does (size classes 4/8 and 16; 256..2^20; the class-16
 *                 budget is for 4-byte elements and scales with the size);
 *   "pipeline"    0/1: prefetch the next tile group in the direct kernel;
 *   "blocked"     sizes above 16 (real types): 0 automatic (the LDS-staged
 *                 sub-blocked kernel where it measured faster), 1 the register
 *                 sub-blocked kernel only, 2 the LDS-staged kernel wherever it
 *                 applies (m, n, k <= 64 and leading dimensions of A and B
 *                 whose byte size is a multiple of 16).
 * Environment variables SBG_WG_PER_CU, SBG_XCD_CHUNK, SBG_STAGED, SBG_PATH,
 * SBG_UNROLL, SBG_GRID, SBG_TABLE, SBG_TILE_BYTES, SBG_TILE_BYTES16,
 * SBG_BLOCKED and SBG_PIPELINE set the initial values.
 * sbg_set_tuning returns the previous value, or -1 for an unknown key or an
 * out-of-range value (nothing changed); sbg_get_tuning returns the value or -1.
 * sbg_tuned_table_info writes "file=<path> version=<v> entries=<count>" into
 * buf (loading the table on first use) and returns the number of entries, or
 * -1 for a null or empty buffer. */
int sbg_set_tuning(const char* key, int value);
int sbg_get_tuning(const char* key);
int sbg_tuned_table_info(char* buf, int buflen);

/* ---- batched LU factorisation with partial pivoting (n <= 32) -------------
 * LAPACK GETRF on each n x n matrix A_p = A + strideA p (column-major, lda):
 * P_p A_p = L_p U_p, the largest magnitude on and below the diagonal chosen as
 * pivot in each column (the first on ties).  The factors overwrite A_p (L
 * unit lower, its ones not stored; U upper), ipiv[strideP p + k] (1-based) is
 * the row interchanged with row k at step k, and info[p] is 0, or the 1-based
 * index of the first exactly zero pivot (the factorisation still completes;
 * U is singular).  The paper proposes building further batched routines on
 * its batched interface (Sec. 9); this is the LU of that family.
 * Positions: 1 n (> 32: SBG_NOT_SUPPORTED), 2 A, 3 lda (>= max(1, n)),
 * 4 strideA (>= lda * n when batch_count > 1), 5 ipiv, 6 strideP (>= n when
 * batch_count > 1), 7 info, 8 batch_count, 9 stream.  n == 0 sets every
 * info[p] to 0; batch_count == 0 returns at once. */
sbg_status_t sbg_sgetrf_strided_batched(int n, float* A, int lda, int64_t strideA, int* ipiv, int64_t strideP,
    int* info, int64_t batch_count, void* stream);
sbg_status_t sbg_dgetrf_strided_batched(int n, double* A, int lda, int64_t strideA, int* ipiv, int64_t strideP,
    int* info, int64_t batch_count, void* stream);

/* ---- diagnostics --------------------------------------------------------
 * sbg_describe_strided: validates the arguments of a strided call (prefix
 *   's', 'd', 'c' or 'z' selects the entry point; alpha = 1, beta = 0.5 are
 *   assumed) and writes into buf the demangled symbol of the kernel that call
 *   would launch, as profilers report it.  Launches nothing, touches no device
 *   memory.  Returns 0, or -1 when the call would be rejected or return early
 *   (buf is then empty).  For benchmarks and profilers that attribute time to
 *   kernels. */
int sbg_describe_strided(char prefix, char transa, char transb, int m, int n, int k, int lda,
                         int64_t strideA, int ldb, int64_t strideB, int ldc, int64_t strideC,
                         int64_t batch_count, char* buf, int buflen);
/* sbg_describe_vbatched: the same for a variable-size call (prefix 's' goes
 *   through sbg_gemm_vbatched_ex with ab_type and mode; 'd', 'c', 'z' through
 *   the typed entry points and need SBG_R_32F / SBG_MODE_PLAIN).  Writes
 *   "kernel=<symbol> grid=<work-groups> units=<work units>": the persistent
 *   kernel, the work-groups the launcher would start (each runs 4 waves) and
 *   its work units (wave steps; for the binned MFMA path the upper bound,
 *   every matrix in the 16 class, followed by "u16= u8= u4=", the matrices
 *   per lane group and wave step of each class).  Launches nothing, touches
 *   no device memory (the grid comes from an occupancy query of the current
 *   device).  Returns 0, or -1 when the call would be rejected or return
 *   early. */
int sbg_describe_vbatched(char prefix, char transa, char transb, int max_m, int max_n, int max_k,
                          int64_t batch_count, sbg_datatype_t ab_type, sbg_compute_mode_t mode, char* buf,
                          int buflen);

#ifdef __cplusplus
}
#endif

#endif /* SBG_H */
