// Batched small-matrix GEMM on CDNA4 matrix cores (gfx950).
//
// Computes C_p <- alpha op(A_p) op(B_p) + beta C_p (Sec. 2, Eq. (1)) for
// m, n, k <= 16.  Design (what differs from the paper's Sec. 7 thread-per-
// entry and register-blocked shared-memory kernels):
//
//  * One wavefront owns a "tile": 16/D independent matrices of size class D
//    (D = 4, 8 or 16) packed block-diagonally into one 16 x 16 x 16 product.
//    The 16 x 16 x 4 MFMA (f32 or f64) is applied D/4 times; the off-diagonal
//    blocks of the product mix two different matrices and are discarded.
//  * MFMA operand layout: lane L = 16 g + c (g = 0..3, c = 0..15) supplies
//    op(A)(row c, k-index pi) and op(B)(k-index pi, column c) at step kb,
//    with pi = (D/4) g + kb, so one lane's k-indices are consecutive.  A lane
//    therefore reads a row of op(A) and a column of op(B) of matrix c / D
//    straight from global memory: no LDS staging, no shuffles.  When the
//    k-index is the fast storage index (op T/C on A, op N/R on B) the lane's
//    D/4 values are one vector load; otherwise neighbouring lanes read
//    neighbouring addresses.
//  * The result registers follow the MFMA's own layout: f32 returns rows
//    4g..4g+3 of column c (one contiguous run, stored with one vector store),
//    f64 returns rows g, g+4, g+8, g+12.  A register is kept when its row and
//    column fall in the same diagonal block.
//  * Transposition selects one of four kernel variants (which operand has k
//    as its fast index); conjugation is a sign on the imaginary part (the
//    paper's functor idea, Sec. 6).
//  * Complex products use four real MFMAs (re*re, -im*im, re*im, im*re); the
//    3M method is not used (Sec. 8).
//  * The a1b0 / axpby distinction of Sec. 6 is a wave-uniform branch: with
//    beta == 0 C is never loaded, with alpha == 0 A and B are never loaded.
//  * Each wave keeps U tiles of loads in flight before it computes; the grid
//    is persistent, and work-groups are renumbered so that each XCD (dispatch
//    is round-robin over the 8 XCDs) takes runs of `xcd_chunk` consecutive
//    tile groups, keeping cache lines shared by neighbouring matrices inside
//    one L2.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>

#include "sbg_internal.h"

namespace sbg {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct Tr;
template <> struct Tr<float>   { using R = float;  static constexpr bool cplx = false; };
template <> struct Tr<double>  { using R = double; static constexpr bool cplx = false; };
template <> struct Tr<float2>  { using R = float;  static constexpr bool cplx = true; };
template <> struct Tr<double2> { using R = double; static constexpr bool cplx = true; };

// 16x16x4 MFMA per real type, with the row held by result register r of lane
// group g (the column is always the lane index mod 16).
template <typename R> struct Mfma;
template <> struct Mfma<float> {
    using acc_t = f32x4;
    static constexpr bool rows_contig = true;
    static __device__ __forceinline__ int row(int g, int r) { return 4 * g + r; }
    static __device__ __forceinline__ acc_t run(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <> struct Mfma<double> {
    using acc_t = f64x4;
    static constexpr bool rows_contig = false;
    static __device__ __forceinline__ int row(int g, int r) { return 4 * r + g; }
    static __device__ __forceinline__ acc_t run(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

template <typename T> __device__ __forceinline__ typename Tr<T>::R re_of(const T& v);
template <typename T> __device__ __forceinline__ typename Tr<T>::R im_of(const T& v);
template <> __device__ __forceinline__ float re_of<float>(const float& v) { return v; }
template <> __device__ __forceinline__ double re_of<double>(const double& v) { return v; }
template <> __device__ __forceinline__ float re_of<float2>(const float2& v) { return v.x; }
template <> __device__ __forceinline__ double re_of<double2>(const double2& v) { return v.x; }
template <> __device__ __forceinline__ float im_of<float>(const float&) { return 0.f; }
template <> __device__ __forceinline__ double im_of<double>(const double&) { return 0.0; }
template <> __device__ __forceinline__ float im_of<float2>(const float2& v) { return v.y; }
template <> __device__ __forceinline__ double im_of<double2>(const double2& v) { return v.y; }

template <typename T> __device__ __forceinline__ T make_val(typename Tr<T>::R re, typename Tr<T>::R im);
template <> __device__ __forceinline__ float make_val<float>(float re, float) { return re; }
template <> __device__ __forceinline__ double make_val<double>(double re, double) { return re; }
template <> __device__ __forceinline__ float2 make_val<float2>(float re, float im) { return make_float2(re, im); }
template <> __device__ __forceinline__ double2 make_val<double2>(double re, double im) { return make_double2(re, im); }

template <typename T>
__device__ __forceinline__ bool is_zero(const T& v) {
    return re_of<T>(v) == 0 && im_of<T>(v) == 0;
}

// Read `cnt` consecutive elements starting at p into v[0..cnt) as one
// (possibly unaligned, element-aligned) vector access.
template <typename T, int CNT>
__device__ __forceinline__ void vload(T (&v)[CNT], const T* p) {
    __builtin_memcpy(v, p, sizeof(T) * CNT);
}
template <typename T, int CNT>
__device__ __forceinline__ void vstore(T* p, const T (&v)[CNT]) {
    __builtin_memcpy(p, v, sizeof(T) * CNT);
}

// D: size class; U: tiles per wave per step; ACONT: op(A) in {T, C} (k is
// A's fast index); BCONT: op(B) in {N, R} (k is B's fast index); PTR:
// pointer-array form.
template <typename T, int D, int U, bool ACONT, bool BCONT, bool PTR>
__global__ __launch_bounds__(256) void gemm_mfma_kernel(const GemmArgs<T> a)
{
    using R = typename Tr<T>::R;
    using M = Mfma<R>;
    using acc_t = typename M::acc_t;
    constexpr bool CPLX = Tr<T>::cplx;
    constexpr int P = 16 / D;       // matrices per tile
    constexpr int KB = D / 4;       // 16x16x4 steps per tile

    const int lane = threadIdx.x & 63;
    const int g = lane >> 4;
    const int c = lane & 15;
    const int sel = c / D;          // matrix of the tile this lane feeds
    const int ij = c % D;           // its row of op(A) / column of op(B) and C
    const int kk0 = KB * g;         // first k-index this lane supplies

    const T alpha = a.alpha_dev ? *a.alpha_dev : a.alpha;
    const T beta = a.beta_dev ? *a.beta_dev : a.beta;
    const bool a0 = is_zero(alpha);
    const bool b0 = is_zero(beta);
    const R ar_ = re_of<T>(alpha), ai_ = im_of<T>(alpha);
    const R br_ = re_of<T>(beta), bi_ = im_of<T>(beta);

    const int m = a.m, n = a.n, k = a.k;
    const bool row_ok = ij < m;   // this lane's op(A) row exists
    const bool col_ok = ij < n;   // this lane's op(B)/C column exists
    const bool kfull = kk0 + KB <= k;
    const int64_t lda = a.lda, ldb = a.ldb, ldc = a.ldc;

    // Result registers this lane keeps: row of the tile = M::row(g, r).
    bool keep[4];
    int orow[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int Rr = M::row(g, r);
        keep[r] = (Rr / D) == sel;
        orow[r] = Rr % D;
    }
    // f32 layout: the 4 rows are one contiguous run (kept together or not)
    const bool crun = M::rows_contig && keep[0] && col_ok && (orow[0] + 3) < m;

    // Persistent traversal with XCD-aware renumbering (gridDim.x % 8 == 0).
    const int64_t W = (int64_t)gridDim.x * 4;
    const int64_t local = (int64_t)(blockIdx.x >> 3) * 4 + (threadIdx.x >> 6);
    const int64_t xcd = blockIdx.x & 7;
    const int64_t S = a.xcd_chunk;
    const int64_t q = ((local / S) * 8 + xcd) * S + (local % S);
    const int64_t ntiles = (a.batch + P - 1) / P;
    const int64_t ngroups = (ntiles + U - 1) / U;

    for (int64_t grp = q; grp < ngroups; grp += W) {
        R xa_r[U][KB], xa_i[U][KB], xb_r[U][KB], xb_i[U][KB];
        T cin[U][4];
        T* Cp[U];
        bool pv[U];

#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t p = ((grp * U + u) * P) + sel;
            pv[u] = p < a.batch;
            const T* Ap = nullptr;
            const T* Bp = nullptr;
            Cp[u] = nullptr;
            if (pv[u]) {
                if (PTR) {
                    if (!a0) { Ap = a.Aarr[p]; Bp = a.Barr[p]; }
                    Cp[u] = a.Carr[p];
                } else {
                    Ap = a.A + p * a.strideA;
                    Bp = a.B + p * a.strideB;
                    Cp[u] = a.C + p * a.strideC;
                }
            }
            T va[KB], vb[KB];
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
                va[kb] = make_val<T>(R(0), R(0));
                vb[kb] = make_val<T>(R(0), R(0));
            }
            const bool live = pv[u] && !a0;
            // ---- op(A) row ij, k-indices kk0 .. kk0+KB-1
            if (live && row_ok) {
                if (ACONT) {
                    const T* src = Ap + ij * lda + kk0;
                    if (kfull) {
                        vload<T, KB>(va, src);
                    } else {
#pragma unroll
                        for (int kb = 0; kb < KB; ++kb)
                            if (kk0 + kb < k) va[kb] = src[kb];
                    }
                } else {
#pragma unroll
                    for (int kb = 0; kb < KB; ++kb)
                        if (kk0 + kb < k) va[kb] = Ap[ij + (kk0 + kb) * lda];
                }
            }
            // ---- op(B) column ij, k-indices kk0 .. kk0+KB-1
            if (live && col_ok) {
                if (BCONT) {
                    const T* src = Bp + ij * ldb + kk0;
                    if (kfull) {
                        vload<T, KB>(vb, src);
                    } else {
#pragma unroll
                        for (int kb = 0; kb < KB; ++kb)
                            if (kk0 + kb < k) vb[kb] = src[kb];
                    }
                } else {
#pragma unroll
                    for (int kb = 0; kb < KB; ++kb)
                        if (kk0 + kb < k) vb[kb] = Bp[ij + (kk0 + kb) * ldb];
                }
            }
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
                xa_r[u][kb] = re_of<T>(va[kb]);
                xb_r[u][kb] = re_of<T>(vb[kb]);
                if (CPLX) {
                    xa_i[u][kb] = im_of<T>(va[kb]) * (R)a.a_conj;
                    xb_i[u][kb] = im_of<T>(vb[kb]) * (R)a.b_conj;
                }
            }
            // ---- C input (only when beta != 0)
#pragma unroll
            for (int r = 0; r < 4; ++r) cin[u][r] = make_val<T>(R(0), R(0));
            if (!b0 && pv[u]) {
                T* cbase = Cp[u] + ij * ldc;
                if (crun) {
                    vload<T, 4>(cin[u], cbase + orow[0]);
                } else if (col_ok) {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (keep[r] && orow[r] < m) cin[u][r] = cbase[orow[r]];
                }
            }
        }

#pragma unroll
        for (int u = 0; u < U; ++u) {
            acc_t acc_r = {0, 0, 0, 0};
            acc_t acc_i = {0, 0, 0, 0};
            if (!a0) {
#pragma unroll
                for (int kb = 0; kb < KB; ++kb) {
                    acc_r = M::run(xa_r[u][kb], xb_r[u][kb], acc_r);
                    if (CPLX) {
                        acc_r = M::run(-xa_i[u][kb], xb_i[u][kb], acc_r);
                        acc_i = M::run(xa_r[u][kb], xb_i[u][kb], acc_i);
                        acc_i = M::run(xa_i[u][kb], xb_r[u][kb], acc_i);
                    }
                }
            }
            if (!(pv[u] && col_ok)) continue;
            T out[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const R cr = re_of<T>(cin[u][r]);
                const R ci = im_of<T>(cin[u][r]);
                R outr, outi = 0;
                if (!CPLX) {
                    if (a0)
                        outr = b0 ? R(0) : br_ * cr;
                    else if (b0)
                        outr = ar_ * acc_r[r];
                    else
                        outr = __builtin_fma(ar_, acc_r[r], br_ * cr);
                } else {
                    R tr = 0, ti = 0;
                    if (!b0) {
                        tr = __builtin_fma(br_, cr, -(bi_ * ci));
                        ti = __builtin_fma(br_, ci, bi_ * cr);
                    }
                    if (!a0) {
                        tr = __builtin_fma(ar_, acc_r[r], __builtin_fma(-ai_, acc_i[r], tr));
                        ti = __builtin_fma(ar_, acc_i[r], __builtin_fma(ai_, acc_r[r], ti));
                    }
                    outr = tr;
                    outi = ti;
                }
                out[r] = make_val<T>(outr, outi);
            }
            T* cbase = Cp[u] + ij * ldc;
            if (crun) {
                vstore<T, 4>(cbase + orow[0], out);
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (keep[r] && orow[r] < m) cbase[orow[r]] = out[r];
            }
        }
    }
}

// Tiles per wave per step: keep roughly 3-6 KB of operand loads in flight per
// wave whatever the element size and size class.
template <typename T, int D> struct Unroll {
    static constexpr int bytes = sizeof(T);
    static constexpr int per_tile = 3 * 16 * D * bytes;   // A, B, C of the packed tile
    static constexpr int value = per_tile >= 6144 ? 1 : (per_tile >= 3072 ? 2 : 4);
};

// Work-groups that fit on one CU at once (registers and LDS), cached per kernel.
template <typename K>
inline int resident_per_cu(K kernel)
{
    static int cached = 0;
    if (cached == 0) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, 256, 0) != hipSuccess || nb <= 0) nb = 1;
        cached = nb;
    }
    return cached;
}

// Persistent grid for `units` independent wave-sized work units: at most the
// resident work-groups (capped by the tuning knob), a multiple of 8 so the
// XCD renumbering is exact; sets the XCD run length to a divisor of the
// waves per XCD.
template <typename T, typename K>
inline int64_t persistent_grid(K kernel, int64_t units, GemmArgs<T>& a)
{
    const Tuning& tu = tuning();
    int per_cu = resident_per_cu(kernel);
    if (per_cu > tu.wg_per_cu) per_cu = tu.wg_per_cu;
    const int64_t wg_needed = (units + 3) / 4;
    const int64_t cap = (int64_t)device_cu_count() * per_cu;
    int64_t grid = wg_needed < cap ? wg_needed : cap;
    grid = ((grid + 7) / 8) * 8;
    const int64_t wx = grid / 8 * 4;   // waves per XCD
    int64_t s = tu.xcd_chunk > 0 ? tu.xcd_chunk : 1;
    if (s > wx) s = wx;
    while (wx % s) --s;
    a.xcd_chunk = s;
    return grid;
}

template <typename T, int D, bool ACONT, bool BCONT, bool PTR>
hipError_t launch_variant(GemmArgs<T> a, hipStream_t stream)
{
    constexpr int U = Unroll<T, D>::value;
    constexpr int P = 16 / D;
    auto kern = gemm_mfma_kernel<T, D, U, ACONT, BCONT, PTR>;
    const int64_t tiles = (a.batch + P - 1) / P;
    const int64_t groups = (tiles + U - 1) / U;
    const int64_t grid = persistent_grid(kern, groups, a);
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(256), 0, stream, a);
    return hipGetLastError();
}

template <typename T, int D, bool ACONT, bool BCONT>
hipError_t launch_staged(GemmArgs<T> a, hipStream_t stream);
template <typename T>
int staged_run_length(int m, int n, int k, int64_t batch, int min_waves);

template <typename T, int D, bool PTR>
hipError_t launch_ops(const GemmArgs<T>& a, hipStream_t stream)
{
    if (!PTR && a.G > 0) {
        if (a.a_trans)
            return a.b_trans ? launch_staged<T, D, true, false>(a, stream)
                             : launch_staged<T, D, true, true>(a, stream);
        return a.b_trans ? launch_staged<T, D, false, false>(a, stream)
                         : launch_staged<T, D, false, true>(a, stream);
    }
    const bool at = a.a_trans, bn = !a.b_trans;
    if (at) {
        if (bn) return launch_variant<T, D, true, true, PTR>(a, stream);
        return launch_variant<T, D, true, false, PTR>(a, stream);
    }
    if (bn) return launch_variant<T, D, false, true, PTR>(a, stream);
    return launch_variant<T, D, false, false, PTR>(a, stream);
}

template <typename T>
hipError_t launch_gemm_impl(GemmArgs<T> a, bool pointer_form, hipStream_t stream)
{
    a.G = 0;
    if (!pointer_form) {
        // packed layout: minimal leading dimensions and strides (lda, ldb are
        // the stored row counts, which depend on the ops)
        const int64_t ra = a.a_trans ? a.k : a.m, ca = a.a_trans ? a.m : a.k;
        const int64_t rb = a.b_trans ? a.n : a.k, cb = a.b_trans ? a.k : a.n;
        const bool packed = a.k >= 1 && a.lda == ra && a.ldb == rb && a.ldc == a.m &&
                            a.strideA == ra * ca && a.strideB == rb * cb &&
                            a.strideC == (int64_t)a.m * a.n;
        if (packed && tuning().staged) a.G = staged_run_length<T>(a.m, a.n, a.k, a.batch, device_cu_count() * 16);
    }
    int mx = a.m > a.n ? a.m : a.n;
    mx = mx > a.k ? mx : a.k;
    if (pointer_form) {
        if (mx <= 4) return launch_ops<T, 4, true>(a, stream);
        if (mx <= 8) return launch_ops<T, 8, true>(a, stream);
        return launch_ops<T, 16, true>(a, stream);
    }
    if (mx <= 4) return launch_ops<T, 4, false>(a, stream);
    if (mx <= 8) return launch_ops<T, 8, false>(a, stream);
    return launch_ops<T, 16, false>(a, stream);
}

template <typename T> struct TypeName;
template <> struct TypeName<float> { static constexpr const char* s = "float"; };
template <> struct TypeName<double> { static constexpr const char* s = "double"; };
template <> struct TypeName<float2> { static constexpr const char* s = "HIP_vector_type<float, 2u>"; };
template <> struct TypeName<double2> { static constexpr const char* s = "HIP_vector_type<double, 2u>"; };

// The kernel symbol (as profilers demangle it) a launch with these arguments
// uses, written into buf.
template <typename T>
int describe_gemm_impl(GemmArgs<T> a, bool pointer_form, char* buf, int len)
{
    const auto tf = [](bool b) { return b ? "true" : "false"; };
    int mx = a.m > a.n ? a.m : a.n;
    mx = mx > a.k ? mx : a.k;
    const int D = mx <= 4 ? 4 : (mx <= 8 ? 8 : 16);
    int G = 0;
    if (!pointer_form) {
        const int64_t ra = a.a_trans ? a.k : a.m, ca = a.a_trans ? a.m : a.k;
        const int64_t rb = a.b_trans ? a.n : a.k, cb = a.b_trans ? a.k : a.n;
        const bool packed = a.k >= 1 && a.lda == ra && a.ldb == rb && a.ldc == a.m &&
                            a.strideA == ra * ca && a.strideB == rb * cb &&
                            a.strideC == (int64_t)a.m * a.n;
        if (packed && tuning().staged) G = 1;
    }
    if (G)
        return snprintf(buf, len, "void sbg::gemm_staged_kernel<%s, %d, %s, %s>(sbg::GemmArgs<%s>)",
                        TypeName<T>::s, D, tf(a.a_trans), tf(!a.b_trans), TypeName<T>::s);
    const int U = D == 4 ? Unroll<T, 4>::value : (D == 8 ? Unroll<T, 8>::value : Unroll<T, 16>::value);
    return snprintf(buf, len, "void sbg::gemm_mfma_kernel<%s, %d, %d, %s, %s, %s>(sbg::GemmArgs<%s>)",
                    TypeName<T>::s, D, U, tf(a.a_trans), tf(!a.b_trans), tf(pointer_form), TypeName<T>::s);
}

}  // namespace sbg

#define SBG_INSTANTIATE_GEMM(T)                                                      \
    namespace sbg {                                                                  \
    template <>                                                                      \
    hipError_t launch_gemm<T>(const GemmArgs<T>& a, bool pointer_form, hipStream_t s) \
    {                                                                                \
        return launch_gemm_impl<T>(a, pointer_form, s);                              \
    }                                                                                \
    template <>                                                                      \
    int describe_gemm<T>(const GemmArgs<T>& a, bool pointer_form, char* buf, int len) \
    {                                                                                \
        return describe_gemm_impl<T>(a, pointer_form, buf, len);                     \
    }                                                                                \
    }
