// Small triangular solves of a strided batch: the diagonal-block step of a
// batched TRSM in the paper's second-leading-dimension interface (the paper
// proposes the interface for other BLAS routines, formulated on batched GEMM,
// Sec. 9; the off-diagonal updates of larger solves are batched GEMM calls
// made by the host, api.cpp).
//
// One 16-lane row of a wave per matrix: lane r holds row r of the triangular
// matrix M and entry r of up to 16 right-hand-side vectors at a time, and the
// substitution runs as 16 steps in which the entries of one lane are final,
// they are broadcast across the row, and the lanes still to be solved
// subtract their share (rows are scaled by the reciprocal of their diagonal
// first).  alpha = 0 writes zeros and reads neither A nor B.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "gemm_tile.h"

namespace sbg {

template <typename T> __device__ __forceinline__ T t_mul(const T& a, const T& b);
template <typename T> __device__ __forceinline__ T t_sub(const T& a, const T& b);
template <typename T> __device__ __forceinline__ T t_div(const T& a, const T& b);
template <typename T> __device__ __forceinline__ T t_conj(const T& a);

template <> __device__ __forceinline__ float t_mul<float>(const float& a, const float& b) { return a * b; }
template <> __device__ __forceinline__ double t_mul<double>(const double& a, const double& b) { return a * b; }
template <> __device__ __forceinline__ float t_sub<float>(const float& a, const float& b) { return a - b; }
template <> __device__ __forceinline__ double t_sub<double>(const double& a, const double& b) { return a - b; }
template <> __device__ __forceinline__ float t_div<float>(const float& a, const float& b) { return a / b; }
template <> __device__ __forceinline__ double t_div<double>(const double& a, const double& b) { return a / b; }
template <> __device__ __forceinline__ float t_conj<float>(const float& a) { return a; }
template <> __device__ __forceinline__ double t_conj<double>(const double& a) { return a; }

template <typename C>
__device__ __forceinline__ C c_mul(const C& a, const C& b)
{
    C r;
    r.x = __builtin_fma(a.x, b.x, -(a.y * b.y));
    r.y = __builtin_fma(a.x, b.y, a.y * b.x);
    return r;
}
// a / b with the divisor scaled by its larger component (Smith's method), so
// |b|^2 neither overflows nor underflows for representable b
template <typename C>
__device__ __forceinline__ C c_div(const C& a, const C& b)
{
    C r;
    if (__builtin_fabs(b.x) >= __builtin_fabs(b.y)) {
        const auto q = b.y / b.x;
        const auto d = __builtin_fma(b.y, q, b.x);
        r.x = __builtin_fma(a.y, q, a.x) / d;
        r.y = __builtin_fma(-a.x, q, a.y) / d;
    } else {
        const auto q = b.x / b.y;
        const auto d = __builtin_fma(b.x, q, b.y);
        r.x = __builtin_fma(a.x, q, a.y) / d;
        r.y = __builtin_fma(a.y, q, -a.x) / d;
    }
    return r;
}
template <> __device__ __forceinline__ float2 t_mul<float2>(const float2& a, const float2& b) { return c_mul(a, b); }
template <> __device__ __forceinline__ double2 t_mul<double2>(const double2& a, const double2& b) { return c_mul(a, b); }
template <> __device__ __forceinline__ float2 t_sub<float2>(const float2& a, const float2& b)
{
    return make_float2(a.x - b.x, a.y - b.y);
}
template <> __device__ __forceinline__ double2 t_sub<double2>(const double2& a, const double2& b)
{
    return make_double2(a.x - b.x, a.y - b.y);
}
template <> __device__ __forceinline__ float2 t_div<float2>(const float2& a, const float2& b) { return c_div(a, b); }
template <> __device__ __forceinline__ double2 t_div<double2>(const double2& a, const double2& b) { return c_div(a, b); }
template <> __device__ __forceinline__ float2 t_conj<float2>(const float2& a) { return make_float2(a.x, -a.y); }
template <> __device__ __forceinline__ double2 t_conj<double2>(const double2& a) { return make_double2(a.x, -a.y); }

// Width-16 broadcast of lane `src` of each 16-lane row.
__device__ __forceinline__ float row_bcast(float v, int src) { return __shfl(v, src, 16); }
__device__ __forceinline__ double row_bcast(double v, int src) { return __shfl(v, src, 16); }
__device__ __forceinline__ float2 row_bcast(float2 v, int src)
{
    return make_float2(__shfl(v.x, src, 16), __shfl(v.y, src, 16));
}
__device__ __forceinline__ double2 row_bcast(double2 v, int src)
{
    return make_double2(__shfl(v.x, src, 16), __shfl(v.y, src, 16));
}

// Substitution with one 16-lane row per matrix (four matrices per wave): lane
// r holds row r of M and entry r of up to 16 right-hand-side vectors at a
// time, both scaled by the reciprocal of M(r, r) (computed once per lane).
// Step i: lane i's entries are final; they are broadcast across the row, and
// every lane below i (lower M; above i for upper) subtracts M(r, i) times
// them.  Loads and stores of one vector entry run across consecutive lanes.
template <typename T, bool LOWER, bool ETRANS>
__global__ __launch_bounds__(256) void trsm_row_kernel(const TrsmArgs<T> a)
{
    using R = typename Tr<T>::R;
    const int lane = threadIdx.x & 63;
    const int r = lane & 15;
    const int64_t p = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 4 + (lane >> 4);
    if (((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 4 >= a.batch) return;   // whole wave past the batch
    const bool live = p < a.batch;
    const int s = a.size;
    const bool row_ok = live && r < s;
    const T alpha = a.alpha_dev ? *a.alpha_dev : a.alpha;
    const T zero = make_val<T>(R(0), R(0));
    const int64_t pe = live ? p : a.batch - 1;
    T* bm = a.B + pe * a.strideB;
    const int64_t ve = a.vec_elem, vs = a.vec_step;
    if (is_zero(alpha)) {
        for (int64_t c0 = 0; c0 < a.nv; c0 += 16) {
#pragma unroll
            for (int v = 0; v < 16; ++v)
                if (row_ok && c0 + v < a.nv) bm[(c0 + v) * vs + r * ve] = zero;
        }
        return;
    }
    // row r of M (the triangle's part of it) and the reciprocal of M(r, r)
    const T* Am = a.A + pe * a.strideA;
    T mr[16];
#pragma unroll
    for (int l = 0; l < 16; ++l) {
        const bool need = row_ok && l < s && (LOWER ? l < r : l > r);
        T e = zero;
        if (need) {
            e = ETRANS ? Am[l + a.lda * r] : Am[r + a.lda * l];
            if (a.conj) e = t_conj<T>(e);
        }
        mr[l] = e;
    }
    // row r scaled by 1 / M(r, r) once: the system becomes unit-diagonal, so a
    // step only broadcasts a finished entry and subtracts its multiples
    T inv = make_val<T>(R(1), R(0));
    if (!a.unit && row_ok) {
        T d = Am[r + a.lda * r];
        if (a.conj) d = t_conj<T>(d);
        inv = t_div<T>(make_val<T>(R(1), R(0)), d);
#pragma unroll
        for (int l = 0; l < 16; ++l) mr[l] = t_mul<T>(inv, mr[l]);
    }
    const T ainv = t_mul<T>(alpha, inv);
    for (int64_t c0 = 0; c0 < a.nv; c0 += 16) {
        const int nvc = a.nv - c0 < 16 ? (int)(a.nv - c0) : 16;
        T x[16];
#pragma unroll
        for (int v = 0; v < 16; ++v)
            x[v] = (row_ok && v < nvc) ? t_mul<T>(ainv, bm[(c0 + v) * vs + r * ve]) : zero;
        // one substitution step for the vectors 0..NV-1 of the chunk
#define SBG_TRSM_STEPS(NV)                                                          \
        _Pragma("unroll") for (int q = 0; q < 16; ++q) {                            \
            const int i = LOWER ? q : 15 - q;                                       \
            if (i < s) {                                                            \
                const bool below = LOWER ? r > i : r < i;                           \
                const T m = mr[i];                                                  \
                _Pragma("unroll") for (int v = 0; v < 16; ++v) {                    \
                    if (v < (NV)) {                                                 \
                        const T xi = row_bcast(x[v], i);                            \
                        if (below) x[v] = t_sub<T>(x[v], t_mul<T>(m, xi));          \
                    }                                                               \
                }                                                                   \
            }                                                                       \
        }
        if (nvc == 16) {
            SBG_TRSM_STEPS(16)   // whole chunks: no per-vector test
        } else {
            SBG_TRSM_STEPS(nvc)
        }
#undef SBG_TRSM_STEPS
#pragma unroll
        for (int v = 0; v < 16; ++v)
            if (row_ok && v < nvc) bm[(c0 + v) * vs + r * ve] = x[v];
    }
}

template <typename T>
hipError_t launch_trsm_small_impl(const TrsmArgs<T>& a, hipStream_t stream)
{
    if (a.batch <= 0 || a.nv <= 0) return hipSuccess;
    const int64_t blocks = (a.batch + 15) / 16;   // 16 matrices per 256-thread work-group
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    auto kern = a.lower ? (a.eff_trans ? trsm_row_kernel<T, true, true> : trsm_row_kernel<T, true, false>)
                        : (a.eff_trans ? trsm_row_kernel<T, false, true> : trsm_row_kernel<T, false, false>);
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(256), 0, stream, a);
    return hipGetLastError();
}

}  // namespace sbg

#define SBG_INSTANTIATE_TRSM(T)                                                      \
    namespace sbg {                                                                  \
    template <>                                                                      \
    hipError_t launch_trsm_small<T>(const TrsmArgs<T>& a, hipStream_t s)             \
    {                                                                                \
        return launch_trsm_small_impl<T>(a, s);                                      \
    }                                                                                \
    }
