// Small triangular solves of a strided batch: the diagonal-block step of a
// batched TRSM in the paper's second-leading-dimension interface (the paper
// proposes the interface for other BLAS routines, formulated on batched GEMM,
// Sec. 9; the off-diagonal updates of larger solves are batched GEMM calls
// made by the host, api.cpp).
//
// One thread owns one right-hand-side vector (a column of B for side L, a row
// for side R) of at most 16 entries, kept in registers, and substitutes
// through the triangle: forward for a lower M, backward for an upper one.
// With at least 8 vectors per matrix each work-group first copies its
// matrices into LDS (trsm_lds_kernel); otherwise entries of M are read from
// memory as they are needed (trsm_small_kernel), the threads of one matrix
// reading the same entries together.  alpha = 0 writes zeros and reads
// neither A nor B.
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

template <typename T, bool LOWER, bool ETRANS>
__global__ __launch_bounds__(256) void trsm_small_kernel(const TrsmArgs<T> a)
{
    using R = typename Tr<T>::R;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= a.batch * a.nv) return;
    const int64_t p = t / a.nv;
    const int64_t v = t - p * a.nv;
    const T alpha = a.alpha_dev ? *a.alpha_dev : a.alpha;
    T* b = a.B + p * a.strideB + v * a.vec_step;
    const int s = a.size;
    const int64_t ve = a.vec_elem;
    if (is_zero(alpha)) {
#pragma unroll
        for (int i = 0; i < 16; ++i)
            if (i < s) b[i * ve] = make_val<T>(R(0), R(0));
        return;
    }
    const T* A = a.A + p * a.strideA;
    const int64_t lda = a.lda;
    // M(i, l); only entries of the triangle (and the diagonal unless unit)
    // are ever requested
    const auto M = [&](int i, int l) -> T {
        const T e = ETRANS ? A[l + lda * i] : A[i + lda * l];
        return a.conj ? t_conj<T>(e) : e;
    };
    T x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i)
        x[i] = i < s ? t_mul<T>(alpha, b[i * ve]) : make_val<T>(R(0), R(0));
    if (LOWER) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            if (i < s) {
                T xi = x[i];
#pragma unroll
                for (int l = 0; l < i; ++l) xi = t_sub<T>(xi, t_mul<T>(M(i, l), x[l]));
                x[i] = a.unit ? xi : t_div<T>(xi, M(i, i));
            }
        }
    } else {
#pragma unroll
        for (int i = 15; i >= 0; --i) {
            if (i < s) {
                T xi = x[i];
#pragma unroll
                for (int l = i + 1; l < 16; ++l)
                    if (l < s) xi = t_sub<T>(xi, t_mul<T>(M(i, l), x[l]));
                x[i] = a.unit ? xi : t_div<T>(xi, M(i, i));
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 16; ++i)
        if (i < s) b[i * ve] = x[i];
}

// The same solves with each work-group staging its matrices in LDS: MB whole
// matrices per work-group (MB * nv <= 256 threads, one vector each), the
// stored size x size blocks copied with consecutive threads on consecutive
// elements, then every M(i, l) read from LDS (the threads of one matrix read
// the same word: a broadcast).  Used when a matrix has at least 8 vectors.
template <typename T, bool LOWER, bool ETRANS>
__global__ __launch_bounds__(256) void trsm_lds_kernel(const TrsmArgs<T> a, int MB)
{
    using R = typename Tr<T>::R;
    __shared__ T lm[16 * 256];                       // MB * size * size <= 16 * 256 entries
    const int s = a.size;
    const int ss = s * s;
    const int64_t p0 = (int64_t)blockIdx.x * MB;
    const int cnt = (int)(a.batch - p0 < MB ? a.batch - p0 : MB);
    const T alpha = a.alpha_dev ? *a.alpha_dev : a.alpha;
    const bool a0 = is_zero(alpha);
    if (!a0) {
        for (int e = threadIdx.x; e < cnt * ss; e += 256) {
            const int q = e / ss, r = e - q * ss;
            const int col = r / s, row = r - col * s;
            lm[e] = a.A[(p0 + q) * a.strideA + row + a.lda * col];
        }
    }
    __syncthreads();
    const int q = threadIdx.x / (int)a.nv;
    const int v = threadIdx.x - q * (int)a.nv;
    if (q >= cnt) return;
    T* b = a.B + (p0 + q) * a.strideB + v * a.vec_step;
    const int64_t ve = a.vec_elem;
    if (a0) {
#pragma unroll
        for (int i = 0; i < 16; ++i)
            if (i < s) b[i * ve] = make_val<T>(R(0), R(0));
        return;
    }
    const T* L = lm + q * ss;
    const auto M = [&](int i, int l) -> T {
        const T e = ETRANS ? L[l + s * i] : L[i + s * l];
        return a.conj ? t_conj<T>(e) : e;
    };
    T x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i)
        x[i] = i < s ? t_mul<T>(alpha, b[i * ve]) : make_val<T>(R(0), R(0));
    if (LOWER) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            if (i < s) {
                T xi = x[i];
#pragma unroll
                for (int l = 0; l < i; ++l) xi = t_sub<T>(xi, t_mul<T>(M(i, l), x[l]));
                x[i] = a.unit ? xi : t_div<T>(xi, M(i, i));
            }
        }
    } else {
#pragma unroll
        for (int i = 15; i >= 0; --i) {
            if (i < s) {
                T xi = x[i];
#pragma unroll
                for (int l = i + 1; l < 16; ++l)
                    if (l < s) xi = t_sub<T>(xi, t_mul<T>(M(i, l), x[l]));
                x[i] = a.unit ? xi : t_div<T>(xi, M(i, i));
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 16; ++i)
        if (i < s) b[i * ve] = x[i];
}

template <typename T>
hipError_t launch_trsm_small_impl(const TrsmArgs<T>& a, hipStream_t stream)
{
    const int64_t threads = a.batch * a.nv;
    if (threads <= 0) return hipSuccess;
    if (a.nv >= 8 && a.nv <= 256 && a.size >= 1 && a.size <= 16) {
        int MB = (int)(256 / a.nv);
        if (MB > 16) MB = 16;
        const int64_t blocks = (a.batch + MB - 1) / MB;
        if (blocks > 0x7fffffff) return hipErrorInvalidValue;
        auto kern = a.lower ? (a.eff_trans ? trsm_lds_kernel<T, true, true> : trsm_lds_kernel<T, true, false>)
                            : (a.eff_trans ? trsm_lds_kernel<T, false, true> : trsm_lds_kernel<T, false, false>);
        hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(256), 0, stream, a, MB);
        return hipGetLastError();
    }
    const int64_t blocks = (threads + 255) / 256;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    auto kern = a.lower ? (a.eff_trans ? trsm_small_kernel<T, true, true> : trsm_small_kernel<T, true, false>)
                        : (a.eff_trans ? trsm_small_kernel<T, false, true> : trsm_small_kernel<T, false, false>);
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
