// Per-matrix absmax quantisation of binary32 matrices (<= 16 x 16) to OCP
// FP8 E4M3, the input format of the scaled fp8 precision mode.
//
// For matrix p: s_p = max |X_p| / 448 (448 = largest finite E4M3; s_p = 1 for
// an all-zero matrix), Q_p = E4M3(X_p / s_p) rounded to nearest, ties to
// even, saturating to +-448.  X_p ~= s_p * decode(Q_p); the GEMM applies s_A s_B
// to the product.  One wavefront per matrix: 4 entries per lane, absmax by a
// butterfly reduction across the wave.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "sbg_internal.h"

namespace sbg {

// binary32 -> E4M3 (OCP "fn"), round to nearest even, saturating finite
// values to 448; NaN maps to the E4M3 NaN code.
__device__ __forceinline__ unsigned char enc_e4m3(float v)
{
    const unsigned u = __float_as_uint(v);
    const unsigned sign = (u >> 24) & 0x80u;
    const unsigned a = u & 0x7FFFFFFFu;
    if (a > 0x7F800000u) return (unsigned char)(sign | 0x7Fu);
    if (a >= 0x43E80000u) return (unsigned char)(sign | 0x7Eu);   // |v| >= 464: saturate
    const int e = (int)(a >> 23) - 127;
    if (e >= -6) {
        // normal: keep 3 fraction bits, round to nearest even at bit 20
        const unsigned mant = a & 0x7FFFFFu;
        const unsigned r = mant + 0x7FFFFu + ((mant >> 20) & 1u);
        unsigned m3 = r >> 20;
        unsigned ef = (unsigned)(e + 7);
        if (m3 == 8u) {
            m3 = 0u;
            ef += 1u;
        }
        return (unsigned char)(sign | (ef << 3) | m3);
    }
    // subnormal: multiples of 2^-9 (a count of 8 is the smallest normal, 0x08)
    const unsigned m = (unsigned)__builtin_rintf(__uint_as_float(a) * 512.0f);
    return (unsigned char)(sign | m);
}


template <bool VAR>
__global__ __launch_bounds__(256) void quant_e4m3_kernel(const QuantArgs q)
{
    const int lane = threadIdx.x & 63;
    const int64_t W = (int64_t)gridDim.x * 4;
    for (int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); p < q.batch; p += W) {
        int rows = q.rows, cols = q.cols;
        int64_t ldx = q.ldx, ldq = q.ldq;
        const float* X;
        unsigned char* Q;
        if (VAR) {
            rows = q.drows[p];
            cols = q.dcols[p];
            ldx = q.dldx[p];
            ldq = q.dldq[p];
            X = q.Xarr[p];
            Q = q.Qarr[p];
            if (rows < 0 || cols < 0 || rows > q.max_rows || cols > q.max_cols || ldx < (rows > 1 ? rows : 1) ||
                ldq < (rows > 1 ? rows : 1))
                continue;   // invalid sizes: matrix skipped (its scale is not written)
        } else {
            X = q.X + p * q.strideX;
            Q = q.Q + p * q.strideQ;
        }
        const int cnt = rows * cols;
        float v[4];
        int ri[4], ci[4];
        float amax = 0.f;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int e = lane + 64 * t;
            v[t] = 0.f;
            ri[t] = 0;
            ci[t] = 0;
            if (e < cnt) {
                ri[t] = e % rows;
                ci[t] = e / rows;
                v[t] = X[ri[t] + ldx * ci[t]];
                amax = fmaxf(amax, fabsf(v[t]));
            }
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) amax = fmaxf(amax, __shfl_xor(amax, off));
        const float s = amax > 0.f ? amax / 448.0f : 1.0f;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int e = lane + 64 * t;
            if (e < cnt) Q[ri[t] + ldq * ci[t]] = enc_e4m3(v[t] / s);
        }
        if (lane == 0) q.scales[p] = s;
    }
}

hipError_t launch_quant_e4m3(const QuantArgs& q, bool var, hipStream_t stream)
{
    int64_t grid = (q.batch + 3) / 4;
    const int64_t cap = (int64_t)device_cu_count() * 8;
    if (grid > cap) grid = cap;
    if (grid < 1) grid = 1;
    if (var)
        hipLaunchKernelGGL(quant_e4m3_kernel<true>, dim3((unsigned)grid), dim3(256), 0, stream, q);
    else
        hipLaunchKernelGGL(quant_e4m3_kernel<false>, dim3((unsigned)grid), dim3(256), 0, stream, q);
    return hipGetLastError();
}

}  // namespace sbg
