// Per-matrix absmax quantisation of binary32 matrices (<= 16 x 16) to OCP
// FP8 E4M3, the input format of the scaled fp8 precision mode.
//
// For matrix p: s_p = max |X_p| / 448 (448 = largest finite E4M3; s_p = 1 for
// an all-zero matrix), Q_p = E4M3(X_p / s_p) rounded to nearest, ties to
// even, saturating to +-448.  X_p ~= s_p * decode(Q_p); the GEMM applies s_A s_B
// to the product.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "gemm_vbteam.h"
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


// Largest value of x over each row of 16 lanes (DPP row rotations).
__device__ __forceinline__ float row16_max(float x)
{
#define SBG_ROR(N)                                                                                       \
    x = fmaxf(x, __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0x120 + (N), \
                                                                    0xF, 0xF, false)));
    SBG_ROR(8)
    SBG_ROR(4)
    SBG_ROR(2)
    SBG_ROR(1)
#undef SBG_ROR
    return x;
}

// One team of 16 lanes per matrix (4 matrices per wave step, a persistent
// grid over the batch): lane t loads column t (<= 16 rows) as 16-byte vectors
// with every load issued before the first wait (the column loader of the
// variable-size team kernel), the team's absmax comes from DPP row
// rotations, and each lane encodes and stores its column.  A lane past the
// matrix's columns, or a team with nothing to load, reads a valid dummy
// address instead.
// Sizes, leading dimensions and pointers of the matrix a team quantises
// (read one step ahead, so the reads overlap the previous step).
struct QuantMat {
    const float* X;
    unsigned char* Q;
    int64_t ldx, ldq;
    int rows, cols;
    bool in;
};

template <bool VAR>
__device__ __forceinline__ QuantMat quant_load(const QuantArgs& q, int64_t p0)
{
    QuantMat r;
    r.in = p0 < q.batch;
    const int64_t p = r.in ? p0 : q.batch - 1;
    if (VAR) {
        r.rows = q.drows[p];
        r.cols = q.dcols[p];
        r.ldx = q.dldx[p];
        r.ldq = q.dldq[p];
        r.X = q.Xarr[p];
        r.Q = q.Qarr[p];
    } else {
        r.rows = q.rows;
        r.cols = q.cols;
        r.ldx = q.ldx;
        r.ldq = q.ldq;
        r.X = q.X + p * q.strideX;
        r.Q = q.Q + p * q.strideQ;
    }
    return r;
}

// One team of 16 lanes per matrix (4 matrices per wave step, a persistent
// grid over the batch): lane t loads column t (<= 16 rows) as 16-byte vectors
// with every load issued before the first wait (the column loader of the
// variable-size team kernel), the team's absmax comes from DPP row
// rotations, and each lane encodes and stores its column.  A lane past the
// matrix's columns, or a team with nothing to load, reads a valid dummy
// address instead.
template <bool VAR>
__global__ __launch_bounds__(256) void quant_e4m3_kernel(const QuantArgs q)
{
    const int lane = threadIdx.x & 63;
    const int team = lane >> 4, t = lane & 15;
    const int64_t steps = (q.batch + 3) / 4;
    const int64_t W = (int64_t)gridDim.x * 4;
    int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (g >= steps) return;
    QuantMat nx = quant_load<VAR>(q, g * 4 + team);
    // the first reads complete before the loop, so that at its head the wait
    // covers only the reads issued one step earlier
    __asm__ volatile("" ::"v"(nx.rows), "v"(nx.cols), "v"(nx.ldx), "v"(nx.ldq), "v"(nx.X), "v"(nx.Q));
    for (; g < steps; g += W) {
        const QuantMat mt = nx;
        const int64_t p = mt.in ? g * 4 + team : q.batch - 1;
        nx = quant_load<VAR>(q, (g + W < steps ? g + W : g) * 4 + team);
        const int rows = mt.rows, cols = mt.cols;
        const int64_t ldx = mt.ldx, ldq = mt.ldq;
        const float* X = mt.X;
        unsigned char* Q = mt.Q;
        bool ok = mt.in;
        if (VAR) {
            // invalid sizes: the matrix is skipped (its scale is not written)
            ok = ok && !(rows < 0 || cols < 0 || rows > q.max_rows || cols > q.max_cols ||
                         ldx < (rows > 1 ? rows : 1) || ldq < (rows > 1 ? rows : 1));
        }
        const bool has = ok && rows > 0 && cols > 0;
        const bool mine = has && t < cols;
        // the dummy: the matrix's row count (variable-size) or its first column
        const GBy dummy = VAR ? gby(q.drows + p) : gby(X);
        const GBy col = mine ? gby(X + (int64_t)t * ldx) : dummy;
        const int L = mine ? rows * 4 : 4;
        VbCol<4> r;
        vb_issue<4>(r, col, L);
        vb_u4 x[4];
        vb_fix<4, false>(x, r, col, L);
        float v[16];
        float amax = 0.f;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const unsigned w = e % 4 == 0 ? x[e / 4].x : (e % 4 == 1 ? x[e / 4].y : (e % 4 == 2 ? x[e / 4].z : x[e / 4].w));
            v[e] = (mine && e < rows) ? __uint_as_float(w) : 0.f;
            amax = fmaxf(amax, fabsf(v[e]));
        }
        amax = row16_max(amax);
        const float s = amax > 0.f ? amax / 448.0f : 1.0f;
        // Fast path: multiply by the hardware reciprocal of s (1 ulp) instead
        // of dividing.  The product is within 2^-22 relative of the exact
        // quotient v / s and of its rounded value fl(v / s), so fl(v / s) lies
        // in [lo, hi] = qa -+ |qa| 2^-20.  The conversion rounds monotonically,
        // so when lo and hi give the same code every value between them does,
        // fl(v / s) included: that code is the exact one.  A wave with an
        // element whose bracket straddles a rounding boundary (about one
        // element in 65,000 for values spread over the e4m3 range), a scale
        // outside [2^-100, 2^100] or a non-finite value divides instead.  The hardware conversion gives the codes of
        // enc_e4m3 for every binary32 value of magnitude below 464 (checked
        // exhaustively on the device); here every converted value is below
        // 460.
        unsigned codes[4];
        bool slow = !(s >= 0x1p-100f && s <= 0x1p100f);   // NaN too
        {
            const float r = __builtin_amdgcn_rcpf(s);
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                float lo[4], hi[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float qa = v[4 * d + j] * r;
                    slow = slow || !(fabsf(qa) < 460.0f);
                    lo[j] = __builtin_fmaf(-fabsf(qa), 0x1p-20f, qa);
                    hi[j] = __builtin_fmaf(fabsf(qa), 0x1p-20f, qa);
                }
                const int l0 = __builtin_amdgcn_cvt_pk_fp8_f32(lo[0], lo[1], 0, false);
                const int l1 = __builtin_amdgcn_cvt_pk_fp8_f32(lo[2], lo[3], l0, true);
                const int h0 = __builtin_amdgcn_cvt_pk_fp8_f32(hi[0], hi[1], 0, false);
                const int h1 = __builtin_amdgcn_cvt_pk_fp8_f32(hi[2], hi[3], h0, true);
                slow = slow || l1 != h1;
                codes[d] = (unsigned)l1;
            }
        }
        if (__builtin_amdgcn_ballot_w64(slow) != 0) {
            float qv[16];
            bool wide = false;
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                qv[e] = v[e] / s;
                wide = wide || !(fabsf(qv[e]) < 464.0f);   // NaN too
            }
            // quotients of finite inputs never exceed 448 (1 + 2^-23); a wave
            // holding a larger value or a NaN takes the software encoder
            if (__builtin_amdgcn_ballot_w64(wide) == 0) {
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    const int lo = __builtin_amdgcn_cvt_pk_fp8_f32(qv[4 * d], qv[4 * d + 1], 0, false);
                    codes[d] = (unsigned)__builtin_amdgcn_cvt_pk_fp8_f32(qv[4 * d + 2], qv[4 * d + 3], lo, true);
                }
            } else {
#pragma unroll
                for (int d = 0; d < 4; ++d)
                    codes[d] = (unsigned)enc_e4m3(qv[4 * d]) | ((unsigned)enc_e4m3(qv[4 * d + 1]) << 8) |
                               ((unsigned)enc_e4m3(qv[4 * d + 2]) << 16) |
                               ((unsigned)enc_e4m3(qv[4 * d + 3]) << 24);
            }
        }
        if (mine) {
            // The column's rows bytes as up to 3 head bytes (to the first
            // 4-byte boundary), whole aligned dwords, and up to 3 tail bytes:
            // at most 10 stores in place of 16 byte stores, every one inside
            // [qc, qc + rows).
            const GByw qc = (GByw)(Q + (int64_t)t * ldq);
            const int h0 = (int)((0u - (unsigned)reinterpret_cast<uintptr_t>(qc)) & 3u);
            const int h = h0 < rows ? h0 : rows;
            const int nd = (rows - h) >> 2;
            const int tb = h + 4 * nd;
#pragma unroll
            for (int j = 0; j < 3; ++j)
                if (j < h) qc[j] = (unsigned char)(codes[0] >> (8 * j));
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (i < nd)
                    *(__attribute__((address_space(1))) unsigned*)(qc + h + 4 * i) =
                        __builtin_amdgcn_alignbyte(i < 3 ? codes[i + 1] : 0u, codes[i], (unsigned)h);
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int e = tb + j;
                const unsigned w = e < 4 ? codes[0] : (e < 8 ? codes[1] : (e < 12 ? codes[2] : codes[3]));
                if (e < rows) qc[e] = (unsigned char)(w >> (8 * (e & 3)));
            }
        }
        if (ok && t == 0) q.scales[p] = s;   // an empty matrix gets scale 1
    }
}

hipError_t launch_quant_e4m3(const QuantArgs& q, bool var, hipStream_t stream)
{
    const int64_t steps = (q.batch + 3) / 4;
    int64_t grid = (steps + 3) / 4;
    const int64_t cap = (int64_t)device_cu_count() * 16;
    if (grid > cap) grid = cap;
    if (grid < 1) grid = 1;
    if (var)
        hipLaunchKernelGGL(quant_e4m3_kernel<true>, dim3((unsigned)grid), dim3(256), 0, stream, q);
    else
        hipLaunchKernelGGL(quant_e4m3_kernel<false>, dim3((unsigned)grid), dim3(256), 0, stream, q);
    return hipGetLastError();
}

}  // namespace sbg
