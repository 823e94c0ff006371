// Batched GEMM for sizes above 16 by sub-blocking.  The paper's kernels stop
// at 16; it notes that the method extends to larger sizes (abstract, Sec. 1)
// and that other shapes can be multiplied as sub-blocks with its square
// kernels (Sec. 7).  Here C_p is cut into 16 x 16 blocks and the k range into
// 16-wide chunks.
//
//  * One wavefront computes one output block (rows 16 bi.., columns 16 bj.. of
//    matrix p) per work unit.  A k-chunk of the block is exactly a 16-class
//    tile of the direct kernel whose matrix is the sub-matrix: op(A) rows of
//    the block x the chunk's k-range, op(B) the chunk's k-range x the block's
//    columns -- the same leading dimensions, offset base pointers, sizes
//    min(16, remaining).  So the direct kernel's tile loads and MFMA steps
//    are reused unchanged.
//  * U consecutive chunks form one group: their loads are all in flight
//    before any is multiplied, and their products go into ONE accumulator;
//    groups repeat until k is exhausted, then a single epilogue applies
//    alpha and beta and writes the block (C is read once, with the first
//    group, when beta != 0).
//  * Work units run block-row fastest, then block-column, then matrix, so
//    the waves of one matrix are neighbours in the XCD-aware persistent grid
//    and re-read that matrix's A and B blocks from the same L2.
#pragma once

#include <map>
#include <mutex>
#include <utility>

#include "gemm_direct.h"

namespace sbg {

template <typename T, int U, bool ACONT, bool BCONT, bool PTR>
__global__ __launch_bounds__(256) void gemm_blocked_kernel(const GemmArgs<T> a)
{
    using R = typename Tr<T>::R;
    using acc_t = typename Mfma<R>::acc_t;
    const LaneGeom<16, R> L;
    T alpha, beta;
    alpha = a.alpha_dev ? *a.alpha_dev : a.alpha;
    beta = a.beta_dev ? *a.beta_dev : a.beta;
    const bool a0 = is_zero(alpha), b0 = is_zero(beta);

    const int m = a.m, n = a.n, k = a.k;
    const int64_t nbm = (m + 15) >> 4, nbn = (n + 15) >> 4;
    const int64_t nbb = nbm * nbn;                  // blocks per matrix
    const int nkc = (k + 15) >> 4;                  // k-chunks
    // at least one group: it loads C (k == 0 or alpha == 0 leave C = beta C)
    const int ngroups = (a0 || nkc <= U) ? 1 : (nkc + U - 1) / U;
    const int64_t units = a.batch * nbb;
    const int64_t W = (int64_t)gridDim.x * 4;

    for (int64_t w = xcd_wave_index(a.xcd_chunk); w < units; w += W) {
        const int64_t p = w / nbb;
        const int64_t rest = w - p * nbb;
        const int64_t bj = rest / nbm;
        const int64_t bi = rest - bj * nbm;
        const int row0 = (int)(16 * bi), col0 = (int)(16 * bj);
        const int mb = m - row0 < 16 ? m - row0 : 16;
        const int nb = n - col0 < 16 ? n - col0 : 16;

        const T* Ab = nullptr;
        const T* Bb = nullptr;
        T* Cb;
        if (PTR) {
            if (!a0) {
                Ab = static_cast<const T*>(a.Aarr[p]);
                Bb = static_cast<const T*>(a.Barr[p]);
            }
            Cb = a.Carr[p];
        } else {
            if (!a0) {
                Ab = static_cast<const T*>(a.A) + p * a.strideA;
                Bb = static_cast<const T*>(a.B) + p * a.strideB;
            }
            Cb = a.C + p * a.strideC;
        }
        // the output block (and the C entries the epilogue reads)
        LaneMat<T, T, 1> blk;
        blk.A = nullptr;
        blk.B = nullptr;
        blk.C = in_space<1>(Cb + row0 + (int64_t)col0 * a.ldc);
        blk.m = mb;
        blk.n = nb;
        blk.k = 0;
        blk.lda = a.lda;
        blk.ldb = a.ldb;
        blk.ldc = a.ldc;
        blk.scale = 1.0f;
        blk.valid = true;
        blk.overA = blk.overB = blk.overC = false;

        acc_t acc_r = {0, 0, 0, 0};
        acc_t acc_i = {0, 0, 0, 0};
        TileRegs<T, T, 16, U> t;
        for (int grp = 0; grp < ngroups; ++grp) {
            LaneMat<T, T, 1> ch[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k0 = 16 * (grp * U + u);
                const int kc = k - k0 < 16 ? k - k0 : 16;   // <= 0: chunk past k, nothing loaded
                ch[u] = blk;
                ch[u].k = kc > 0 ? kc : 0;
                if (!a0 && kc > 0) {
                    // op(A) rows row0.., k-indices k0..: A[i + lda l] (N) or A[l + lda i] (T, C)
                    ch[u].A = in_space<1>(ACONT ? Ab + k0 + (int64_t)row0 * a.lda : Ab + row0 + (int64_t)k0 * a.lda);
                    // op(B) k-indices k0.., columns col0..: B[l + ldb j] (N) or B[j + ldb l] (T, C)
                    ch[u].B = in_space<1>(BCONT ? Bb + k0 + (int64_t)col0 * a.ldb : Bb + col0 + (int64_t)k0 * a.ldb);
                }
            }
            // C with the first group only; its registers stay live to the epilogue
            tile_load<T, T, 16, U, ACONT, BCONT, 1, false>(ch, L, a0, b0 || grp > 0, t);
#pragma unroll
            for (int u = 0; u < U; ++u)
                tile_mma<T, T, 0, 16, 1>(ch[u], L, !a0, a.a_conj, a.b_conj, t.va[u], t.vb[u], acc_r, acc_i);
        }
        tile_store<T, T, 16, 1>(blk, L, alpha, beta, a0, b0, acc_r, acc_i, t.cin[0]);
    }
}

// ---- LDS-staged variant (real types, m, n, k <= 64) -------------------------
//
// The register kernel above re-reads a matrix's A block-row and B
// block-column once per output block; from n = 24 on, a quarter or more of
// those re-reads miss L2 and come from HBM again (rocprofv3 counters: 1.02x
// to 1.41x the algorithmic bytes), and with a k-contiguous op(A) (op T or C)
// each of its 16-byte loads spans 16 rows.  Here a work-group of 4 waves
// owns one matrix at a time (persistent over the batch):
//  1. the stored A and B (A: m x k for op N, k x m for op T; B likewise) are
//     copied into LDS column by column as 16-byte chunks ALIGNED in global
//     memory -- chunk q of column j starts at the 16-byte boundary at or below
//     the column's start, plus 16 q, so every chunk holds a byte of its
//     column and an aligned chunk never crosses a page: no load can fault,
//     and the bytes outside the column are never used.  With leading
//     dimensions whose byte size is a multiple of 16 every column has the
//     same offset within its first chunk, so element (i, j) sits at
//     offset + i s + j pitch in LDS: a uniform leading dimension for the
//     tile routine.  The pitch is an odd multiple of 16 bytes, so the 16
//     rows a k-contiguous operand's lanes read fall in distinct LDS banks;
//  2. each wave computes output blocks wave, wave + 4, ...: C's block comes
//     straight from HBM, op(A) and op(B) chunks from LDS through the same
//     tile loads and MFMA steps as the register kernel (so both kernels give
//     the same bits);
//  3. a barrier, then the next matrix overwrites the images.
// A and B are read from HBM once per matrix.  The host takes this kernel
// where it measured faster than the register kernel: when both A and B are
// reused (at least two block-rows and two block-columns) and the largest size
// reaches 32, or 48 for 4-byte types whose op(A) is not k-contiguous.

typedef unsigned int blk_u4 __attribute__((ext_vector_type(4)));

struct BlkLds {
    int rowsA, colsA, rowsB, colsB;   // stored shapes
    int pitchA, pitchB;               // LDS bytes per stored column
    int offB;                         // LDS byte offset of B's image
};

template <typename T, int U, bool ACONT, bool BCONT, bool PTR>
__global__ __launch_bounds__(256) void gemm_blocked_lds_kernel(const GemmArgs<T> a, const BlkLds g)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char blk_smem[];
    using R = typename Tr<T>::R;
    using acc_t = typename Mfma<R>::acc_t;
    constexpr int S = (int)sizeof(T);
    constexpr int CHL = 5;                          // chunks of each operand per thread per copy pass
    using G4 = __attribute__((address_space(1))) const blk_u4*;
    using L4 = __attribute__((address_space(3))) blk_u4*;
    const LaneGeom<16, R> L;
    T alpha, beta;
    alpha = a.alpha_dev ? *a.alpha_dev : a.alpha;
    beta = a.beta_dev ? *a.beta_dev : a.beta;
    const bool a0 = is_zero(alpha), b0 = is_zero(beta);

    const int m = a.m, n = a.n, k = a.k;
    const bool skipAB = a0 || k == 0;               // A and B are not read
    const int nbm = (m + 15) >> 4, nbn = (n + 15) >> 4;
    const int nbb = nbm * nbn;
    const int wave = threadIdx.x >> 6;
    const int64_t ldab = a.lda * S, ldbb = a.ldb * S;
    const int64_t lla = g.pitchA / S, llb = g.pitchB / S;

    for (int64_t p = blockIdx.x; p < a.batch; p += gridDim.x) {
        const T* Ab = nullptr;
        const T* Bb = nullptr;
        T* Cb;
        if (PTR) {
            if (!skipAB) {
                Ab = static_cast<const T*>(a.Aarr[p]);
                Bb = static_cast<const T*>(a.Barr[p]);
            }
            Cb = a.Carr[p];
        } else {
            if (!skipAB) {
                Ab = static_cast<const T*>(a.A) + p * a.strideA;
                Bb = static_cast<const T*>(a.B) + p * a.strideB;
            }
            Cb = a.C + p * a.strideC;
        }
        const uintptr_t ga = reinterpret_cast<uintptr_t>(Ab), gb = reinterpret_cast<uintptr_t>(Bb);
        const int offA = (int)(ga & 15), offB = (int)(gb & 15);

        // 1. A and B into LDS: thread t copies chunks t, t + 256, ... of each
        // operand's list (chunk i = column i / nq, chunk i % nq of it), A's and
        // B's in flight together; the (column, chunk) pair advances by the
        // constant step 256 = dj nq + dq, so no division per chunk
        if (!skipAB) {
            const int nqA = (offA + g.rowsA * S + 15) >> 4, nqB = (offB + g.rowsB * S + 15) >> 4;
            const int totA = g.colsA * nqA, totB = g.colsB * nqB;
            const int tot = totA > totB ? totA : totB;
            const uintptr_t a16 = ga & ~(uintptr_t)15, b16 = gb & ~(uintptr_t)15;
            const int tid = (int)threadIdx.x;
            int jA = tid / nqA, qA = tid - jA * nqA;
            int jB = tid / nqB, qB = tid - jB * nqB;
            const int djA = 256 / nqA, dqA = 256 - djA * nqA;
            const int djB = 256 / nqB, dqB = 256 - djB * nqB;
            for (int base = 0; base < tot; base += 256 * CHL) {
                blk_u4 ra[CHL], rb[CHL];
                int da[CHL], db[CHL];
#pragma unroll
                for (int c = 0; c < CHL; ++c) {
                    const int idx = base + tid + 256 * c;
                    const bool okA = idx < totA, okB = idx < totB;
                    // a slot past its list reads chunk 0 of its operand (holds its first element)
                    const uintptr_t sa = okA ? a16 + jA * ldab + 16 * qA : a16;
                    const uintptr_t sb = okB ? b16 + jB * ldbb + 16 * qB : b16;
                    da[c] = okA ? jA * g.pitchA + 16 * qA : -1;
                    db[c] = okB ? g.offB + jB * g.pitchB + 16 * qB : -1;
                    ra[c] = *(G4)sa;
                    rb[c] = *(G4)sb;
                    qA += dqA;
                    jA += djA;
                    if (qA >= nqA) {
                        qA -= nqA;
                        ++jA;
                    }
                    qB += dqB;
                    jB += djB;
                    if (qB >= nqB) {
                        qB -= nqB;
                        ++jB;
                    }
                }
#pragma unroll
                for (int c = 0; c < CHL; ++c) {
                    if (da[c] >= 0) *(L4)(blk_smem + da[c]) = ra[c];
                    if (db[c] >= 0) *(L4)(blk_smem + db[c]) = rb[c];
                }
            }
        }
        __syncthreads();

        // 2. the wave's output blocks
        const T* lA = reinterpret_cast<const T*>(blk_smem + offA);
        const T* lB = reinterpret_cast<const T*>(blk_smem + g.offB + offB);
        for (int b = wave; b < nbb; b += 4) {
            const int bj = b / nbm, bi = b - bj * nbm;
            const int row0 = 16 * bi, col0 = 16 * bj;
            const int mb = m - row0 < 16 ? m - row0 : 16;
            const int nb = n - col0 < 16 ? n - col0 : 16;
            LaneMat<T, T, 1> cm[1];
            cm[0].A = nullptr;
            cm[0].B = nullptr;
            cm[0].C = in_space<1>(Cb + row0 + (int64_t)col0 * a.ldc);
            cm[0].m = mb;
            cm[0].n = nb;
            cm[0].k = 0;
            cm[0].lda = cm[0].ldb = 0;
            cm[0].ldc = a.ldc;
            cm[0].scale = 1.0f;
            cm[0].valid = true;
            cm[0].overA = cm[0].overB = cm[0].overC = false;
            TileRegs<T, T, 16, 1> tc;
            tile_load<T, T, 16, 1, ACONT, BCONT, 1, false>(cm, L, true, b0, tc);

            LaneMat<T, T, 3> ch[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k0 = 16 * u;
                const int kc = k - k0 < 16 ? k - k0 : 16;
                ch[u].m = mb;
                ch[u].n = nb;
                ch[u].k = kc > 0 ? kc : 0;
                ch[u].lda = lla;
                ch[u].ldb = llb;
                ch[u].ldc = 0;
                ch[u].scale = 1.0f;
                ch[u].valid = true;
                ch[u].overA = ch[u].overB = ch[u].overC = false;
                ch[u].C = in_space<3>(reinterpret_cast<T*>(blk_smem));   // not read (C comes from HBM)
                ch[u].A = in_space<3>(kc > 0 ? (ACONT ? lA + k0 + row0 * lla : lA + row0 + k0 * lla) : lA);
                ch[u].B = in_space<3>(kc > 0 ? (BCONT ? lB + k0 + col0 * llb : lB + col0 + k0 * llb) : lB);
            }
            TileRegs<T, T, 16, U> t;
            tile_load<T, T, 16, U, ACONT, BCONT, 3, false>(ch, L, skipAB, true, t);
            acc_t acc_r = {0, 0, 0, 0};
            acc_t acc_i = {0, 0, 0, 0};
#pragma unroll
            for (int u = 0; u < U; ++u)
                tile_mma<T, T, 0, 16, 3>(ch[u], L, !skipAB, a.a_conj, a.b_conj, t.va[u], t.vb[u], acc_r, acc_i);
            tile_store<T, T, 16, 1>(cm[0], L, alpha, beta, a0, b0, acc_r, acc_i, tc.cin[0]);
        }
        // 3. every wave is done with the images before the next matrix
        __syncthreads();
    }
}

// Bytes per stored column of an LDS image: room for the chunks of a column
// at any offset, rounded to an odd multiple of 16.
inline int blk_pitch(int rows, int s)
{
    int p = ((rows * s + 30) / 16) * 16;
    if (((p / 16) & 1) == 0) p += 16;
    return p;
}

constexpr int kBlkLdsMax = 96 * 1024;

// The LDS images of a call, or 0 when the LDS-staged kernel does not apply:
// complex types, a size above 64, k = 0, a leading dimension of A or B
// whose byte size is not a multiple of 16, images above kBlkLdsMax, or a
// shape where it measured slower than the register kernel (A or B not
// reused across blocks; sizes below 32; 4-byte types with op(A) N or R
// below 48).
template <typename T>
inline int blocked_lds_plan(const GemmArgs<T>& a, BlkLds& g)
{
    if constexpr (Tr<T>::cplx) {
        return 0;
    } else {
        constexpr int S = (int)sizeof(T);
        if (tuning().blocked == 1) return 0;
        if (a.m > 64 || a.n > 64 || a.k > 64 || a.k < 1) return 0;
        if ((a.lda * S) % 16 || (a.ldb * S) % 16) return 0;
        if (tuning().blocked != 2) {
            const int mx = a.m > a.n ? (a.m > a.k ? a.m : a.k) : (a.n > a.k ? a.n : a.k);
            if (a.m <= 16 || a.n <= 16) return 0;
            if (!a.a_trans && mx < (S == 4 ? 48 : 32)) return 0;
            if (a.a_trans && mx < 32) return 0;
        }
        g.rowsA = a.a_trans ? a.k : a.m;
        g.colsA = a.a_trans ? a.m : a.k;
        g.rowsB = a.b_trans ? a.n : a.k;
        g.colsB = a.b_trans ? a.k : a.n;
        g.pitchA = blk_pitch(g.rowsA, S);
        g.pitchB = blk_pitch(g.rowsB, S);
        g.offB = g.colsA * g.pitchA;
        const int bytes = g.offB + g.colsB * g.pitchB;
        return bytes <= kBlkLdsMax ? bytes : 0;
    }
}

template <typename T, int U, bool PTR>
hipError_t launch_blocked_lds_u(GemmArgs<T> a, const BlkLds& g, int bytes, hipStream_t stream)
{
    const bool at = a.a_trans, bn = !a.b_trans;
    auto kern = at ? (bn ? gemm_blocked_lds_kernel<T, U, true, true, PTR> : gemm_blocked_lds_kernel<T, U, true, false, PTR>)
                   : (bn ? gemm_blocked_lds_kernel<T, U, false, true, PTR>
                         : gemm_blocked_lds_kernel<T, U, false, false, PTR>);
    if (bytes > 64 * 1024) {
        // raised once per kernel and device to the largest image size any call needs
        static std::mutex mu;
        static std::map<std::pair<const void*, int>, bool> raised;
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) dev = -1;
        std::lock_guard<std::mutex> lock(mu);
        bool& done = raised[{reinterpret_cast<const void*>(kern), dev}];
        if (!done) {
            const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, kBlkLdsMax);
            if (e != hipSuccess) return e;
            done = true;
        }
    }
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, bytes) != hipSuccess || per_cu < 1)
        per_cu = 1;
    const Tuning& tu = tuning();
    const int want = tu.wg_per_cu > 0 ? tu.wg_per_cu : 4;
    if (per_cu > want) per_cu = want;
    const int64_t cap = tu.grid > 0 ? (int64_t)tu.grid : (int64_t)device_cu_count() * per_cu;
    const int64_t grid = a.batch < cap ? a.batch : cap;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(256), bytes, stream, a, g);
    return hipGetLastError();
}

// Chunks per group: 4 for real types, 2 for complex (register budget), fewer
// when k has fewer chunks.
template <typename T>
inline int blocked_unroll(int k)
{
    const int nkc = (k + 15) / 16;
    const int cap = Tr<T>::cplx ? 2 : 4;
    return nkc <= 1 ? 1 : (nkc <= 2 || cap == 2 ? 2 : 4);
}

template <typename T, int U, bool PTR>
hipError_t launch_blocked_u(GemmArgs<T> a, hipStream_t stream)
{
    const bool at = a.a_trans, bn = !a.b_trans;
    auto kern = at ? (bn ? gemm_blocked_kernel<T, U, true, true, PTR> : gemm_blocked_kernel<T, U, true, false, PTR>)
                   : (bn ? gemm_blocked_kernel<T, U, false, true, PTR> : gemm_blocked_kernel<T, U, false, false, PTR>);
    const int64_t units = a.batch * (int64_t)((a.m + 15) / 16) * ((a.n + 15) / 16);
    // 32 work-groups per CU, more than can be resident (measured: n = 24 f32 NN 0.38 -> 0.44, f64 0.45 ->
    // 0.50 of HBM peak against the persistent default of 4; equal at n = 32); the knob still overrides
    if (tuning().wg_per_cu == 0) a.plan_wg = 32;
    const int64_t grid = persistent_grid(kern, units, a);
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(256), 0, stream, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_blocked(GemmArgs<T> a, bool pointer_form, hipStream_t stream)
{
    const int u = blocked_unroll<T>(a.k);
    BlkLds g;
    if (const int bytes = blocked_lds_plan<T>(a, g)) {
        if constexpr (!Tr<T>::cplx) {
            if (pointer_form) {
                if (u == 1) return launch_blocked_lds_u<T, 1, true>(a, g, bytes, stream);
                if (u == 2) return launch_blocked_lds_u<T, 2, true>(a, g, bytes, stream);
                return launch_blocked_lds_u<T, 4, true>(a, g, bytes, stream);
            }
            if (u == 1) return launch_blocked_lds_u<T, 1, false>(a, g, bytes, stream);
            if (u == 2) return launch_blocked_lds_u<T, 2, false>(a, g, bytes, stream);
            return launch_blocked_lds_u<T, 4, false>(a, g, bytes, stream);
        }
    }
    if (pointer_form) {
        if (u == 1) return launch_blocked_u<T, 1, true>(a, stream);
        if (u == 2) return launch_blocked_u<T, 2, true>(a, stream);
        if constexpr (!Tr<T>::cplx) return launch_blocked_u<T, 4, true>(a, stream);
    } else {
        if (u == 1) return launch_blocked_u<T, 1, false>(a, stream);
        if (u == 2) return launch_blocked_u<T, 2, false>(a, stream);
        if constexpr (!Tr<T>::cplx) return launch_blocked_u<T, 4, false>(a, stream);
    }
    return hipErrorInvalidValue;
}

template <typename T>
int describe_blocked(const GemmArgs<T>& a, bool pointer_form, char* buf, int len)
{
    const auto tf = [](bool b) { return b ? "true" : "false"; };
    const int U = blocked_unroll<T>(a.k);
    BlkLds g;
    if (blocked_lds_plan<T>(a, g))
        return snprintf(buf, len, "void sbg::gemm_blocked_lds_kernel<%s, %d, %s, %s, %s>(sbg::GemmArgs<%s>, sbg::BlkLds)",
                        TypeName<T>::s, U, tf(a.a_trans), tf(!a.b_trans), tf(pointer_form), TypeName<T>::s);
    return snprintf(buf, len, "void sbg::gemm_blocked_kernel<%s, %d, %s, %s, %s>(sbg::GemmArgs<%s>)", TypeName<T>::s,
                    U, tf(a.a_trans), tf(!a.b_trans), tf(pointer_form), TypeName<T>::s);
}

}  // namespace sbg
