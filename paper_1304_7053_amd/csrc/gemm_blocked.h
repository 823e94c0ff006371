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
    const int64_t grid = persistent_grid(kern, units, a);
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(256), 0, stream, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_blocked(GemmArgs<T> a, bool pointer_form, hipStream_t stream)
{
    const int u = blocked_unroll<T>(a.k);
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

}  // namespace sbg
