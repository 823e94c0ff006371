// Variable-size batched GEMM: every matrix p has its own (m_p, n_p, k_p) and
// leading dimensions, all <= 16, in one call.
//
// The paper handles unequal sizes by grouping the matrices into sets of
// identical size and calling the uniform routine per set (Sec. 1).  Here the
// grouping happens on the device and the whole batch is one persistent
// launch, so the sequence can be captured once in a HIP graph and replayed
// with no host round trip:
//   1. zero_kernel    clears the four counters of the caller's workspace
//                     (a kernel, not a memset node, so graph replays are safe);
//   2. bin_kernel     classifies every matrix by size class D in {4, 8, 16}
//                     (max of m, n, k) and appends a record of it -- its
//                     three pointers, leading dimensions, packed sizes and
//                     fp8 scale product -- to that class's list, with one
//                     atomic per work-group and class (records keep their
//                     order within a work-group); matrices whose sizes or
//                     leading dimensions are invalid are counted and skipped
//                     (C untouched);
//   3. vbatched_kernel walks the tiles of the three lists (largest class
//                     first) with the same tile routine as the uniform forms;
//                     each lane reads its own matrix's record, one contiguous
//                     48-byte load, so operands are one dependent step away.
// Workspace (16-byte aligned): int32 words [0..2] class counts, [3] rejected
// matrices; from byte 64 the three record lists of capacity N each.
#pragma once

#include "gemm_direct.h"

namespace sbg {

constexpr int VB_HEADER_BYTES = 64;
constexpr int VB_BIN_PER = 2;        // matrices per thread of the binning kernel
constexpr int VB_BIN_THREADS = 1024;  // threads per work-group of the binning kernel

// One binned matrix.
struct alignas(16) VbRec {
    const void* A;
    const void* B;
    void* C;
    int lda, ldb, ldc;
    int mnk;      // m | n << 8 | k << 16
    float scale;  // sA * sB for scaled fp8 inputs, 1 otherwise
    int pad;
};
static_assert(sizeof(VbRec) == 48, "record layout");

constexpr size_t vbatched_workspace_bytes(int64_t batch)
{
    return (size_t)VB_HEADER_BYTES + 3 * (size_t)(batch > 0 ? batch : 0) * sizeof(VbRec);
}

__device__ __host__ inline const VbRec* vb_list(const int* ws, int64_t batch, int c)
{
    return reinterpret_cast<const VbRec*>(reinterpret_cast<const unsigned char*>(ws) + VB_HEADER_BYTES) +
           (int64_t)c * batch;
}

__global__ void vb_zero_kernel(int* ws);
__global__ __launch_bounds__(VB_BIN_THREADS) void vb_bin_kernel(const int* dm, const int* dn, const int* dk, const int* dlda,
                                                     const int* dldb, const int* dldc, const void* const* Aarr,
                                                     const void* const* Barr, void* const* Carr,
                                                     const float* scaleA, const float* scaleB, int max_m,
                                                     int max_n, int max_k, bool a_trans, bool b_trans,
                                                     int64_t batch, int* ws);

template <typename T, typename TI, int MODE, int D, bool ACONT, bool BCONT>
__device__ __forceinline__ void vb_process(const GemmArgs<T>& a, int64_t grp, int count, const VbRec* list,
                                           const T& alpha, const T& beta, bool a0, bool b0)
{
    using R = typename Tr<T>::R;
    constexpr int P = 16 / D;
    constexpr int U = Unroll<T, D>::value;
    const LaneGeom<D, R> L;
    LaneMat<T, TI, 1> mats[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t li = (grp * U + u) * P + L.sel;
        LaneMat<T, TI, 1>& mt = mats[u];
        mt.valid = li < count;
        // lanes past the list carry its last matrix (loads in bounds, nothing stored)
        const VbRec r = list[mt.valid ? li : count - 1];
        mt.m = r.mnk & 0xFF;
        mt.n = (r.mnk >> 8) & 0xFF;
        mt.k = (r.mnk >> 16) & 0xFF;
        mt.lda = r.lda;
        mt.ldb = r.ldb;
        mt.ldc = r.ldc;
        mt.A = nullptr;
        mt.B = nullptr;
        if (!a0) {
            mt.A = in_space<1>(static_cast<const TI*>(r.A));
            mt.B = in_space<1>(static_cast<const TI*>(r.B));
        }
        mt.C = in_space<1>(static_cast<T*>(r.C));
        mt.scale = r.scale;
        mt.overA = mt.overB = mt.overC = false;   // each matrix may be its own allocation
    }
    tile_group<T, TI, MODE, D, U, ACONT, BCONT>(mats, L, alpha, beta, a0, b0, a.a_conj, a.b_conj);
}

template <typename T, typename TI, int MODE, bool ACONT, bool BCONT>
__global__ __launch_bounds__(256) void gemm_vbatched_kernel(const GemmArgs<T> a)
{
    T alpha, beta;
    load_scalars(a, alpha, beta);
    const bool a0 = is_zero(alpha), b0 = is_zero(beta);
    const int c4 = a.ws[0], c8 = a.ws[1], c16 = a.ws[2];
    const VbRec* l4 = vb_list(a.ws, a.batch, 0);
    const VbRec* l8 = vb_list(a.ws, a.batch, 1);
    const VbRec* l16 = vb_list(a.ws, a.batch, 2);
    constexpr int U4 = Unroll<T, 4>::value, U8 = Unroll<T, 8>::value, U16 = Unroll<T, 16>::value;
    const int64_t g16 = (c16 + U16 - 1) / U16;
    const int64_t g8 = ((c8 + 1) / 2 + U8 - 1) / U8;
    const int64_t g4 = ((c4 + 3) / 4 + U4 - 1) / U4;
    const int64_t total = g16 + g8 + g4;
    const int64_t W = (int64_t)gridDim.x * 4;
    for (int64_t grp = xcd_wave_index(a.xcd_chunk); grp < total; grp += W) {
        if (grp < g16)
            vb_process<T, TI, MODE, 16, ACONT, BCONT>(a, grp, c16, l16, alpha, beta, a0, b0);
        else if (grp < g16 + g8)
            vb_process<T, TI, MODE, 8, ACONT, BCONT>(a, grp - g16, c8, l8, alpha, beta, a0, b0);
        else
            vb_process<T, TI, MODE, 4, ACONT, BCONT>(a, grp - g16 - g8, c4, l4, alpha, beta, a0, b0);
    }
}

template <typename T, typename TI, int MODE, bool ACONT, bool BCONT>
hipError_t launch_vb_variant(GemmArgs<T> a, hipStream_t stream)
{
    if (VbDescribe& ds = vb_describe(); ds.buf) {
        // the class counts are only known on the device: units is the upper
        // bound (every matrix in the 16 class); the lists are walked 16, 8, 4
        const auto tf = [](bool b) { return b ? "true" : "false"; };
        auto kern = gemm_vbatched_kernel<T, TI, MODE, ACONT, BCONT>;
        const int64_t units = (a.batch + Unroll<T, 16>::value - 1) / Unroll<T, 16>::value;
        const int64_t grid = persistent_grid(kern, units, a);
        snprintf(ds.buf, ds.len,
                 "kernel=void sbg::gemm_vbatched_kernel<%s, %s, %d, %s, %s>(sbg::GemmArgs<%s>) grid=%lld units=%lld "
                 "u16=%d u8=%d u4=%d",
                 TypeName<T>::s, TypeName<TI>::s, MODE, tf(ACONT), tf(BCONT), TypeName<T>::s, (long long)grid,
                 (long long)units, Unroll<T, 16>::value, Unroll<T, 8>::value, Unroll<T, 4>::value);
        return hipSuccess;
    }
    hipLaunchKernelGGL(vb_zero_kernel, dim3(1), dim3(64), 0, stream, a.ws);
    const int64_t nb = (a.batch + VB_BIN_THREADS * VB_BIN_PER - 1) / (VB_BIN_THREADS * VB_BIN_PER);
    hipLaunchKernelGGL(vb_bin_kernel, dim3((unsigned)nb), dim3(VB_BIN_THREADS), 0, stream, a.dm, a.dn, a.dk, a.dlda, a.dldb,
                       a.dldc, a.Aarr, a.Barr, reinterpret_cast<void* const*>(a.Carr), a.scaleA, a.scaleB,
                       a.max_m, a.max_n, a.max_k, a.a_trans, a.b_trans, a.batch, a.ws);
    auto kern = gemm_vbatched_kernel<T, TI, MODE, ACONT, BCONT>;
    // the class counts are only known on the device: size the grid for the
    // case with the most work units (every matrix in the 16 class)
    const int64_t units = (a.batch + Unroll<T, 16>::value - 1) / Unroll<T, 16>::value;
    const int64_t grid = persistent_grid(kern, units, a);
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(256), 0, stream, a);
    return hipGetLastError();
}

template <typename T, typename TI>
hipError_t launch_vbteam(const GemmArgs<T>& a, hipStream_t stream);

template <typename T, typename TI, int MODE>
hipError_t launch_vbatched_t(const GemmArgs<T>& a, hipStream_t stream)
{
    // real types in plain mode: one team of lanes per matrix (gemm_vbteam.h);
    // complex types, BF16x3 and the `path` knob set to 1: the MFMA tiles
    if constexpr (MODE == 0 && !Tr<T>::cplx)
        if (tuning().path != 1) return launch_vbteam<T, TI>(a, stream);
    const bool at = a.a_trans, bn = !a.b_trans;
    if (at) {
        if (bn) return launch_vb_variant<T, TI, MODE, true, true>(a, stream);
        return launch_vb_variant<T, TI, MODE, true, false>(a, stream);
    }
    if (bn) return launch_vb_variant<T, TI, MODE, false, true>(a, stream);
    return launch_vb_variant<T, TI, MODE, false, false>(a, stream);
}

}  // namespace sbg
