// Internal declarations shared by the C-ABI layer (api.cpp) and the kernel
// translation units.  Not installed; the public interface is include/sbg.h.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "sbg.h"

namespace sbg {

// Batched-GEMM launch description after host-side decoding of the op
// characters (Sec. 2) and the storage rule of Sec. 5.
//   op(A)(i, l) = A_p[i + lda * l]  (a_trans: A_p[l + lda * i]), conjugated when a_conj < 0
//   op(B)(l, j) = B_p[l + ldb * j]  (b_trans: B_p[j + ldb * l]), conjugated when b_conj < 0
//   C_p(i, j)   = C_p[i + ldc * j]
// The strided form locates matrix p at base + stride * p; the pointer-array
// form reads Xarr[p].  Scalars come by value (host mode) or through the
// *_dev pointers (device mode, read by the kernel).
template <typename T>
struct GemmArgs {
    int m, n, k;
    int64_t lda, ldb, ldc;
    bool a_trans, b_trans;
    int64_t strideA, strideB, strideC;
    const T* A;
    const T* B;
    T* C;
    const T* const* Aarr;
    const T* const* Barr;
    T* const* Carr;
    T alpha, beta;
    const T* alpha_dev;
    const T* beta_dev;
    float a_conj, b_conj;
    int64_t batch;
    int64_t xcd_chunk;   // consecutive tile groups per XCD run (set by the launcher)
    int G;               // matrices per wave step of the LDS-staged kernel
};

// Launch-shape knobs: work-groups per CU of the persistent grid, the XCD run
// length and whether packed batches take the LDS-staged kernel.  Defaults
// are the tuned values; SBG_WG_PER_CU, SBG_XCD_CHUNK and SBG_STAGED override
// them (read once per process) for tuning sweeps and A/B comparisons.
struct Tuning {
    int wg_per_cu;
    int xcd_chunk;
    bool staged;   // use the LDS-staged kernel for packed strided batches
};
const Tuning& tuning();

template <typename T>
hipError_t launch_gemm(const GemmArgs<T>& a, bool pointer_form, hipStream_t stream);

template <typename T>
int describe_gemm(const GemmArgs<T>& a, bool pointer_form, char* buf, int len);

int device_cu_count();

}  // namespace sbg
