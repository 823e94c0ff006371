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
    const void* A;                 // stored type of A and B may be narrower than T
    const void* B;
    T* C;
    const void* const* Aarr;
    const void* const* Barr;
    T* const* Carr;
    T alpha, beta;
    const T* alpha_dev;
    const T* beta_dev;
    float a_conj, b_conj;
    const float* scaleA;           // per-matrix operand scales (fp8 inputs) or null
    const float* scaleB;
    int64_t batch;
    int64_t xcd_chunk;             // consecutive work units per XCD run (set by the launcher)
    int64_t blocks;                // work-groups with work in a one-shot grid (set by the launcher)
    int plan_wg, plan_xcd;         // launch shape chosen for this call (0: the tuning knobs' defaults)
    int plan_unroll;               // tiles per wave step of the direct kernel (0: from the byte budgets)
    int G;                         // matrices per wave step of the LDS-staged kernel
    // variable-size form: per-matrix sizes and leading dimensions, workspace
    const int* dm;
    const int* dn;
    const int* dk;
    const int* dlda;
    const int* dldb;
    const int* dldc;
    int max_m, max_n, max_k;
    int* ws;
};

// Launch-shape and kernel-choice knobs.  A value of 0 (2 for `staged`) means
// automatic: the entry of the tuned table for the call when one is loaded,
// else the built-in rule or default (4 work-groups per CU, XCD runs of 16,
// tile unroll from the byte budgets).  Non-automatic values, set through
// sbg_set_tuning or the SBG_* environment variables (read once per process),
// override the table -- for tuning sweeps and A/B comparisons.
struct Tuning {
    int wg_per_cu;     // persistent grids: work-groups per CU (0: 4, capped by occupancy; set: as given)
    int xcd_chunk;     // consecutive work units per XCD run
    int staged;        // 0 never, 1 every packed strided batch, 2 automatic
    int tile_bytes;    // per-wave bytes in flight per step, size classes 4 and 8
    int tile_bytes16;  // the same for size class 16, per 4-byte element size (scaled by sizeof(T) / 4)
    bool pipeline;     // issue the next group's loads before computing the current one
    int path;          // 0 automatic, 1 MFMA tile kernels only, 2 team kernel for sizes <= 8, 3 also for the
                       // real types up to 16
    int unroll;        // tiles per wave step of the direct kernel (a power of two, capped per class)
    int grid;          // work-groups of a persistent grid (rounded up to a multiple of 8)
    int table;         // 1: use the tuned table when one is loaded
    int blocked;       // sizes above 16 (real types): 0 automatic (the LDS-staged kernel where it measured
                       // faster), 1 the register kernel only, 2 the LDS-staged kernel wherever it applies
};
const Tuning& tuning();
Tuning& tuning_mut();

// One entry of the tuned table (kernel choice and launch shape measured for a
// type, batch form, op pair and size), read from the versioned JSON file the
// autotuner writes.  path: 1 MFMA tile kernel, 2 team kernel, 3 LDS-staged
// kernel; 0 fields mean "no preference".
struct TunedEntry {
    int path, unroll, wg_per_cu, xcd_chunk;
};
// Entry for type code (0 S, 1 D, 2 C, 3 Z), form (pointer arrays or strided),
// transposed op(A) / op(B) and size max(m, n, k) in 1..16, or null.
const TunedEntry* tuned_entry(int type, bool pointer_form, bool a_trans, bool b_trans, int size);
// "file=... version=... entries=..." into buf; returns the entry count.
int tuned_table_info(char* buf, int len);

// Compute units of the current device, cached per device.
int device_cu_count();
// Resident 256-thread work-groups per CU of a kernel, cached per kernel.
int resident_blocks_per_cu(const void* kernel);

template <typename T>
hipError_t launch_gemm(const GemmArgs<T>& a, bool pointer_form, hipStream_t stream);

template <typename T>
int describe_gemm(const GemmArgs<T>& a, bool pointer_form, char* buf, int len);

// Describe mode of the variable-size launchers (thread-local, set by
// sbg_describe_vbatched): while buf is non-null a launcher writes the kernel
// it would launch, its grid and its work units into buf and launches nothing.
struct VbDescribe {
    char* buf = nullptr;
    int len = 0;
};
VbDescribe& vb_describe();

// Variable-size form (per-matrix sizes in a.dm .. a.dldc, workspace a.ws of
// vb_workspace_bytes(batch) bytes).
template <typename T>
hipError_t launch_vbatched(const GemmArgs<T>& a, hipStream_t stream);
size_t vb_workspace_bytes(int64_t batch);

// The library's device scratch for the allocation-free variable-size entry
// point (room for the workspace of SBG_NOALLOC_MAX_BATCH matrices): its
// device address on the current device (looked up once per device) and size.
hipError_t noalloc_scratch(void** ptr, size_t* bytes);

// Mixed precision on binary32 C: ab_type 0 f32, 1 bf16, 2 f16, 3 e4m3;
// mode 0 plain, 1 BF16x3 (ab_type 0 only); form 0 strided, 1 pointer, 2 var-size.
hipError_t launch_gemm_ex(const GemmArgs<float>& a, int ab_type, int mode, int form, hipStream_t stream);

// Per-matrix absmax E4M3 quantisation: uniform (rows, cols, X, ldx, strideX,
// Q, ldq, strideQ) or variable-size (drows .. dldq, max_rows, max_cols) batch.
struct QuantArgs {
    int rows, cols;
    const float* X;
    int64_t ldx, strideX;
    unsigned char* Q;
    int64_t ldq, strideQ;
    const int* drows;
    const int* dcols;
    const float* const* Xarr;
    unsigned char* const* Qarr;
    const int* dldx;
    const int* dldq;
    int max_rows, max_cols;
    float* scales;
    int64_t batch;
};

hipError_t launch_quant_e4m3(const QuantArgs& q, bool var, hipStream_t stream);

// Small triangular solves (size <= 16) of a strided batch, one 16-lane row
// of a wave per matrix: element e of vector v of matrix p is
// B[strideB p + vec_step v + vec_elem e]; the triangular matrix M acts on
// those vectors, M(i, l) = A_p[l + lda i] when eff_trans, else A_p[i + lda l],
// conjugated when conj; lower selects forward substitution; unit takes the
// diagonal as ones.  Solves M x = alpha b in place for every vector.
template <typename T>
struct TrsmArgs {
    int size;                     // order of M (<= 16)
    int64_t nv;                   // vectors per matrix
    bool lower, eff_trans, conj, unit;
    const T* A;
    int64_t lda, strideA;
    T* B;
    int64_t vec_elem, vec_step, strideB;
    int64_t batch;
    T alpha;
    const T* alpha_dev;           // device scalar, or null for `alpha`
};

template <typename T>
hipError_t launch_trsm_small(const TrsmArgs<T>& a, hipStream_t stream);

// Batched LU with partial pivoting of n x n matrices (n <= 64), a strided
// batch: A_p at A + strideA p (column-major, lda), factors in place,
// interchanges ipiv[strideP p + k] (1-based) and info[p] (0, or the 1-based
// index of the first zero pivot).
template <typename T>
struct GetrfArgs {
    int n;
    T* A;
    int64_t lda, strideA;
    int* ipiv;
    int64_t strideP;
    int* info;
    int64_t batch;
};

template <typename T>
hipError_t launch_getrf(const GetrfArgs<T>& g, hipStream_t stream);

}  // namespace sbg
