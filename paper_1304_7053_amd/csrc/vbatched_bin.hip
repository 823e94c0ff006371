// Device-side size binning of a variable-size batch (see gemm_vbatched.h).
#include "gemm_vbatched.h"

namespace sbg {

size_t vb_workspace_bytes(int64_t batch) { return vbatched_workspace_bytes(batch); }

__global__ void vb_zero_kernel(int* ws)
{
    if (threadIdx.x < VB_HEADER_BYTES / 4) ws[threadIdx.x] = 0;
}

// One work-group of VB_BIN_THREADS threads bins VB_BIN_PER * VB_BIN_THREADS
// consecutive matrices (work-groups this large keep the number of global
// atomics, which serialise per counter, small).  Every load of a thread's
// matrices (sizes, leading dimensions, pointers, scales) is issued before any
// is used: a thread past the batch re-reads the last matrix and drops it, and
// a null pointer or scale array is read at a valid address with the value
// replaced.  Per-wave ballots count each class, the counts are prefix-summed
// in LDS (in matrix order) and one global atomic per class and work-group
// reserves the group's range of each list.  Within a work-group the lists
// keep the matrices' order.  Pointer arrays A and B may be null (alpha == 0
// with host scalars: never dereferenced); scales may be null (unscaled
// inputs).
__global__ __launch_bounds__(VB_BIN_THREADS) void vb_bin_kernel(
    const int* dm, const int* dn, const int* dk, const int* dlda, const int* dldb, const int* dldc,
    const void* const* Aarr, const void* const* Barr, void* const* Carr, const float* scaleA, const float* scaleB,
    int max_m, int max_n, int max_k, bool a_trans, bool b_trans, int64_t batch, int* ws)
{
    constexpr int NW = VB_BIN_THREADS / 64;
    __shared__ int cnt[VB_BIN_PER][NW][4];   // [step][wave][class 0..2, invalid 3] -> exclusive prefix
    __shared__ int base[4];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t p0 = (int64_t)blockIdx.x * (VB_BIN_THREADS * VB_BIN_PER) + tid;

    int m[VB_BIN_PER], n[VB_BIN_PER], k[VB_BIN_PER], lda[VB_BIN_PER], ldb[VB_BIN_PER], ldc[VB_BIN_PER];
    const void* A[VB_BIN_PER];
    const void* B[VB_BIN_PER];
    void* C[VB_BIN_PER];
    float sa[VB_BIN_PER], sb[VB_BIN_PER];
#pragma unroll
    for (int it = 0; it < VB_BIN_PER; ++it) {
        const int64_t p = p0 + it * VB_BIN_THREADS;
        const int64_t q = p < batch ? p : batch - 1;
        m[it] = dm[q];
        n[it] = dn[q];
        k[it] = dk[q];
        lda[it] = dlda[q];
        ldb[it] = dldb[q];
        ldc[it] = dldc[q];
        A[it] = *(Aarr ? Aarr + q : const_cast<const void* const*>(Carr) + q);
        B[it] = *(Barr ? Barr + q : const_cast<const void* const*>(Carr) + q);
        C[it] = Carr[q];
        sa[it] = *(scaleA ? scaleA + q : reinterpret_cast<const float*>(dm + q));
        sb[it] = *(scaleB ? scaleB + q : reinterpret_cast<const float*>(dm + q));
    }
    int cls[VB_BIN_PER], rank[VB_BIN_PER];
#pragma unroll
    for (int it = 0; it < VB_BIN_PER; ++it) {
        const bool in = p0 + it * VB_BIN_THREADS < batch;
        const int rowsA = a_trans ? k[it] : m[it];
        const int rowsB = b_trans ? n[it] : k[it];
        const bool bad = in && (m[it] < 0 || n[it] < 0 || k[it] < 0 || m[it] > max_m || n[it] > max_n ||
                                k[it] > max_k || lda[it] < (rowsA > 1 ? rowsA : 1) ||
                                ldb[it] < (rowsB > 1 ? rowsB : 1) || ldc[it] < (m[it] > 1 ? m[it] : 1));
        int c = -1;
        if (in && !bad && m[it] > 0 && n[it] > 0) {
            const int D = size_class(m[it], n[it], k[it]);
            c = D == 4 ? 0 : (D == 8 ? 1 : 2);
        }
        cls[it] = c;
        rank[it] = 0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const unsigned long long mask = __ballot(c == j);
            if (c == j) rank[it] = __popcll(mask & below);
            if (lane == 0) cnt[it][w][j] = __popcll(mask);
        }
        const unsigned long long badm = __ballot(bad);
        if (lane == 0) cnt[it][w][3] = __popcll(badm);
    }
    __syncthreads();
    if (tid < 4) {
        int run = 0;
        for (int it = 0; it < VB_BIN_PER; ++it)
            for (int ww = 0; ww < NW; ++ww) {
                const int x = cnt[it][ww][tid];
                cnt[it][ww][tid] = run;
                run += x;
            }
        base[tid] = run ? atomicAdd(&ws[tid], run) : 0;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < VB_BIN_PER; ++it) {
        const int c = cls[it];
        if (c >= 0) {
            VbRec r;
            r.A = Aarr ? A[it] : nullptr;
            r.B = Barr ? B[it] : nullptr;
            r.C = C[it];
            r.lda = lda[it];
            r.ldb = ldb[it];
            r.ldc = ldc[it];
            r.mnk = m[it] | (n[it] << 8) | (k[it] << 16);
            r.scale = scaleA ? sa[it] * sb[it] : 1.0f;
            r.pad = 0;
            VbRec* list = const_cast<VbRec*>(vb_list(ws, batch, c));
            list[base[c] + cnt[it][w][c] + rank[it]] = r;
        }
    }
}

}  // namespace sbg
