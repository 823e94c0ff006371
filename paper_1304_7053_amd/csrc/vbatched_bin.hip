// Device-side size binning of a variable-size batch (see gemm_vbatched.h).
#include "gemm_vbatched.h"

namespace sbg {

size_t vb_workspace_bytes(int64_t batch) { return vbatched_workspace_bytes(batch); }

__global__ void vb_zero_kernel(int* ws)
{
    if (threadIdx.x < VB_HEADER_BYTES / 4) ws[threadIdx.x] = 0;
}

// One work-group bins VB_BIN_PER * 256 consecutive matrices: per-wave ballots
// count each class, the counts are prefix-summed in LDS (in matrix order),
// and one global atomic per class and work-group reserves the group's range
// of each list.  Within a work-group the lists keep the matrices' order.
// Pointer arrays A and B may be null (alpha == 0 with host scalars: never
// dereferenced); scales may be null (unscaled inputs).
__global__ __launch_bounds__(256) void vb_bin_kernel(const int* dm, const int* dn, const int* dk, const int* dlda,
                                                     const int* dldb, const int* dldc, const void* const* Aarr,
                                                     const void* const* Barr, void* const* Carr,
                                                     const float* scaleA, const float* scaleB, int max_m,
                                                     int max_n, int max_k, bool a_trans, bool b_trans,
                                                     int64_t batch, int* ws)
{
    __shared__ int cnt[VB_BIN_PER][4][4];   // [step][wave][class 0..2, invalid 3] -> exclusive prefix
    __shared__ int base[4];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t p0 = (int64_t)blockIdx.x * (256 * VB_BIN_PER);
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int cls[VB_BIN_PER];
    VbRec rec[VB_BIN_PER];
    unsigned long long rank[VB_BIN_PER];   // this lane's position among its wave's lanes of the same class
#pragma unroll
    for (int it = 0; it < VB_BIN_PER; ++it) {
        const int64_t p = p0 + it * 256 + tid;
        int c = -1;
        bool bad = false;
        if (p < batch) {
            const int m = dm[p], n = dn[p], k = dk[p];
            const int lda = dlda[p], ldb = dldb[p], ldc = dldc[p];
            const int rowsA = a_trans ? k : m;
            const int rowsB = b_trans ? n : k;
            bad = m < 0 || n < 0 || k < 0 || m > max_m || n > max_n || k > max_k ||
                  lda < (rowsA > 1 ? rowsA : 1) || ldb < (rowsB > 1 ? rowsB : 1) || ldc < (m > 1 ? m : 1);
            if (!bad && m > 0 && n > 0) {
                const int D = size_class(m, n, k);
                c = D == 4 ? 0 : (D == 8 ? 1 : 2);
                VbRec& r = rec[it];
                r.A = Aarr ? Aarr[p] : nullptr;
                r.B = Barr ? Barr[p] : nullptr;
                r.C = Carr[p];
                r.lda = lda;
                r.ldb = ldb;
                r.ldc = ldc;
                r.mnk = m | (n << 8) | (k << 16);
                r.scale = scaleA ? scaleA[p] * scaleB[p] : 1.0f;
                r.pad = 0;
            }
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
            for (int ww = 0; ww < 4; ++ww) {
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
            VbRec* list = const_cast<VbRec*>(vb_list(ws, batch, c));
            list[base[c] + cnt[it][w][c] + (int)rank[it]] = rec[it];
        }
    }
}

}  // namespace sbg
