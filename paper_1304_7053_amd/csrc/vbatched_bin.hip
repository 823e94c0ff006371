// Device-side size binning of a variable-size batch (see gemm_vbatched.h).
#include "gemm_vbatched.h"

namespace sbg {

size_t vb_workspace_bytes(int64_t batch) { return vbatched_workspace_bytes(batch); }

__global__ void vb_zero_kernel(int* ws)
{
    if (threadIdx.x < VB_HEADER) ws[threadIdx.x] = 0;
}

__global__ __launch_bounds__(256) void vb_bin_kernel(const int* dm, const int* dn, const int* dk, const int* dlda,
                                                     const int* dldb, const int* dldc, int max_m, int max_n,
                                                     int max_k, bool a_trans, bool b_trans, int64_t batch,
                                                     int* ws)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int lane = threadIdx.x & 63;
    int cls = -1;
    bool bad = false;
    if (p < batch) {
        const int m = dm[p], n = dn[p], k = dk[p];
        const int rowsA = a_trans ? k : m;
        const int rowsB = b_trans ? n : k;
        bad = m < 0 || n < 0 || k < 0 || m > max_m || n > max_n || k > max_k ||
              dlda[p] < (rowsA > 1 ? rowsA : 1) || dldb[p] < (rowsB > 1 ? rowsB : 1) ||
              dldc[p] < (m > 1 ? m : 1);
        if (!bad && m > 0 && n > 0) {
            const int D = size_class(m, n, k);
            cls = D == 4 ? 0 : (D == 8 ? 1 : 2);
        }
    }
    // one atomic per wave and class; lanes take consecutive slots
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const unsigned long long mask = __ballot(cls == c);
        if (mask == 0) continue;
        const int leader = __ffsll((long long)mask) - 1;
        int base = 0;
        if (lane == leader) base = atomicAdd(&ws[c], __popcll(mask));
        base = __shfl(base, leader);
        if (cls == c) ws[VB_HEADER + (int64_t)c * batch + base + __popcll(mask & below)] = (int)p;
    }
    const unsigned long long badm = __ballot(bad);
    if (badm && lane == __ffsll((long long)badm) - 1) atomicAdd(&ws[3], __popcll(badm));
}

}  // namespace sbg
