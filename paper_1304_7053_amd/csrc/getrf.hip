// Batched LU factorisation with partial pivoting (LAPACK GETRF semantics) of
// small square matrices (n <= 32), a strided batch.  The paper proposes
// carrying its batched interface over to other batched BLAS / LAPACK kernels
// (Sec. 9); this is the first of them beside GEMV and TRSM.
//
// One team of D lanes per matrix (D = 4, 8, 16 or 32 >= n; 64 / D
// matrices per wave), ROW per lane: lane t holds row t of the matrix in
// registers for the whole factorisation, so no row is ever moved.  Step k:
//   1. the eligible rows (not yet pivots) offer |a_t[k]|; a team reduction
//      (shuffles) picks the largest, the lowest current position on ties --
//      LAPACK's choice, which takes the first maximum of the interchanged
//      matrix;
//   2. the pivot row is broadcast to the team through the team's LDS slot;
//   3. every other eligible row forms its multiplier a_t[k] / pivot (an
//      IEEE division; unscaled when the pivot is zero) and updates
//      a_t[j] -= l_t u_j for j > k (FMA);
//   4. the interchange is book-keeping only: each row tracks its current
//      position (the pivot row takes position k, the row that was there
//      takes the pivot's old position), which is ipiv[k].
// At the end each row is stored at its final position: the factors land in
// the interchanged order, exactly as GETRF leaves them.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "sbg_internal.h"

namespace sbg {

namespace {

// The team's pivot candidate: largest magnitude v, then lowest current
// position cur; lane is where it lives.  Ineligible lanes offer v = -1.
template <typename T, int D>
__device__ __forceinline__ void team_argmax(T& v, int& cur, int& lane)
{
#pragma unroll
    for (int off = D / 2; off >= 1; off >>= 1) {
        const T w = __shfl_xor(v, off);
        const int wc = __shfl_xor(cur, off);
        const int wl = __shfl_xor(lane, off);
        if (w > v || (w == v && wc < cur)) {
            v = w;
            cur = wc;
            lane = wl;
        }
    }
}

template <typename T, int D>
__global__ __launch_bounds__(256) void getrf_kernel(const GetrfArgs<T> g)
{
    constexpr int TPW = 64 / D;
    __shared__ __attribute__((aligned(16))) T lds[4 * 64];
    const int lane = threadIdx.x & 63;
    const int team = lane / D, t = lane - team * D;
    T* slot = lds + (threadIdx.x >> 6) * 64 + team * D;
    const int64_t p0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * TPW + team;
    if ((p0 - team) >= g.batch) return;   // the whole wave is past the batch
    const bool live = p0 < g.batch;
    const int64_t p = live ? p0 : g.batch - 1;
    const int n = g.n;
    const T* A = g.A + p * g.strideA;

    // row t (columns past n repeat the last one; rows past n read row n - 1:
    // every load stays inside the matrix)
    const int trow = t < n ? t : (n > 0 ? n - 1 : 0);
    T a[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const int jc = j < n ? j : (n > 0 ? n - 1 : 0);
        a[j] = n > 0 ? A[trow + (int64_t)jc * g.lda] : T(0);
    }

    const bool mine = t < n;   // this lane holds a row of the matrix
    int cur = t;               // current position of the row
    int ipiv = t;              // lane t: the interchange of step t
    int info = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        if (k >= n) continue;   // n is uniform; the loop keeps its constant trip count (fully unrolled)
        // 1. pivot choice among the rows at positions >= k
        const bool elig = mine && cur >= k;
        T v = elig ? T(__builtin_fabs(a[k])) : T(-1);
        int pcur = elig ? cur : 0x7FFFFFFF, plane = lane;
        team_argmax<T, D>(v, pcur, plane);
        const bool upd = elig && lane != plane;   // rows that take a multiplier
        // 2. the pivot row to every lane of the team, 3. multipliers and
        // the trailing update (the pivot row itself is not changed in step k)
        if (lane == plane) {
#pragma unroll
            for (int j = 0; j < D; ++j)
                if (j >= k) slot[j] = a[j];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const T piv = slot[k];
        T l = T(0);
        if (upd) l = piv != T(0) ? a[k] / piv : a[k];
#pragma unroll
        for (int j = 0; j < D; ++j) {
            if (j > k) {
                const T uj = slot[j];
                if (upd) a[j] = __builtin_fma(-l, uj, a[j]);
            }
        }
        // the slot is rewritten in the next step only after every lane read it
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (upd) a[k] = l;
        if (piv == T(0) && info == 0) info = k + 1;
        // 4. positions: the pivot row takes position k, the row there moves
        if (t == k) ipiv = pcur;
        if (mine) {
            if (lane == plane) cur = k;
            else if (cur == k) cur = pcur;
        }
    }

    if (live) {
        if (mine) {
            T* Aw = g.A + p * g.strideA;
#pragma unroll
            for (int j = 0; j < D; ++j)
                if (j < n) Aw[cur + (int64_t)j * g.lda] = a[j];
            g.ipiv[p * g.strideP + t] = ipiv + 1;
        }
        if (t == 0) g.info[p] = info;
    }
}

template <typename T, int D>
hipError_t launch_getrf_d(const GetrfArgs<T>& g, hipStream_t stream)
{
    const int64_t waves = (g.batch + 64 / D - 1) / (64 / D);
    const int64_t grid = (waves + 3) / 4;
    hipLaunchKernelGGL((getrf_kernel<T, D>), dim3((unsigned)grid), dim3(256), 0, stream, g);
    return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_getrf(const GetrfArgs<T>& g, hipStream_t stream)
{
    if (g.batch <= 0) return hipSuccess;
    if (g.n <= 4) return launch_getrf_d<T, 4>(g, stream);
    if (g.n <= 8) return launch_getrf_d<T, 8>(g, stream);
    if (g.n <= 16) return launch_getrf_d<T, 16>(g, stream);
    return launch_getrf_d<T, 32>(g, stream);
}

template hipError_t launch_getrf<float>(const GetrfArgs<float>&, hipStream_t);
template hipError_t launch_getrf<double>(const GetrfArgs<double>&, hipStream_t);

}  // namespace sbg
