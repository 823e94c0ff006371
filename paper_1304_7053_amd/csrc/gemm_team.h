// Batched GEMM for small matrices (size classes 4 and 8, and 16 for the real
// types): one team of lanes per matrix, one lane per column.
//
// The operation is memory-bound at these sizes (at most 2 flops per byte), so
// the design is about moving each matrix's bytes in as few, as wide and as
// early loads as possible (the paper's Sec. 7 kernels use thread teams per
// matrix for the same reason):
//
//  * A team of TS = max(n, k) consecutive lanes owns one matrix; a wave holds
//    floor(64 / TS) matrices.  Lane t of a team loads column t of op(A)
//    (m values, t < k), column t of op(B) (k values, t < n) and column t of C
//    (m values, t < n), keeps C's column in registers and produces it.
//  * Columns stored contiguously (op N/R on A or B, and C) load as 16-byte
//    vectors: the whole vectors of the column and, when its length is not a
//    multiple of the vector, the vector ending at the column's last element
//    (overlapping the previous one); the lane then shifts those elements into
//    place after the data has arrived.  No load leaves the column.  Columns
//    shorter than one vector, and transposed operands (whose column runs
//    across neighbouring lanes of the team instead), load element by element.
//  * Every load of a lane is issued before any is consumed: load addresses are
//    selected, never branched around, and one empty asm statement makes the
//    loaded A and B registers live before the compute, so the compiler
//    neither waits between the operands nor sinks a load into a branch.
//  * C(:, t) = sum_l op(A)(:, l) op(B)(l, t): op(A)'s columns are spread over
//    the team, so each lane writes its column to LDS once and every lane reads
//    column l back as broadcast 16-byte reads (one read per 16 bytes of the
//    column for all lanes of the team) -- no per-entry shuffles.  The k loop
//    is a switch on k with fully unrolled cases (registers stay statically
//    indexed; no branch inside a case).
//  * Stores mirror the loads (whole vectors plus the overlapping last one).
//  * The grid is one wave per floor(64 / TS) matrices (no persistence: every
//    wave issues all its loads at once), with work-groups renumbered so that
//    each XCD takes one contiguous range of the batch.
#pragma once

#include "gemm_direct.h"

namespace sbg {

// c + a b in the working precision (complex: four real FMAs).
template <typename T> __device__ __forceinline__ T team_fma(const T& a, const T& b, const T& c);
template <> __device__ __forceinline__ float team_fma<float>(const float& a, const float& b, const float& c)
{
    return __builtin_fmaf(a, b, c);
}
template <> __device__ __forceinline__ double team_fma<double>(const double& a, const double& b, const double& c)
{
    return __builtin_fma(a, b, c);
}
template <> __device__ __forceinline__ float2 team_fma<float2>(const float2& a, const float2& b, const float2& c)
{
    return make_float2(__builtin_fmaf(a.x, b.x, __builtin_fmaf(-a.y, b.y, c.x)),
                       __builtin_fmaf(a.x, b.y, __builtin_fmaf(a.y, b.x, c.y)));
}
template <> __device__ __forceinline__ double2 team_fma<double2>(const double2& a, const double2& b, const double2& c)
{
    return make_double2(__builtin_fma(a.x, b.x, __builtin_fma(-a.y, b.y, c.x)),
                        __builtin_fma(a.x, b.y, __builtin_fma(a.y, b.x, c.y)));
}

template <typename T> __device__ __forceinline__ T conj_val(const T& v) { return v; }
template <> __device__ __forceinline__ float2 conj_val<float2>(const float2& v) { return make_float2(v.x, -v.y); }
template <> __device__ __forceinline__ double2 conj_val<double2>(const double2& v) { return make_double2(v.x, -v.y); }

template <typename T> __device__ __forceinline__ T zero_val() { return make_val<T>(0, 0); }

// Empty asm reading v: the value must be available here (its load waited
// for), and a load feeding it cannot be moved past this point.
__device__ __forceinline__ void keep_live(float v) { __asm__ volatile("" ::"v"(v)); }
__device__ __forceinline__ void keep_live(double v) { __asm__ volatile("" ::"v"(v)); }
__device__ __forceinline__ void keep_live(float2 v) { __asm__ volatile("" ::"v"(v.x), "v"(v.y)); }
__device__ __forceinline__ void keep_live(double2 v) { __asm__ volatile("" ::"v"(v.x), "v"(v.y)); }

// Elements per 16-byte vector.


// Issue the loads of a contiguous column of `len` (1..MX) elements at p.
// VEC: whole 16-byte vectors plus the vector ending at element len - 1
// (requires len >= V); otherwise one load per element.  Slots past the
// column re-read a valid part of it.  Nothing here waits for the data.
template <typename T, int MX, bool VEC, typename P>
__device__ __forceinline__ void col_issue(T (&x)[MX], P p, int len)
{
    constexpr int V = TeamVec<T>::V;
    if (VEC) {
#pragma unroll
        for (int v = 0; v < MX / V; ++v) {
            const int off = (V * v + V <= len) ? V * v : len - V;
            vload<T, V>(*reinterpret_cast<T(*)[V]>(&x[V * v]), p + off);
        }
    } else {
#pragma unroll
        for (int e = 0; e < MX; ++e) x[e] = ld1<T>(p + (e < len ? e : 0));
    }
}

// Element e < len of the column from the raw registers of col_issue (the
// last vector of a VEC column holds elements len - V .. len - 1); zero past
// len.
template <typename T, int MX, bool VEC>
__device__ __forceinline__ void col_fix(T (&d)[MX], const T (&x)[MX], int len)
{
    constexpr int V = TeamVec<T>::V;
    if (!VEC || V == 1) {
#pragma unroll
        for (int e = 0; e < MX; ++e) d[e] = e < len ? x[e] : zero_val<T>();
        return;
    }
    const int rem = len % V, sh = V - rem;
#pragma unroll
    for (int v = 0; v < MX / V; ++v) {
        const bool full = V * v + V <= len;
        const bool part = !full && V * v < len;
#pragma unroll
        for (int r = 0; r < V; ++r) {
            // the tail vector's element r + sh is column element V v + r
            T t = x[V * v + V - 1];
#pragma unroll
            for (int j = V - 2; j >= 0; --j) t = (r + sh == j) ? x[V * v + j] : t;
            d[V * v + r] = full ? x[V * v + r] : ((part && r < rem) ? t : zero_val<T>());
        }
    }
}

// Store elements 0 .. len-1 of o to the contiguous column at p (VEC: whole
// vectors plus the vector ending at len - 1, rewriting the overlap with the
// same values).
template <typename T, int MX, bool VEC, typename P>
__device__ __forceinline__ void col_store(P p, const T (&o)[MX], int len)
{
    constexpr int V = TeamVec<T>::V;
    if (!VEC) {
#pragma unroll
        for (int e = 0; e < MX; ++e)
            if (e < len) st1<T>(p + e, o[e]);
        return;
    }
#pragma unroll
    for (int v = 0; v < MX / V; ++v) {
        if (V * v + V <= len) {
            vstore<T, V>(p + V * v, *reinterpret_cast<const T(*)[V]>(&o[V * v]));
        } else if (V > 1 && V * v < len) {
            T w[V];
#pragma unroll
            for (int r = 0; r < V; ++r) {
                T t = o[0];
#pragma unroll
                for (int e = 1; e < MX; ++e) t = (e == len - V + r) ? o[e] : t;
                w[r] = t;
            }
            vstore<T, V>(p + (len - V), w);
        }
    }
}

// The work-group of a one-shot grid (gridDim.x a multiple of 8) after
// renumbering: dispatch sends work-group b to XCD b % 8, and XCD x takes the
// contiguous range of logical work-groups [x G/8, (x+1) G/8).
__device__ __forceinline__ int64_t xcd_block_index()
{
    const int64_t per = gridDim.x >> 3;
    return (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
}

// D: size class (4, 8, or 16 for the real types; bounds m, n, k); AC / BC: op(A) / op(B) is N or R
// (a stored column is a column of the operand) rather than T or C (a stored
// column is a row of the operand); VEC: every column a lane loads or stores
// holds at least one 16-byte vector (loaded as vectors), else element by
// element; PTR: pointer-array form.
//
// Every lane loads one stored column of A, of B and of C (contiguous in
// memory whatever the op).  The operands then reach the layout of the
// product through the wave's LDS slice: op(A)'s column l of the team sits in
// the slot of the team's lane l (written as a vector when the lane holds that
// column, element by element when it holds a row), and for op T/C on B each
// lane reads its column of op(B) back element by element from the rows the
// team wrote.
template <typename T, int D, bool AC, bool BC, bool VEC, bool PTR>
__global__ __launch_bounds__(256) void gemm_team_kernel(const GemmArgs<T> a)
{
    __shared__ __attribute__((aligned(16))) T lds[(BC ? 1 : 2) * 4 * 64 * D];
    const int64_t blk = xcd_block_index();
    if (blk >= a.blocks) return;
    T alpha, beta;
    load_scalars(a, alpha, beta);
    const int m = a.m, n = a.n, k = a.k;
    // k == 0 or alpha == 0: A and B are never read
    const bool skip_ab = is_zero(alpha) || k == 0;
    const bool b0 = is_zero(beta);
    const int TS = team_size(m, n, k, !AC);
    const int TPW = 64 / TS;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int team = lane / TS, t = lane - team * TS;
    const bool act = team < TPW;
    const int64_t p = (blk * 4 + wave) * TPW + team;
    const bool ok = act && p < a.batch;
    const int64_t pe = ok ? p : a.batch - 1;   // lanes past the batch read the last matrix
    const int base = (act ? team : 0) * TS;
    // the stored columns this lane loads, and their lengths
    const int la = AC ? m : k, na = AC ? k : m;
    const int lb = BC ? k : n, nb = BC ? n : k;
    const int ta = t < na ? t : 0, tb = t < nb ? t : 0, tc = t < n ? t : 0;

    using GT = typename SpacePtr<const T, 1>::type;
    using GTw = typename SpacePtr<T, 1>::type;
    GT A0;
    GT B0;
    GTw C0;
    if (PTR) {
        A0 = skip_ab ? nullptr : in_space<1>(static_cast<const T*>(a.Aarr[pe]));
        B0 = skip_ab ? nullptr : in_space<1>(static_cast<const T*>(a.Barr[pe]));
        C0 = in_space<1>(a.Carr[pe]);
    } else {
        A0 = in_space<1>(static_cast<const T*>(a.A) + pe * a.strideA);
        B0 = in_space<1>(static_cast<const T*>(a.B) + pe * a.strideB);
        C0 = in_space<1>(a.C + pe * a.strideC);
    }
    const GTw ccol = C0 + (int64_t)tc * a.ldc;

    T xa[D], xb[D], xc[D];
    if (!skip_ab) {
        col_issue<T, D, VEC>(xa, A0 + (int64_t)ta * a.lda, la);
        col_issue<T, D, VEC>(xb, B0 + (int64_t)tb * a.ldb, lb);
    }
    if (!b0) col_issue<T, D, VEC>(xc, ccol, m);

    T acc[D];
#pragma unroll
    for (int i = 0; i < D; ++i) acc[i] = zero_val<T>();
    if (!skip_ab) {
        // every load is in flight: make A and B live here (one wait, for the
        // data the compute needs next) so that no load sinks into the switch
#pragma unroll
        for (int e = 0; e < D; ++e) {
            keep_live(xa[e]);
            keep_live(xb[e]);
        }
        T ra[D], rb[D];
        col_fix<T, D, VEC>(ra, xa, la);
        col_fix<T, D, VEC>(rb, xb, lb);
        if (a.a_conj < 0) {
#pragma unroll
            for (int e = 0; e < D; ++e) ra[e] = conj_val(ra[e]);
        }
        if (a.b_conj < 0) {
#pragma unroll
            for (int e = 0; e < D; ++e) rb[e] = conj_val(rb[e]);
        }
        // op(A) column l of the team -> slot base + l of this wave's slice
        T* wl = lds + wave * 64 * D;
        if (AC) {
            vstore<T, D>(wl + lane * D, ra);
        } else if (act && t < m) {
#pragma unroll
            for (int l = 0; l < D; ++l)
                if (l < k) wl[(base + l) * D + t] = ra[l];
        }
        T* bl = lds + (4 + wave) * 64 * D;
        if (!BC) vstore<T, D>(bl + lane * D, rb);   // row t of op(B)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        T cb[D];
        if (BC) {
#pragma unroll
            for (int l = 0; l < D; ++l) cb[l] = rb[l];
        } else {
#pragma unroll
            for (int l = 0; l < D; ++l) cb[l] = bl[(base + (l < k ? l : 0)) * D + t];
        }
        const T* tcol = wl + base * D;
#define SBG_TEAM_CASE(KK)                                                        \
    case KK:                                                                     \
        _Pragma("unroll") for (int l = 0; l < KK; ++l) {                         \
            T av[D];                                                             \
            vload<T, D>(av, tcol + l * D);                                       \
            _Pragma("unroll") for (int i = 0; i < D; ++i) acc[i] = team_fma<T>(av[i], cb[l], acc[i]); \
        }                                                                        \
        break;
        switch (k) {
            SBG_TEAM_CASE(1)
            SBG_TEAM_CASE(2)
            SBG_TEAM_CASE(3)
            SBG_TEAM_CASE(4)
            default:
                if constexpr (D >= 8) {
                    switch (k) {
                        SBG_TEAM_CASE(5)
                        SBG_TEAM_CASE(6)
                        SBG_TEAM_CASE(7)
                        SBG_TEAM_CASE(8)
                        default:
                            if constexpr (D == 16) {
                                switch (k) {
                                    SBG_TEAM_CASE(9)
                                    SBG_TEAM_CASE(10)
                                    SBG_TEAM_CASE(11)
                                    SBG_TEAM_CASE(12)
                                    SBG_TEAM_CASE(13)
                                    SBG_TEAM_CASE(14)
                                    SBG_TEAM_CASE(15)
                                    SBG_TEAM_CASE(16)
                                    default: break;
                                }
                            }
                            break;
                    }
                }
                break;
        }
#undef SBG_TEAM_CASE
    }
    T cc[D];
    if (!b0) col_fix<T, D, VEC>(cc, xc, m);
    else {
#pragma unroll
        for (int e = 0; e < D; ++e) cc[e] = zero_val<T>();
    }
    // epilogue for every lane (stores only for the lanes that own a column)
    using R = typename Tr<T>::R;
    const R ar = re_of<T>(alpha), ai = im_of<T>(alpha), br = re_of<T>(beta), bi = im_of<T>(beta);
    const bool a0 = is_zero(alpha);
    T out[D];
#pragma unroll
    for (int i = 0; i < D; ++i)
        out[i] = axpby<T>(ar, ai, br, bi, a0, b0, re_of<T>(acc[i]), im_of<T>(acc[i]), cc[i]);
    if (ok && t < n) col_store<T, D, VEC>(ccol, out, m);
}

// Launch: one wave per floor(64 / team size) matrices, 4 waves per
// work-group, work-groups rounded up to a multiple of 8 for the XCD
// renumbering.
template <typename T, int D, bool AC, bool BC, bool VEC, bool PTR>
hipError_t launch_team_v(GemmArgs<T> a, hipStream_t stream)
{
    const int64_t tpw = 64 / team_size(a.m, a.n, a.k, !AC);
    const int64_t waves = (a.batch + tpw - 1) / tpw;
    const int64_t blocks = (waves + 3) / 4;
    const int64_t grid = (blocks + 7) / 8 * 8;
    if (grid > 0x7FFFFFF8LL) return hipErrorInvalidValue;
    a.blocks = blocks;
    hipLaunchKernelGGL((gemm_team_kernel<T, D, AC, BC, VEC, PTR>), dim3((unsigned)grid), dim3(256), 0, stream, a);
    return hipGetLastError();
}

template <typename T, int D, bool AC, bool BC, bool PTR>
hipError_t launch_team_modes(const GemmArgs<T>& a, hipStream_t stream)
{
    if (team_vec(a)) return launch_team_v<T, D, AC, BC, true, PTR>(a, stream);
    return launch_team_v<T, D, AC, BC, false, PTR>(a, stream);
}

template <typename T, int D, bool PTR>
hipError_t launch_team_ops(const GemmArgs<T>& a, hipStream_t stream)
{
    const bool ac = !a.a_trans, bc = !a.b_trans;
    if (ac) return bc ? launch_team_modes<T, D, true, true, PTR>(a, stream)
                      : launch_team_modes<T, D, true, false, PTR>(a, stream);
    return bc ? launch_team_modes<T, D, false, true, PTR>(a, stream)
              : launch_team_modes<T, D, false, false, PTR>(a, stream);
}

// Entry from the strided / pointer-array dispatch (sizes <= 8, and <= 16 for
// the real types).
template <typename T>
hipError_t launch_team(const GemmArgs<T>& a, bool pointer_form, hipStream_t stream)
{
    const int D = size_class(a.m, a.n, a.k);
    if (D == 16) {
        if constexpr (!Tr<T>::cplx) {
            return pointer_form ? launch_team_ops<T, 16, true>(a, stream) : launch_team_ops<T, 16, false>(a, stream);
        }
        return hipErrorInvalidValue;
    }
    if (pointer_form) return D == 4 ? launch_team_ops<T, 4, true>(a, stream) : launch_team_ops<T, 8, true>(a, stream);
    return D == 4 ? launch_team_ops<T, 4, false>(a, stream) : launch_team_ops<T, 8, false>(a, stream);
}

}  // namespace sbg
