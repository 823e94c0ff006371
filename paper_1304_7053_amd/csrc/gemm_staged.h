// Batched small-matrix GEMM for PACKED strided batches (lda = rows of A,
// strideA = rows * cols, likewise for B and C -- the minimal leading
// dimensions of the paper's experiments, Sec. 8), staged through LDS.
//
// In a packed batch any run of consecutive matrices is one contiguous span of
// each operand.  A wave therefore moves G matrices per step as three flat
// streams:
//   1. HBM -> registers -> LDS: every lane copies 16-byte chunks of the A, B
//      (and, when beta != 0, C) spans; consecutive lanes take consecutive
//      chunks, so each load instruction reads 1 KB of contiguous memory
//      whatever m, n, k are (no per-size coalescing problem, no masks but
//      the span ends);
//   2. LDS -> MFMA operand registers: the same block-diagonal packing as the
//      direct kernel (16/D matrices of size class D per 16x16x16 product),
//      gathered from LDS with the op folded into the addressing;
//   3. results are written back into the C span in LDS and leave as one
//      contiguous, fully written span of 16-byte stores.
// G is chosen on the host so that the three spans fill the wave's LDS slice;
// small matrices thus move as many bytes per step as large ones.  Each wave
// owns its LDS slice: no work-group barriers, only wave-level ordering.
#pragma once

#include "gemm_direct.h"

namespace sbg {

template <typename T> struct StagedCfg {
    static constexpr int LDSW = sizeof(T) >= 16 ? 16384 : 8192;  // LDS bytes per wave
    static constexpr int MAXCH = LDSW / 1024;                     // 16-B chunks per lane
};

__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int align16(int x) { return (x + 15) & ~15; }

template <typename T, int D, bool ACONT, bool BCONT>
__global__ __launch_bounds__(256) void gemm_staged_kernel(const GemmArgs<T> a)
{
    using R = typename Tr<T>::R;
    using M = Mfma<R>;
    using acc_t = typename M::acc_t;
    using u32x4 = unsigned int __attribute__((ext_vector_type(4)));
    constexpr bool CPLX = Tr<T>::cplx;
    constexpr int P = 16 / D;
    constexpr int KB = D / 4;
    constexpr int LDSW = StagedCfg<T>::LDSW;
    constexpr int MAXCH = StagedCfg<T>::MAXCH;
    constexpr int ESZ = (int)sizeof(T);

    __shared__ __attribute__((aligned(16))) unsigned char lds_all[4 * LDSW];
    unsigned char* lds = lds_all + (threadIdx.x >> 6) * LDSW;

    const int lane = threadIdx.x & 63;
    const int g = lane >> 4;
    const int c = lane & 15;
    const int sel = c / D;
    const int ij = c % D;
    const int kk0 = KB * g;

    const T alpha = a.alpha_dev ? *a.alpha_dev : a.alpha;
    const T beta = a.beta_dev ? *a.beta_dev : a.beta;
    const bool a0 = is_zero(alpha);
    const bool b0 = is_zero(beta);
    const R ar_ = re_of<T>(alpha), ai_ = im_of<T>(alpha);
    const R br_ = re_of<T>(beta), bi_ = im_of<T>(beta);

    const int m = a.m, n = a.n, k = a.k;
    const int eA = m * k, eB = k * n, eC = m * n;   // elements per matrix
    const int G = a.G;
    const int offB = align16(G * eA * ESZ);
    const int offC = offB + align16(G * eB * ESZ);
    const bool row_ok = ij < m;
    const bool col_ok = ij < n;

    bool keep[4];
    int orow[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int Rr = M::row(g, r);
        keep[r] = (Rr / D) == sel && (Rr % D) < m && col_ok;
        orow[r] = Rr % D;
    }

    const int64_t W = (int64_t)gridDim.x * 4;
    const int64_t q0 = xcd_wave_index(a.xcd_chunk);
    const int64_t nsteps = (a.batch + G - 1) / G;

    // One run = G consecutive matrices; its spans and their chunk counts.
    struct Run {
        int cnt, bytesA, bytesB, bytesC, bytesCin, FA, FB, FC;
        const unsigned char* gA;
        const unsigned char* gB;
        unsigned char* gC;
    };
    auto make_run = [&](int64_t step) {
        Run r;
        const int64_t p0 = step * G;
        r.cnt = (int)((a.batch - p0) < G ? (a.batch - p0) : G);
        if (r.cnt < 0) r.cnt = 0;
        r.gA = reinterpret_cast<const unsigned char*>(static_cast<const T*>(a.A) + p0 * eA);
        r.gB = reinterpret_cast<const unsigned char*>(static_cast<const T*>(a.B) + p0 * eB);
        r.gC = reinterpret_cast<unsigned char*>(a.C + p0 * eC);
        r.bytesA = a0 ? 0 : r.cnt * eA * ESZ;
        r.bytesB = a0 ? 0 : r.cnt * eB * ESZ;
        r.bytesC = r.cnt * eC * ESZ;
        r.bytesCin = b0 ? 0 : r.bytesC;
        r.FA = r.bytesA >> 4;
        r.FB = r.bytesB >> 4;
        r.FC = r.bytesCin >> 4;
        return r;
    };

    u32x4 buf[MAXCH];
    unsigned int tail = 0;
    int tail_off = -1;

    // HBM -> registers: 16-byte chunks of the A, B, C spans (lane-consecutive),
    // then the < 16-byte span tails (lanes 0-3 A, 4-7 B, 8-11 C).
    auto issue_loads = [&](const Run& r) {
#pragma unroll
        for (int t = 0; t < MAXCH; ++t) {
            const int qq = lane + 64 * t;
            const unsigned char* src;
            if (qq < r.FA) src = r.gA + 16 * qq;
            else if (qq < r.FA + r.FB) src = r.gB + 16 * (qq - r.FA);
            else src = r.gC + 16 * (qq - r.FA - r.FB);
            if (qq < r.FA + r.FB + r.FC)
                __builtin_memcpy(&buf[t], reinterpret_cast<const unsigned int*>(src), 16);
        }
        tail_off = -1;
        const int which = lane >> 2, w = lane & 3;
        if (which < 3) {
            const int bytes = which == 0 ? r.bytesA : (which == 1 ? r.bytesB : r.bytesCin);
            const int F = bytes >> 4;
            const int tw = (bytes & 15) >> 2;
            if (w < tw) {
                const unsigned char* base = which == 0 ? r.gA : (which == 1 ? r.gB : r.gC);
                tail = reinterpret_cast<const unsigned int*>(base + 16 * F)[w];
                tail_off = (which == 0 ? 0 : (which == 1 ? offB : offC)) + 16 * F + 4 * w;
            }
        }
    };
    // registers -> this wave's LDS slice
    auto commit = [&](const Run& r) {
#pragma unroll
        for (int t = 0; t < MAXCH; ++t) {
            const int qq = lane + 64 * t;
            int dst;
            if (qq < r.FA) dst = 16 * qq;
            else if (qq < r.FA + r.FB) dst = offB + 16 * (qq - r.FA);
            else dst = offC + 16 * (qq - r.FA - r.FB);
            if (qq < r.FA + r.FB + r.FC) *reinterpret_cast<u32x4*>(lds + dst) = buf[t];
        }
        if (tail_off >= 0) *reinterpret_cast<unsigned int*>(lds + tail_off) = tail;
    };

    const T* lA = reinterpret_cast<const T*>(lds);
    const T* lB = reinterpret_cast<const T*>(lds + offB);
    T* lC = reinterpret_cast<T*>(lds + offC);

    // One tile (P matrices of the run starting at index mi0): operands from
    // LDS into MFMA registers.
    struct Ops { R ar[KB], ai[KB], br[KB], bi[KB]; };
    auto gather = [&](int mi, int cnt, Ops& o) {
        const bool mv = mi < cnt;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
            const int kk = kk0 + kb;
            T va = make_val<T>(R(0), R(0)), vb = make_val<T>(R(0), R(0));
            if (mv && kk < k) {
                if (row_ok) va = lA[mi * eA + (ACONT ? kk + ij * k : ij + kk * m)];
                if (col_ok) vb = lB[mi * eB + (BCONT ? kk + ij * k : ij + kk * n)];
            }
            o.ar[kb] = re_of<T>(va);
            o.br[kb] = re_of<T>(vb);
            if (CPLX) {
                o.ai[kb] = im_of<T>(va) * (R)a.a_conj;
                o.bi[kb] = im_of<T>(vb) * (R)a.b_conj;
            } else {
                o.ai[kb] = 0;
                o.bi[kb] = 0;
            }
        }
    };
    auto product = [&](const Ops& o, acc_t& acc_r, acc_t& acc_i) {
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
            acc_r = M::run(o.ar[kb], o.br[kb], acc_r);
            if (CPLX) {
                acc_r = M::run(-o.ai[kb], o.bi[kb], acc_r);
                acc_i = M::run(o.ar[kb], o.bi[kb], acc_i);
                acc_i = M::run(o.ai[kb], o.br[kb], acc_i);
            }
        }
    };
    // epilogue of one tile: C_in from LDS (if beta != 0), result back to LDS
    auto finish = [&](int mi, int cnt, const acc_t& acc_r, const acc_t& acc_i) {
        if (mi >= cnt) return;
        T* cm = lC + mi * eC + ij * m;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (!keep[r]) continue;
            R cr = 0, ci = 0;
            if (!b0) {
                const T cv = cm[orow[r]];
                cr = re_of<T>(cv);
                ci = im_of<T>(cv);
            }
            R outr, outi = 0;
            if (!CPLX) {
                if (a0)
                    outr = b0 ? R(0) : br_ * cr;
                else if (b0)
                    outr = ar_ * acc_r[r];
                else
                    outr = __builtin_fma(ar_, acc_r[r], br_ * cr);
            } else {
                R tr = 0, ti = 0;
                if (!b0) {
                    tr = __builtin_fma(br_, cr, -(bi_ * ci));
                    ti = __builtin_fma(br_, ci, bi_ * cr);
                }
                if (!a0) {
                    tr = __builtin_fma(ar_, acc_r[r], __builtin_fma(-ai_, acc_i[r], tr));
                    ti = __builtin_fma(ar_, acc_i[r], __builtin_fma(ai_, acc_r[r], ti));
                }
                outr = tr;
                outi = ti;
            }
            cm[orow[r]] = make_val<T>(outr, outi);
        }
    };

    Run cur = make_run(q0);
    if (q0 < nsteps) issue_loads(cur);
    for (int64_t step = q0; step < nsteps; step += W) {
        commit(cur);
        wave_lds_sync();
        // prefetch the next run into registers while this one is processed
        const Run nxt = make_run(step + W);
        if (step + W < nsteps) issue_loads(nxt);

        // tiles of the run, two at a time so their LDS reads overlap
        const int ntiles = (cur.cnt + P - 1) / P;
        int tile = 0;
        for (; tile + 1 < ntiles; tile += 2) {
            Ops o0, o1;
            acc_t r0 = {0, 0, 0, 0}, i0 = {0, 0, 0, 0}, r1 = {0, 0, 0, 0}, i1 = {0, 0, 0, 0};
            if (!a0) {
                gather(tile * P + sel, cur.cnt, o0);
                gather((tile + 1) * P + sel, cur.cnt, o1);
                product(o0, r0, i0);
                product(o1, r1, i1);
            }
            finish(tile * P + sel, cur.cnt, r0, i0);
            finish((tile + 1) * P + sel, cur.cnt, r1, i1);
        }
        if (tile < ntiles) {
            Ops o0;
            acc_t r0 = {0, 0, 0, 0}, i0 = {0, 0, 0, 0};
            if (!a0) {
                gather(tile * P + sel, cur.cnt, o0);
                product(o0, r0, i0);
            }
            finish(tile * P + sel, cur.cnt, r0, i0);
        }
        wave_lds_sync();

        // C span LDS -> HBM, every byte of the span written once
        const int FCo = cur.bytesC >> 4;
#pragma unroll
        for (int t = 0; t < MAXCH; ++t) {
            const int qq = lane + 64 * t;
            if (qq < FCo) {
                const u32x4 v = *reinterpret_cast<const u32x4*>(lds + offC + 16 * qq);
                __builtin_memcpy(reinterpret_cast<unsigned int*>(cur.gC + 16 * qq), &v, 16);
            }
        }
        const int tw = (cur.bytesC & 15) >> 2;
        if (lane < tw)
            reinterpret_cast<unsigned int*>(cur.gC + 16 * FCo)[lane] =
                *reinterpret_cast<const unsigned int*>(lds + offC + 16 * FCo + 4 * lane);
        wave_lds_sync();
        cur = nxt;
    }
}

// Matrices per step for the staged kernel, or 0 when one matrix's spans do
// not fit the wave's LDS slice.
template <typename T>
inline int staged_run_length(int m, int n, int k, int64_t batch, int min_waves)
{
    const int per = (m * k + k * n + m * n) * (int)sizeof(T);
    const int room = StagedCfg<T>::LDSW - 32;   // two 16-byte alignment pads
    if (per <= 0 || per > room) return 0;
    int G = room / per;
    if (G > 256) G = 256;
    // enough runs to keep min_waves waves busy
    const int64_t fair = (batch + min_waves - 1) / min_waves;
    if (fair < G) G = fair < 1 ? 1 : (int)fair;
    // whole tiles per run where possible
    int mx = m > n ? m : n;
    mx = mx > k ? mx : k;
    const int P = mx <= 4 ? 4 : (mx <= 8 ? 2 : 1);
    if (G >= P) G -= G % P;
    return G;
}

template <typename T, int D, bool ACONT, bool BCONT>
hipError_t launch_staged(GemmArgs<T> a, hipStream_t stream)
{
    auto kern = gemm_staged_kernel<T, D, ACONT, BCONT>;
    const int64_t steps = (a.batch + a.G - 1) / a.G;
    const int64_t grid = persistent_grid(kern, steps, a);
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(256), 0, stream, a);
    return hipGetLastError();
}

}  // namespace sbg
