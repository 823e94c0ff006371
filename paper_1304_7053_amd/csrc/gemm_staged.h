// Batched small-matrix GEMM for PACKED strided batches (lda = stored rows of
// A, strideA = rows * cols, likewise for B and C: the minimal leading
// dimensions of the paper's experiments, Sec. 8), streamed through LDS.
//
// In a packed batch a run of G consecutive matrices is one contiguous span of
// each operand.  Each wavefront owns an LDS slice and processes runs:
//   1. spans -> registers: the whole 16-byte chunks of the A, B (and, when
//      beta != 0, C) spans form one flat list; lane i loads chunks i, i+64,
//      ...  A span whose length is not a multiple of 16 also has a tail: the
//      16 bytes ending at the span's end (overlapping the last whole chunk),
//      loaded by one lane.  No access leaves a span;
//   2. registers -> LDS at the chunks' own offsets (16-byte aligned, so one
//      128-bit LDS write each; the tails are written as 32-bit words); the
//      next run's loads are issued right away and stay in flight while this
//      run computes;
//   3. LDS -> MFMA operands (the block-diagonal packing of the direct kernel:
//      16/D matrices of size class D per 16x16x16 product), results written
//      back into the C span in LDS;
//   4. C span LDS -> HBM: whole chunks plus the overlapping tail.
// Whatever m, n, k are, every global access of a wave is part of a 1 KB
// contiguous stream; small matrices move as many bytes per wave step as
// large ones.
#pragma once

#include "gemm_direct.h"

namespace sbg {

template <typename T> struct StagedCfg {
    static constexpr int LDSW = sizeof(T) >= 16 ? 16384 : 8192;  // LDS bytes per wave
    static constexpr int MAXCH = LDSW / 1024;                     // 16-B chunks per lane (bound)
};

__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__host__ __device__ inline int align16i(int x) { return (x + 15) & ~15; }

template <typename T, typename TI, int MODE, int D, bool ACONT, bool BCONT, bool FAST>
__global__ __launch_bounds__(256) void gemm_staged_kernel(const GemmArgs<T> a)
{
    using R = typename Tr<T>::R;
    using u32x4 = unsigned int __attribute__((ext_vector_type(4)));
    // 16-byte vector at 4-byte alignment (global chunk addresses follow the spans)
    typedef unsigned int u32x4a4 __attribute__((ext_vector_type(4), aligned(4)));
    constexpr int P = 16 / D;
    constexpr int LDSW = StagedCfg<T>::LDSW;
    constexpr int MAXCH = StagedCfg<T>::MAXCH;
    constexpr int EI = (int)sizeof(TI);
    constexpr int EC = (int)sizeof(T);

    __shared__ __attribute__((aligned(16))) unsigned char lds_all[4 * LDSW];
    unsigned char* lds = lds_all + (threadIdx.x >> 6) * LDSW;
    const int lane = threadIdx.x & 63;
    const LaneGeom<D, R> L;

    T alpha, beta;
    load_scalars(a, alpha, beta);
    const bool a0 = is_zero(alpha), b0 = is_zero(beta);

    const int m = a.m, n = a.n, k = a.k;
    const int eA = m * k, eB = k * n, eC = m * n;   // elements per matrix
    const int G = a.G;
    const int offB = align16i(G * eA * EI);
    const int offC = offB + align16i(G * eB * EI);

    const int64_t W = (int64_t)gridDim.x * 4;
    const int64_t nruns = (a.batch + G - 1) / G;
    const unsigned char* gA0 = static_cast<const unsigned char*>(a.A);
    const unsigned char* gB0 = static_cast<const unsigned char*>(a.B);
    unsigned char* gC0 = reinterpret_cast<unsigned char*>(a.C);

    // the run index is wave-uniform: keep it (and all span arithmetic) scalar
    const int64_t r0 = xcd_wave_index(a.xcd_chunk);
    int64_t r = ((int64_t)__builtin_amdgcn_readfirstlane((int)(r0 >> 32)) << 32) |
                (uint32_t)__builtin_amdgcn_readfirstlane((int)(r0 & 0xFFFFFFFF));
    if (r >= nruns) return;

    // Spans of run RR (the last run may be shorter; every span is >= 16 bytes
    // of whole 4-byte words, which the host guarantees): byte sizes SA, SB,
    // SCin (loaded) and SC (stored), whole-chunk counts FA, FB and the flat
    // list length FT.  All wave-uniform.
    int cnt = 0, SA = 0, SB = 0, SC = 0, SCin = 0, FA = 0, FB = 0, FT = 0;
    const unsigned char* gA = nullptr;
    const unsigned char* gB = nullptr;
    unsigned char* gC = nullptr;
#define SBG_RUN_SPANS(RR)                                                           \
    {                                                                               \
        const int64_t p0 = (RR) * G;                                                \
        cnt = (int)((a.batch - p0) < G ? (a.batch - p0) : G);                       \
        gA = gA0 + p0 * eA * EI;                                                    \
        gB = gB0 + p0 * eB * EI;                                                    \
        gC = gC0 + p0 * eC * EC;                                                    \
        SA = a0 ? 0 : cnt * eA * EI;                                                \
        SB = a0 ? 0 : cnt * eB * EI;                                                \
        SC = cnt * eC * EC;                                                         \
        SCin = b0 ? 0 : SC;                                                         \
        FA = SA >> 4;                                                               \
        FB = SB >> 4;                                                               \
        FT = FA + FB + (SCin >> 4);                                                 \
    }
    // whole chunk Q (< FT) of the flat list: global source and LDS destination
#define SBG_CHUNK(Q, SRC, DST)                                                      \
    {                                                                               \
        const bool inA = (Q) < FA;                                                  \
        const bool inB = !inA && (Q) < FA + FB;                                     \
        const int off = 16 * (inA ? (Q) : (inB ? (Q) - FA : (Q) - FA - FB));        \
        SRC = (inA ? gA : (inB ? gB : (const unsigned char*)gC)) + off;             \
        DST = (inA ? 0 : (inB ? offB : offC)) + off;                                \
    }
    // tail of span J (0 A, 1 B, 2 C): the 16 bytes ending at the span's end,
    // needed when the span is not a multiple of 16 bytes (HAS)
#define SBG_TAIL(J, SRC, DST, HAS)                                                  \
    {                                                                               \
        const int S_ = (J) == 0 ? SA : ((J) == 1 ? SB : SCin);                      \
        SRC = ((J) == 0 ? gA : ((J) == 1 ? gB : (const unsigned char*)gC)) + (S_ - 16); \
        DST = ((J) == 0 ? 0 : ((J) == 1 ? offB : offC)) + (S_ - 16);                \
        HAS = (S_ & 15) != 0;                                                       \
    }
#define SBG_ISSUE()                                                                 \
    {                                                                               \
        const int nt_ = (FT + 63) >> 6;                                             \
        _Pragma("unroll") for (int t = 0; t < MAXCH; ++t) {                         \
            if (t < nt_) {                                                          \
                const int q = lane + 64 * t;                                        \
                if (q < FT) {                                                       \
                    const unsigned char* src;                                       \
                    int dst;                                                        \
                    SBG_CHUNK(q, src, dst)                                          \
                    (void)dst;                                                      \
                    buf[t] = *reinterpret_cast<const u32x4a4*>(src);                \
                }                                                                   \
            }                                                                       \
        }                                                                           \
        if (lane < 3) {                                                             \
            const unsigned char* src;                                               \
            int dst;                                                                \
            bool has;                                                               \
            SBG_TAIL(lane, src, dst, has)                                           \
            (void)dst;                                                              \
            /* without a tail the lane re-reads the head of the C span (never   */ \
            /* empty), so the load is issued on every run                       */ \
            tbuf = *reinterpret_cast<const u32x4a4*>(has ? src : (const unsigned char*)gC); \
        }                                                                           \
    }
#define SBG_COMMIT()                                                                \
    {                                                                               \
        const int nt_ = (FT + 63) >> 6;                                             \
        _Pragma("unroll") for (int t = 0; t < MAXCH; ++t) {                         \
            if (t < nt_) {                                                          \
                const int q = lane + 64 * t;                                        \
                if (q < FT) {                                                       \
                    const unsigned char* src;                                       \
                    int dst;                                                        \
                    SBG_CHUNK(q, src, dst)                                          \
                    (void)src;                                                      \
                    *reinterpret_cast<u32x4*>(lds + dst) = buf[t];                  \
                }                                                                   \
            }                                                                       \
        }                                                                           \
        if (lane < 3) {                                                             \
            const unsigned char* src;                                               \
            int dst;                                                                \
            bool has;                                                               \
            SBG_TAIL(lane, src, dst, has)                                           \
            (void)src;                                                              \
            if (has) {                                                              \
                unsigned int* w = reinterpret_cast<unsigned int*>(lds + dst);       \
                w[0] = tbuf.x;                                                      \
                w[1] = tbuf.y;                                                      \
                w[2] = tbuf.z;                                                      \
                w[3] = tbuf.w;                                                      \
            }                                                                       \
        }                                                                           \
        /* the tail register is consumed here on every path, so the next       */ \
        /* run's tail load never waits for this one                            */ \
        __asm__ volatile("" ::"v"(tbuf));                                           \
    }

    u32x4 buf[MAXCH];
    u32x4 tbuf = {0u, 0u, 0u, 0u};

    const auto lA = in_space<3>(reinterpret_cast<const TI*>(lds));
    const auto lB = in_space<3>(reinterpret_cast<const TI*>(lds + offB));
    const auto lC = in_space<3>(reinterpret_cast<T*>(lds + offC));

    // tiles of a run of CCNT matrices from LDS: each lane's matrix mi, operand
    // entries gathered with the op folded into the LDS addressing
#define SBG_COMPUTE(CCNT)                                                           \
    {                                                                               \
        const int ccnt_ = (CCNT);                                                   \
        const int ntiles = (ccnt_ + P - 1) / P;                                     \
        for (int tile = 0; tile < ntiles; ++tile) {                                 \
            const int mi0 = tile * P + L.sel;                                       \
            LaneMat<T, TI, 3> mt[1];                                                \
            mt[0].valid = mi0 < ccnt_;                                              \
            /* lanes past the run read its last matrix */                          \
            const int mi = mt[0].valid ? mi0 : ccnt_ - 1;                           \
            mt[0].m = m;                                                            \
            mt[0].n = n;                                                            \
            mt[0].k = k;                                                            \
            mt[0].lda = ACONT ? k : m;                                              \
            mt[0].ldb = BCONT ? k : n;                                              \
            mt[0].ldc = m;                                                          \
            mt[0].A = lA + mi * eA;                                                 \
            mt[0].B = lB + mi * eB;                                                 \
            mt[0].C = lC + mi * eC;                                                 \
            mt[0].scale = 1.0f; /* per-matrix scales never take this kernel */      \
            mt[0].overA = mt[0].overB = mt[0].overC = false;                        \
            tile_group<T, TI, MODE, D, 1, ACONT, BCONT>(mt, L, alpha, beta, a0, b0, \
                                                        a.a_conj, a.b_conj);        \
        }                                                                           \
    }
    // C span LDS -> HBM for a run of the general path: whole chunks, then the
    // overlapping tail
#define SBG_STORE(CGC, CSC)                                                         \
    {                                                                               \
        const int FC = (CSC) >> 4;                                                  \
        const int nt = (FC + 63) >> 6;                                              \
        _Pragma("unroll") for (int t = 0; t < MAXCH; ++t) {                         \
            if (t < nt) {                                                           \
                const int q = lane + 64 * t;                                        \
                if (q < FC) {                                                       \
                    const u32x4 v = *reinterpret_cast<const u32x4*>(lds + offC + 16 * q); \
                    *reinterpret_cast<u32x4a4*>((CGC) + 16 * q) = v;                \
                }                                                                   \
            }                                                                       \
        }                                                                           \
        if (lane == 0 && ((CSC) & 15)) {                                            \
            const unsigned int* w = reinterpret_cast<const unsigned int*>(lds + offC + (CSC) - 16); \
            const u32x4 v = {w[0], w[1], w[2], w[3]};                               \
            *reinterpret_cast<u32x4a4*>((CGC) + (CSC) - 16) = v;                    \
        }                                                                           \
    }

    // Fast-path load and LDS write of one full run through the slot table
#define SBG_FAST_ISSUE(RR)                                                          \
    {                                                                               \
        const int64_t p0_ = (RR) * G;                                               \
        const unsigned char* bA_ = gA0 + p0_ * eA * EI;                             \
        const unsigned char* bB_ = gB0 + p0_ * eB * EI;                             \
        const unsigned char* bC_ = gC0 + p0_ * eC * EC;                             \
        _Pragma("unroll") for (int t = 0; t < MAXCH; ++t) {                         \
            const unsigned w_ = slot[t];                                            \
            const unsigned j_ = w_ >> 28;                                           \
            const unsigned char* b_ = j_ == 0 ? bA_ : (j_ == 1 ? bB_ : bC_);        \
            buf[t] = *reinterpret_cast<const u32x4a4*>(b_ + (w_ & 0x3FFF));         \
        }                                                                           \
    }
#define SBG_FAST_COMMIT(NT)                                                         \
    {                                                                               \
        _Pragma("unroll") for (int t = 0; t < MAXCH; ++t) {                         \
            if (t < (NT))                                                           \
                *reinterpret_cast<u32x4*>(lds + ((slot[t] >> 14) & 0x3FFF)) = buf[t]; \
        }                                                                           \
    }

    if constexpr (FAST) {
        // Full runs (G matrices) whose spans are whole 16-byte chunks (the
        // host prefers such G and picks this instance only then): every full
        // run has the same chunk list, so each lane packs, per slot, the
        // chunk's byte offset in its span (14 bits), its LDS offset (14 bits)
        // and its span (2 bits) once; a run then only selects the span's
        // base.  Loads are unconditional (a conditional load would leave the
        // buffer registers to be merged across paths); only slots of the list
        // are written to LDS.  The last, shorter run takes the general code.
        const int fSA = a0 ? 0 : G * eA * EI, fSB = a0 ? 0 : G * eB * EI;
        const int fSC = G * eC * EC, fSCin = b0 ? 0 : fSC;
        const int64_t nfull = a.batch / G;
        const int fFA = fSA >> 4, fFB = fSB >> 4, fFT = fFA + fFB + (fSCin >> 4);
        const int fNT = (fFT + 63) >> 6;            // load slots of a full run
        const int fFC = fSC >> 4;
        const int fNC = (fFC + 63) >> 6;            // store slots of a full run
        unsigned int slot[MAXCH];
#pragma unroll
        for (int t = 0; t < MAXCH; ++t) {
            // every slot loads on every full run: past the list it repeats the
            // last chunk; with nothing to load (alpha = beta = 0) it reads the
            // head of the run's C span, which a full run always has, unused
            int q = lane + 64 * t;
            q = q < fFT ? q : (fFT > 0 ? fFT - 1 : 0);
            const int j = q < fFA ? 0 : (q < fFA + fFB ? 1 : 2);
            const int off = 16 * (j == 0 ? q : (j == 1 ? q - fFA : q - fFA - fFB));
            const int dst = (j == 0 ? 0 : (j == 1 ? offB : offC)) + off;
            slot[t] = (unsigned)off | ((unsigned)dst << 14) | ((unsigned)j << 28);
        }
        // Full runs through the slot table, the next run's loads in flight
        // while this one computes.  One loop with one load path, so the wait
        // before each LDS write counts only the loads still ahead of it.
        if (r < nfull) SBG_FAST_ISSUE(r)
        for (; r < nfull; r += W) {
            // slot counts re-read each run: kept as two scalars instead of
            // sixteen hoisted lane masks
            int nt = fNT, nc = fNC;
            __asm__ volatile("" : "+s"(nt), "+s"(nc));
            SBG_FAST_COMMIT(nt)
            wave_lds_sync();
            if (r + W < nfull) SBG_FAST_ISSUE(r + W)
            SBG_COMPUTE(G)
            wave_lds_sync();
            unsigned char* cgC = gC0 + r * G * eC * EC;
#pragma unroll
            for (int t = 0; t < MAXCH; ++t) {
                if (t < nc) {
                    int q = lane + 64 * t;
                    q = q < fFC ? q : fFC - 1;   // repeats: the same bytes to the same address
                    const u32x4 v = *reinterpret_cast<const u32x4*>(lds + offC + 16 * q);
                    *reinterpret_cast<u32x4a4*>(cgC + 16 * q) = v;
                }
            }
            wave_lds_sync();
        }
        // the last, shorter run (index nfull) falls to at most one wave
        if (r < nruns) {
            SBG_RUN_SPANS(r)
            SBG_ISSUE()
            SBG_COMMIT()
            wave_lds_sync();
            SBG_COMPUTE(cnt)
            wave_lds_sync();
            SBG_STORE(gC, SC)
        }
    } else {
        // General path: runs with tails, the next run's chunks in flight
        // while this run computes.
        SBG_RUN_SPANS(r)
        SBG_ISSUE()
        for (; r < nruns; r += W) {
            SBG_COMMIT()
            wave_lds_sync();
            const int ccnt = cnt, cSC = SC;
            unsigned char* cgC = gC;
            if (r + W < nruns) {
                SBG_RUN_SPANS(r + W)
                SBG_ISSUE()
            }
            SBG_COMPUTE(ccnt)
            wave_lds_sync();
            SBG_STORE(cgC, cSC)
            wave_lds_sync();
        }
    }
#undef SBG_COMPUTE
#undef SBG_STORE
#undef SBG_FAST_ISSUE
#undef SBG_FAST_COMMIT
#undef SBG_ISSUE
#undef SBG_COMMIT
#undef SBG_TAIL
#undef SBG_CHUNK
#undef SBG_RUN_SPANS
}

// Matrices per wave step of the staged kernel, or 0 when it does not apply:
// the run's spans must fit the wave's LDS slice, be at least 16 bytes and
// consist of whole 4-byte words (for the last, possibly shorter run too).
template <typename T, typename TI>
inline int staged_run_length(int m, int n, int k, int64_t batch, int min_waves)
{
    if (m < 1 || n < 1 || k < 1 || batch < 1) return 0;
    const int64_t ei = (int64_t)sizeof(TI), ec = (int64_t)sizeof(T);
    const int64_t per = (int64_t)(m * k + k * n) * ei + (int64_t)m * n * ec;
    const int64_t room = StagedCfg<T>::LDSW - 32;   // two 16-byte alignment pads
    if (per > room) return 0;
    int64_t G = room / per;
    if (G > 256) G = 256;
    // enough runs to keep min_waves waves busy
    const int64_t fair = (batch + min_waves - 1) / min_waves;
    if (fair < G) G = fair < 1 ? 1 : fair;
    // whole tiles per run, and whole 4-byte words for narrow inputs; when a
    // run of whole 16-byte chunks fits (a multiple of `unit` matrices), take
    // the largest such G: full runs then need no tails (the fast path)
    const int64_t P = 16 / size_class(m, n, k);
    const int64_t step = (ei < 4 && P < 4) ? 4 : P;
    const auto whole16 = [](int64_t b) { const int64_t low = b & -b; return 16 / (low < 16 ? low : 16); };
    int64_t unit = step;
    for (const int64_t b : {(int64_t)m * k * ei, (int64_t)k * n * ei, (int64_t)m * n * ec})
        unit = whole16(b) > unit ? whole16(b) : unit;
    if (G >= unit) G -= G % unit;
    else if (unit * per <= room) G = unit;
    else if (G >= step) G -= G % step;
    else if (step * per <= room) G = step;
    if (G > batch) G = batch;
    const int64_t last = batch - ((batch - 1) / G) * G;   // matrices in the last run
    for (const int64_t c : {G, last}) {
        if (c * m * k * ei < 16 || c * k * n * ei < 16 || c * m * n * ec < 16) return 0;
        if ((c * m * k * ei) % 4 || (c * k * n * ei) % 4) return 0;
    }
    return (int)G;
}

template <typename T, typename TI, int MODE, int D, bool ACONT, bool BCONT>
hipError_t launch_staged(GemmArgs<T> a, hipStream_t stream)
{
    // the slot-table kernel only where every full run is whole 16-byte chunks
    const bool fast = staged_whole_chunks(a.m, a.n, a.k, a.G, (int)sizeof(TI), (int)sizeof(T));
    auto kern = fast ? gemm_staged_kernel<T, TI, MODE, D, ACONT, BCONT, true>
                     : gemm_staged_kernel<T, TI, MODE, D, ACONT, BCONT, false>;
    const int64_t runs = (a.batch + a.G - 1) / a.G;
    const int64_t grid = persistent_grid(kern, runs, a);
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(256), 0, stream, a);
    return hipGetLastError();
}

}  // namespace sbg
