// Batched small-matrix GEMM on CDNA4 matrix cores (gfx950): strided and
// pointer-array forms.
//
// Computes C_p <- alpha op(A_p) op(B_p) + beta C_p (Sec. 2, Eq. (1)) for
// m, n, k <= 16 (larger sizes: gemm_blocked.h, whose blocks reuse the tile
// routines here).  Design (what differs from the paper's Sec. 7 thread-per-
// entry and register-blocked shared-memory kernels):
//
//  * One wavefront owns a "tile": 16/D independent matrices of size class D
//    (D = 4, 8 or 16) packed block-diagonally into one 16 x 16 x 16 product.
//    The 16 x 16 x 4 MFMA (f32 or f64) is applied D/4 times; the off-diagonal
//    blocks of the product mix two different matrices and are discarded.
//  * MFMA operand layout: lane L = 16 g + c (g = 0..3, c = 0..15) supplies
//    op(A)(row c, k-index pi) and op(B)(k-index pi, column c) at step kb,
//    with pi = (D/4) g + kb, so one lane's k-indices are consecutive.  A lane
//    therefore reads a row of op(A) and a column of op(B) of matrix c / D
//    straight from global memory: no LDS staging, no shuffles.  When the
//    k-index is the fast storage index (op T/C on A, op N/R on B) the lane's
//    D/4 values are one vector load; otherwise neighbouring lanes read
//    neighbouring addresses.
//  * The result registers follow the MFMA's own layout: f32 returns rows
//    4g..4g+3 of column c (one contiguous run, stored with one vector store),
//    f64 returns rows g, g+4, g+8, g+12.  A register is kept when its row and
//    column fall in the same diagonal block.
//  * Transposition selects one of four kernel variants (which operand has k
//    as its fast index); conjugation is a sign on the imaginary part (the
//    paper's functor idea, Sec. 6).
//  * Complex products use four real MFMAs (re*re, -im*im, re*im, im*re); the
//    3M method is not used (Sec. 8).
//  * The a1b0 / axpby distinction of Sec. 6 is a wave-uniform branch: with
//    beta == 0 C is never loaded, with alpha == 0 A and B are never loaded.
//  * Narrow inputs (bf16, fp16, fp8-e4m3 with per-matrix scales) are decoded
//    exactly to binary32 as they are loaded; BF16x3 splits binary32 operands
//    into bf16 hi + lo on the fly.  Accumulation is binary32.
//  * Each wave keeps U tiles of loads in flight before it computes (U chosen
//    per call from the actual sizes, about 8 KB per wave); the grid
//    is persistent, and work-groups are renumbered so that each XCD (dispatch
//    is round-robin over the 8 XCDs) takes runs of `xcd_chunk` consecutive
//    tile groups, keeping cache lines shared by neighbouring matrices inside
//    one L2.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>
#include <type_traits>

#include "gemm_tile.h"

namespace sbg {

template <typename T> __device__ __forceinline__ void load_scalars(const GemmArgs<T>& a, T& alpha, T& beta)
{
    alpha = a.alpha_dev ? *a.alpha_dev : a.alpha;
    beta = a.beta_dev ? *a.beta_dev : a.beta;
}

// TI: stored type of A and B; MODE: 0 plain, 1 BF16x3; PTR: pointer-array
// form; PIPE: issue the next group's loads before computing the current one.
template <typename T, typename TI, int MODE, int D, int U, bool ACONT, bool BCONT, bool PTR, bool PIPE>
__global__ __launch_bounds__(256) void gemm_mfma_kernel(const GemmArgs<T> a)
{
    using R = typename Tr<T>::R;
    constexpr int P = 16 / D;
    const LaneGeom<D, R> L;
    T alpha, beta;
    load_scalars(a, alpha, beta);
    const bool a0 = is_zero(alpha), b0 = is_zero(beta);

    const int64_t W = (int64_t)gridDim.x * 4;
    const int64_t q = xcd_wave_index(a.xcd_chunk);
    const int64_t ntiles = (a.batch + P - 1) / P;
    const int64_t ngroups = (ntiles + U - 1) / U;

    // the matrices this lane serves in the U tiles of group grp
    auto setup = [&](int64_t grp, LaneMat<T, TI, 1> (&mats)[U]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t p = ((grp * U + u) * P) + L.sel;
            LaneMat<T, TI, 1>& mt = mats[u];
            mt.valid = p < a.batch;
            // lanes past the batch carry the last matrix's pointers (their
            // loads stay in bounds; nothing of theirs is stored)
            const int64_t pe = mt.valid ? p : a.batch - 1;
            mt.m = a.m;
            mt.n = a.n;
            mt.k = a.k;
            mt.lda = a.lda;
            mt.ldb = a.ldb;
            mt.ldc = a.ldc;
            mt.A = nullptr;
            mt.B = nullptr;
            mt.scale = 1.0f;
            if (PTR) {
                if (!a0) {
                    mt.A = in_space<1>(static_cast<const TI*>(a.Aarr[pe]));
                    mt.B = in_space<1>(static_cast<const TI*>(a.Barr[pe]));
                }
                mt.C = in_space<1>(a.Carr[pe]);
            } else {
                if (!a0) {
                    mt.A = in_space<1>(static_cast<const TI*>(a.A) + pe * a.strideA);
                    mt.B = in_space<1>(static_cast<const TI*>(a.B) + pe * a.strideB);
                }
                mt.C = in_space<1>(a.C + pe * a.strideC);
            }
            if (a.scaleA) mt.scale = a.scaleA[pe] * a.scaleB[pe];
            // over-reads of up to 3 elements stay inside the buffer when
            // later matrices of the batch follow at least that far on
            const int64_t after = a.batch - 1 - pe;
            mt.overA = !PTR && after * a.strideA >= 3;
            mt.overB = !PTR && after * a.strideB >= 3;
            mt.overC = !PTR && after * a.strideC >= 3;
        }
    };

    if (!PIPE) {
        for (int64_t grp = q; grp < ngroups; grp += W) {
            LaneMat<T, TI, 1> mats[U];
            setup(grp, mats);
            tile_group<T, TI, MODE, D, U, ACONT, BCONT>(mats, L, alpha, beta, a0, b0, a.a_conj, a.b_conj);
        }
        return;
    }
    // software pipeline across groups: loads of group grp + W are in flight
    // while group grp is multiplied and stored
    if (q >= ngroups) return;
    LaneMat<T, TI, 1> cur[U], nxt[U];
    TileRegs<T, TI, D, U> rc, rn;
    setup(q, cur);
    tile_load<T, TI, D, U, ACONT, BCONT>(cur, L, a0, b0, rc);
    for (int64_t grp = q; grp < ngroups; grp += W) {
        const bool more = grp + W < ngroups;
        if (more) {
            setup(grp + W, nxt);
            tile_load<T, TI, D, U, ACONT, BCONT>(nxt, L, a0, b0, rn);
        }
        tile_finish<T, TI, MODE, D, U>(cur, L, alpha, beta, a0, b0, a.a_conj, a.b_conj, rc);
        if (more) {
#pragma unroll
            for (int u = 0; u < U; ++u) cur[u] = nxt[u];
            rc = rn;
        }
    }
}

// Work-groups of 256 threads that fit on one CU at once (registers and LDS),
// cached per kernel (the cache is keyed by the kernel's address: kernels of
// one argument type share a C++ type, not an occupancy).
template <typename K>
inline int resident_per_cu(K kernel)
{
    return resident_blocks_per_cu(reinterpret_cast<const void*>(kernel));
}

// Persistent grid for `units` independent wave-sized work units, a multiple
// of 8 so the XCD renumbering is exact: by default 4 work-groups per CU
// capped by the kernel's residency; an explicit choice (tuned table entry or
// knob) is taken as given, so it may also ask for more work-groups than can
// be resident at once (they start as earlier ones finish, which evens out
// the end of the launch).  Sets the XCD run length to a divisor of the waves
// per XCD.
template <typename T, typename K>
inline int64_t persistent_grid(K kernel, int64_t units, GemmArgs<T>& a)
{
    const Tuning& tu = tuning();
    int per_cu = resident_per_cu(kernel);
    const int want = a.plan_wg > 0 ? a.plan_wg : (tu.wg_per_cu > 0 ? tu.wg_per_cu : 4);
    if (a.plan_wg > 0 || tu.wg_per_cu > 0) per_cu = want;
    else if (per_cu > want) per_cu = want;
    const int64_t wg_needed = (units + 3) / 4;
    const int64_t cap = tu.grid > 0 ? (int64_t)tu.grid : (int64_t)device_cu_count() * per_cu;
    int64_t grid = wg_needed < cap ? wg_needed : cap;
    if (grid < 1) grid = 1;
    grid = ((grid + 7) / 8) * 8;
    const int64_t wx = grid / 8 * 4;   // waves per XCD
    const int xc = a.plan_xcd > 0 ? a.plan_xcd : (tu.xcd_chunk > 0 ? tu.xcd_chunk : 16);
    int64_t s = xc;
    if (s > wx) s = wx;
    while (wx % s) --s;
    a.xcd_chunk = s;
    return grid;
}

template <typename T, typename TI, int MODE, int D, int U, bool ACONT, bool BCONT, bool PTR, bool PIPE>
hipError_t launch_up(GemmArgs<T> a, hipStream_t stream)
{
    constexpr int P = 16 / D;
    auto kern = gemm_mfma_kernel<T, TI, MODE, D, U, ACONT, BCONT, PTR, PIPE>;
    const int64_t tiles = (a.batch + P - 1) / P;
    const int64_t groups = (tiles + U - 1) / U;
    const int64_t grid = persistent_grid(kern, groups, a);
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(256), 0, stream, a);
    return hipGetLastError();
}

template <typename T, typename TI, int MODE, int D, int U, bool ACONT, bool BCONT, bool PTR>
hipError_t launch_u(GemmArgs<T> a, hipStream_t stream)
{
    if (tuning().pipeline) return launch_up<T, TI, MODE, D, U, ACONT, BCONT, PTR, true>(a, stream);
    return launch_up<T, TI, MODE, D, U, ACONT, BCONT, PTR, false>(a, stream);
}

// Largest tile unroll instantiated per element type and size class (bounded
// by registers: the unrolled tiles' operands and accumulators stay resident).
template <typename T, int D> struct UMax {
    static constexpr int bytes = (int)sizeof(T);
    static constexpr int value = bytes >= 16 ? (D == 16 ? 1 : (D == 8 ? 2 : 4))
                               : bytes == 8 ? (D == 16 ? 2 : (D == 8 ? 4 : 8))
                               : (D == 16 ? 4 : 8);
};

// Tiles per wave per step for the actual sizes: the largest power of two
// (up to UMax) whose loads and stores stay within the per-wave byte target,
// so partly filled tiles (e.g. n = 9 in the 16 class) keep as many bytes in
// flight as full ones.
template <typename T, typename TI, int D>
inline int choose_unroll(const GemmArgs<T>& a)
{
    if (a.plan_unroll > 0) {
        int U = 1;
        while (U * 2 <= UMax<T, D>::value && U * 2 <= a.plan_unroll) U *= 2;
        return U;
    }
    const int64_t P = 16 / D;
    const int64_t tile = P * ((int64_t)(a.m * a.k + a.k * a.n) * (int64_t)sizeof(TI) +
                              2 * (int64_t)a.m * a.n * (int64_t)sizeof(T));
    // class 16: the budget is stated for 4-byte elements and grows with the
    // element size (measured: U = 2 at n = 16 for f32 and f64 alike)
    const int64_t target = D == 16 ? tuning().tile_bytes16 * (int64_t)sizeof(T) / 4 : tuning().tile_bytes;
    int U = 1;
    while (U * 2 <= UMax<T, D>::value && (U * 2) * tile <= target) U *= 2;
    return U;
}

template <typename T, typename TI, int MODE, int D, bool ACONT, bool BCONT, bool PTR>
hipError_t launch_variant(GemmArgs<T> a, hipStream_t stream)
{
    constexpr int UM = UMax<T, D>::value;
    const int U = choose_unroll<T, TI, D>(a);
    if constexpr (UM >= 8)
        if (U == 8) return launch_u<T, TI, MODE, D, 8, ACONT, BCONT, PTR>(a, stream);
    if constexpr (UM >= 4)
        if (U == 4) return launch_u<T, TI, MODE, D, 4, ACONT, BCONT, PTR>(a, stream);
    if constexpr (UM >= 2)
        if (U == 2) return launch_u<T, TI, MODE, D, 2, ACONT, BCONT, PTR>(a, stream);
    return launch_u<T, TI, MODE, D, 1, ACONT, BCONT, PTR>(a, stream);
}

template <typename T, typename TI, int MODE, int D, bool ACONT, bool BCONT>
hipError_t launch_staged(GemmArgs<T> a, hipStream_t stream);
template <typename T>
hipError_t launch_team(const GemmArgs<T>& a, bool pointer_form, hipStream_t stream);
template <typename T>
hipError_t launch_blocked(GemmArgs<T> a, bool pointer_form, hipStream_t stream);
template <typename T, typename TI>
int staged_run_length(int m, int n, int k, int64_t batch, int min_waves);

template <typename T, typename TI, int MODE, int D, bool PTR>
hipError_t launch_ops(const GemmArgs<T>& a, hipStream_t stream)
{
    const bool at = a.a_trans, bn = !a.b_trans;
    if (at) {
        if (bn) return launch_variant<T, TI, MODE, D, true, true, PTR>(a, stream);
        return launch_variant<T, TI, MODE, D, true, false, PTR>(a, stream);
    }
    if (bn) return launch_variant<T, TI, MODE, D, false, true, PTR>(a, stream);
    return launch_variant<T, TI, MODE, D, false, false, PTR>(a, stream);
}

__host__ __device__ inline int size_class(int m, int n, int k)
{
    int mx = m > n ? m : n;
    mx = mx > k ? mx : k;
    return mx <= 4 ? 4 : (mx <= 8 ? 8 : 16);
}

// Do runs of G packed matrices span whole 16-byte chunks of every operand
// (A and B at ei bytes per element, C at ec)?  Then the LDS-staged kernel
// needs no span tails for full runs.
inline bool staged_whole_chunks(int m, int n, int k, int G, int ei, int ec)
{
    const int64_t g = G;
    return (g * m * k * ei) % 16 == 0 && (g * k * n * ei) % 16 == 0 && (g * m * n * ec) % 16 == 0;
}

// Packed layout: minimal leading dimensions and strides (lda, ldb are the
// stored row counts, which depend on the ops).
template <typename T>
inline bool is_packed(const GemmArgs<T>& a)
{
    const int64_t ra = a.a_trans ? a.k : a.m, ca = a.a_trans ? a.m : a.k;
    const int64_t rb = a.b_trans ? a.n : a.k, cb = a.b_trans ? a.k : a.n;
    return a.k >= 1 && a.lda == ra && a.ldb == rb && a.ldc == a.m && a.strideA == ra * ca &&
           a.strideB == rb * cb && a.strideC == (int64_t)a.m * a.n;
}

template <typename T, typename TI, int MODE, int D>
hipError_t launch_staged_ops(const GemmArgs<T>& a, hipStream_t stream)
{
    const bool at = a.a_trans, bn = !a.b_trans;
    if (at) return bn ? launch_staged<T, TI, MODE, D, true, true>(a, stream)
                      : launch_staged<T, TI, MODE, D, true, false>(a, stream);
    return bn ? launch_staged<T, TI, MODE, D, false, true>(a, stream)
              : launch_staged<T, TI, MODE, D, false, false>(a, stream);
}

// Team kernel geometry (gemm_team.h).  Elements per 16-byte vector:
template <typename T> struct TeamVec { static constexpr int V = 16 / (int)sizeof(T); };

// Lanes per team: one per column of C and of op(B) (n), one per stored
// column of A (k columns for op N/R, m for T/C) and of B (k for op T/C).
__host__ __device__ inline int team_size(int m, int n, int k, bool a_trans)
{
    int ts = n > k ? n : k;
    if (a_trans && m > ts) ts = m;
    return ts < 1 ? 1 : ts;
}

// Vector columns when every column the call loads or stores holds at least
// one 16-byte vector: C's and (op N/R) A's columns have m elements, B's (op
// N/R) and A's (op T/C) k, B's (op T/C) n.
template <typename T>
inline bool team_vec(const GemmArgs<T>& a)
{
    constexpr int V = TeamVec<T>::V;
    const bool kused = a.k > 0;
    return a.m >= V && (!kused || a.k >= V || (!a.a_trans && a.b_trans)) && (!kused || !a.b_trans || a.n >= V);
}

// The built-in rule for the staged kernel (measured): in the 16 class it wins
// when the direct kernel cannot use whole vectors -- for 4-byte inputs unless
// m and k are multiples of 4 (then the k-contiguous operand and C load as
// 16-byte vectors), for 8-byte inputs up to 11 rows/columns (longer f64 rows
// fill their cache lines directly).  The smaller classes and the complex
// types (four real products per step double the LDS gathers) stay direct.
template <typename T, typename TI>
inline bool staged_rule(const GemmArgs<T>& a)
{
    const int mx = a.m > a.n ? (a.m > a.k ? a.m : a.k) : (a.n > a.k ? a.n : a.k);
    if (Tr<T>::cplx || size_class(a.m, a.n, a.k) != 16) return false;
    return sizeof(TI) >= 8 ? mx <= 11 : !((a.m & 3) == 0 && (a.k & 3) == 0);
}

// The built-in rule for the team kernel (measured, N = 100,000, square): it
// is ahead for every size <= 8 except 8-byte and larger elements at 7 and 8,
// where the MFMA tiles are full enough to win.
template <typename T>
inline bool team_rule(const GemmArgs<T>& a)
{
    const int mx = a.m > a.n ? (a.m > a.k ? a.m : a.k) : (a.n > a.k ? a.n : a.k);
    return mx <= 8 && !(sizeof(T) >= 8 && mx >= 7);
}

template <typename T> struct TypeCode;
template <> struct TypeCode<float> { static constexpr int v = 0; };
template <> struct TypeCode<double> { static constexpr int v = 1; };
template <> struct TypeCode<float2> { static constexpr int v = 2; };
template <> struct TypeCode<double2> { static constexpr int v = 3; };

enum class Kern { Direct, Staged, Team, Blocked };

// The kernel and launch shape of one call: explicit knobs first, then the
// tuned table's entry for (type, form, op pair, size), then the built-in
// rules.  Fills the plan_* fields of a, and G for the staged kernel.
template <typename T, typename TI, int MODE>
inline Kern plan_gemm(GemmArgs<T>& a, bool pointer_form)
{
    a.plan_wg = a.plan_xcd = a.plan_unroll = 0;
    a.G = 0;
    if (a.m > 16 || a.n > 16 || a.k > 16) return Kern::Blocked;
    const Tuning& tu = tuning();
    const int mx = a.m > a.n ? (a.m > a.k ? a.m : a.k) : (a.n > a.k ? a.n : a.k);
    const int D = size_class(a.m, a.n, a.k);
    constexpr bool plain = MODE == 0 && std::is_same<T, TI>::value;
    const TunedEntry* te = (plain && tu.table) ? tuned_entry(TypeCode<T>::v, pointer_form, a.a_trans, a.b_trans, mx)
                                               : nullptr;
    if (te) {
        if (tu.wg_per_cu == 0) a.plan_wg = te->wg_per_cu;
        if (tu.xcd_chunk == 0) a.plan_xcd = te->xcd_chunk;
        a.plan_unroll = te->unroll;
    }
    if (tu.unroll > 0) a.plan_unroll = tu.unroll;
    if (plain) {
        const bool team_ok = D <= 8 || (D == 16 && !Tr<T>::cplx);
        bool team;
        if (tu.path == 1) team = false;
        else if (tu.path == 2) team = D <= 8;
        else if (tu.path == 3) team = team_ok;
        else if (te && te->path) team = te->path == 2;
        else team = team_rule(a);
        if (team && team_ok) return Kern::Team;
    }
    if (!pointer_form && is_packed(a) && !a.scaleA && tu.staged != 0) {
        bool st;
        if (tu.staged == 1) st = true;
        else if (te && te->path && tu.path == 0) st = te->path == 3;
        else st = staged_rule<T, TI>(a);
        if (st) a.G = staged_run_length<T, TI>(a.m, a.n, a.k, a.batch, device_cu_count() * 16);
        if (a.G > 0) return Kern::Staged;
    }
    return Kern::Direct;
}

// Strided / pointer-array dispatch after plan_gemm: the team kernel, the
// LDS-staged kernel for packed strided batches, the direct MFMA tile kernel,
// or the sub-blocked kernel above 16.
template <typename T, typename TI, int MODE>
hipError_t launch_direct(GemmArgs<T> a, bool pointer_form, hipStream_t stream)
{
    const Kern kind = plan_gemm<T, TI, MODE>(a, pointer_form);
    if (kind == Kern::Blocked) {
        if constexpr (MODE == 0 && std::is_same<T, TI>::value) return launch_blocked<T>(a, pointer_form, stream);
        return hipErrorInvalidValue;
    }
    const int D = size_class(a.m, a.n, a.k);
    if constexpr (MODE == 0 && std::is_same<T, TI>::value)
        if (kind == Kern::Team) return launch_team<T>(a, pointer_form, stream);
    if (kind == Kern::Staged) {
        if (D == 4) return launch_staged_ops<T, TI, MODE, 4>(a, stream);
        if (D == 8) return launch_staged_ops<T, TI, MODE, 8>(a, stream);
        return launch_staged_ops<T, TI, MODE, 16>(a, stream);
    }
    if (pointer_form) {
        if (D == 4) return launch_ops<T, TI, MODE, 4, true>(a, stream);
        if (D == 8) return launch_ops<T, TI, MODE, 8, true>(a, stream);
        return launch_ops<T, TI, MODE, 16, true>(a, stream);
    }
    if (D == 4) return launch_ops<T, TI, MODE, 4, false>(a, stream);
    if (D == 8) return launch_ops<T, TI, MODE, 8, false>(a, stream);
    return launch_ops<T, TI, MODE, 16, false>(a, stream);
}

// Plain S/D/C/Z.
template <typename T>
hipError_t launch_gemm_impl(GemmArgs<T> a, bool pointer_form, hipStream_t stream)
{
    return launch_direct<T, T, 0>(a, pointer_form, stream);
}

template <typename T> struct TypeName;
template <> struct TypeName<float> { static constexpr const char* s = "float"; };
template <> struct TypeName<double> { static constexpr const char* s = "double"; };
template <> struct TypeName<float2> { static constexpr const char* s = "HIP_vector_type<float, 2u>"; };
template <> struct TypeName<double2> { static constexpr const char* s = "HIP_vector_type<double, 2u>"; };
template <> struct TypeName<bf16_t> { static constexpr const char* s = "sbg::bf16_t"; };
template <> struct TypeName<f16_t> { static constexpr const char* s = "sbg::f16_t"; };
template <> struct TypeName<e4m3_t> { static constexpr const char* s = "sbg::e4m3_t"; };

// The kernel symbol of a call above size 16 (gemm_blocked.h).
template <typename T>
int describe_blocked(const GemmArgs<T>& a, bool pointer_form, char* buf, int len);

// The kernel symbol (as profilers demangle it) a plain launch with these
// arguments uses, written into buf.
template <typename T>
int describe_gemm_impl(GemmArgs<T> a, bool pointer_form, char* buf, int len)
{
    const auto tf = [](bool b) { return b ? "true" : "false"; };
    if (a.m > 16 || a.n > 16 || a.k > 16) return describe_blocked<T>(a, pointer_form, buf, len);
    const Kern kind = plan_gemm<T, T, 0>(a, pointer_form);
    const int D = size_class(a.m, a.n, a.k);
    if (kind == Kern::Team)
        return snprintf(buf, len, "void sbg::gemm_team_kernel<%s, %d, %s, %s, %s, %s>(sbg::GemmArgs<%s>)",
                        TypeName<T>::s, D, tf(!a.a_trans), tf(!a.b_trans), tf(team_vec(a)), tf(pointer_form),
                        TypeName<T>::s);
    if (kind == Kern::Staged)
        return snprintf(buf, len, "void sbg::gemm_staged_kernel<%s, %s, 0, %d, %s, %s, %s>(sbg::GemmArgs<%s>)",
                        TypeName<T>::s, TypeName<T>::s, D, tf(a.a_trans), tf(!a.b_trans),
                        tf(staged_whole_chunks(a.m, a.n, a.k, a.G, (int)sizeof(T), (int)sizeof(T))), TypeName<T>::s);
    const int U = D == 4 ? choose_unroll<T, T, 4>(a) : (D == 8 ? choose_unroll<T, T, 8>(a) : choose_unroll<T, T, 16>(a));
    return snprintf(buf, len, "void sbg::gemm_mfma_kernel<%s, %s, 0, %d, %d, %s, %s, %s, %s>(sbg::GemmArgs<%s>)",
                    TypeName<T>::s, TypeName<T>::s, D, U, tf(a.a_trans), tf(!a.b_trans), tf(pointer_form),
                    tf(tuning().pipeline), TypeName<T>::s);
}

}  // namespace sbg

#define SBG_INSTANTIATE_GEMM(T)                                                      \
    namespace sbg {                                                                  \
    template <>                                                                      \
    hipError_t launch_gemm<T>(const GemmArgs<T>& a, bool pointer_form, hipStream_t s) \
    {                                                                                \
        return launch_gemm_impl<T>(a, pointer_form, s);                              \
    }                                                                                \
    template <>                                                                      \
    int describe_gemm<T>(const GemmArgs<T>& a, bool pointer_form, char* buf, int len) \
    {                                                                                \
        return describe_gemm_impl<T>(a, pointer_form, buf, len);                     \
    }                                                                                \
    template <>                                                                      \
    hipError_t launch_vbatched<T>(const GemmArgs<T>& a, hipStream_t s)               \
    {                                                                                \
        return launch_vbatched_t<T, T, 0>(a, s);                                     \
    }                                                                                \
    }
