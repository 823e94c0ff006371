// Variable-size batched GEMM with one team of lanes per matrix, for the real
// types and the narrow input formats (binary32 / binary64 C and
// accumulation).  The batch is walked in its own order, with no binning
// pass: a persistent kernel serves 64 / D consecutive matrices per wave step
// with teams of D lanes, D being the size class (4, 8 or 16) of the declared
// bounds max(max_m, max_n, max_k).  The column-per-lane scheme of
// gemm_team.h, with per-matrix sizes:
//
//  * The team reads its matrix's sizes, leading dimensions and pointers from
//    the caller's arrays, and checks them (rejected matrices are skipped and
//    counted in word 3 of the workspace).
//  * Lane t of a team loads one stored column of A, of B and of C (length
//    m, k or n by the op; the lengths differ from team to team).  Columns of
//    16 bytes or more load as 16-byte vectors inside the column, the last one
//    ending at the column's end; a shorter column loads the 16-byte ALIGNED
//    chunk(s) holding it -- an aligned chunk never crosses a page, so a load
//    is never a fault even at the end of an allocation, and bytes outside
//    the column are dropped.  The partial 16 bytes are re-aligned in
//    registers: selects over dwords, then (2- and 1-byte types) a byte
//    funnel shift.
//  * Every load is issued before the first wait (branch-free addresses; an
//    empty asm makes the loaded registers live before any branch).
//  * op(A)'s entries reach the team's lanes by DPP broadcasts (no LDS): for
//    teams of 16 fused into the FMA.  Entries past a matrix's k are zero on
//    both sides, so the k loop runs to the wave's largest k (a switch with
//    fully unrolled cases).
//  * C is stored as whole 16-byte vectors plus the vector ending at the
//    column's end (built in LDS), or element by element for columns shorter
//    than 16 bytes.
// Narrow inputs (bf16, fp16, fp8-e4m3 with the matrix's scale product; e4m3
// by the hardware conversion) are decoded to binary32 after loading; products of decoded values are exact in
// binary32, so the result differs from binary32 inputs only by their rounding.
#pragma once

#include <utility>

#include "gemm_team.h"
#include "gemm_vbatched.h"


namespace sbg {

typedef unsigned int vb_u4 __attribute__((ext_vector_type(4)));
typedef unsigned int vb_u4u __attribute__((ext_vector_type(4), aligned(1)));

using GBy = __attribute__((address_space(1))) const unsigned char*;
using GByw = __attribute__((address_space(1))) unsigned char*;
using LBy = __attribute__((address_space(3))) unsigned char*;

__device__ __forceinline__ GBy gby(const void* p) { return (GBy)(const unsigned char*)p; }
__device__ __forceinline__ LBy lby(unsigned char* p) { return (LBy)p; }

__device__ __forceinline__ vb_u4 g16(GBy p) { return *reinterpret_cast<__attribute__((address_space(1))) const vb_u4u*>(p); }

// Raw registers of one column: NV slots of 16 bytes plus the last vector
// (t0).  A short column (under 16 bytes) loads the aligned chunk holding its
// start into t0 and the following chunk, when the column straddles it, into
// slot 1 (t1 when NV = 1).
template <int NV>
struct VbCol {
    vb_u4 s[NV];
    vb_u4 t0, t1;
    __device__ __forceinline__ const vb_u4& next() const
    {
        if constexpr (NV >= 2) return s[1];
        else return t1;
    }
};

// Issue the loads of a column of L bytes (1 <= L <= 16 NV) at col.  The
// addresses are integer arithmetic on one base (no selects between
// pointers, which the compiler may turn into branches and waits).
template <int NV>
__device__ __forceinline__ void vb_issue(VbCol<NV>& r, GBy col, int L)
{
    const bool lng = L >= 16;
    const int nfull = L >> 4;
    const uintptr_t ci = reinterpret_cast<uintptr_t>(col);
    const unsigned bs = (unsigned)ci & 15u;
    const GBy base = reinterpret_cast<GBy>(ci - (lng ? 0u : bs));
    const unsigned st = bs + (unsigned)L > 16u ? 16u : 0u;   // next aligned chunk of a straddling short column
    const unsigned last = 16u * (unsigned)(nfull - 1);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const unsigned o = 16u * v < last ? 16u * v : last;
        r.s[v] = g16(base + (lng ? o : (NV >= 2 && v == 1 ? st : 0u)));
    }
    r.t0 = g16(base + (lng ? (unsigned)L - 16u : 0u));
    if constexpr (NV == 1) r.t1 = g16(base + (lng ? 0u : st));
}

// Dword j + sh of x (sh in 0..3).
__device__ __forceinline__ unsigned sel4(const unsigned (&x)[8], int j, int sh)
{
    const unsigned a = x[j], b = x[j + 1], c = x[j + 2], d = x[j + 3];
    return sh == 0 ? a : (sh == 1 ? b : (sh == 2 ? c : d));
}

// Column bytes 0 .. 16 NV - 1 (past L: garbage) from the raw registers: the
// partial slot is the last vector (long column) or the aligned chunk (short
// one) shifted down by a byte count -- whole dwords by selects, the rest
// (2- and 1-byte elements only, BYTES) by a byte funnel shift.
template <int NV, bool BYTES>
__device__ __forceinline__ void vb_fix(vb_u4 (&out)[NV], const VbCol<NV>& r, GBy col, int L)
{
    const bool lng = L >= 16;
    const int nfull = L >> 4;
    int shb = lng ? 16 * nfull - (L - 16) : (int)(reinterpret_cast<uintptr_t>(col) & 15);
    shb &= 15;   // 16 (a long column without a partial slot): none
    const int sh = shb >> 2;
    const vb_u4& t1 = r.next();
    const unsigned x[8] = {r.t0.x, r.t0.y, r.t0.z, r.t0.w, t1.x, t1.y, t1.z, t1.w};
    unsigned q[4];
    if constexpr (BYTES) {
        unsigned y[5];
#pragma unroll
        for (int w = 0; w < 5; ++w) y[w] = sel4(x, w, sh);
        const unsigned sb = (unsigned)shb & 3u;
#pragma unroll
        for (int w = 0; w < 4; ++w) q[w] = __builtin_amdgcn_alignbyte(y[w + 1], y[w], sb);
    } else {
#pragma unroll
        for (int w = 0; w < 4; ++w) q[w] = sel4(x, w, sh);
    }
    vb_u4 p;
    p.x = q[0];
    p.y = q[1];
    p.z = q[2];
    p.w = q[3];
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v] = (lng && v < nfull) ? r.s[v] : p;
}

// Element e of a column held as 16-byte slots, decoded to the compute type.
template <typename T, typename TI, int NV>
__device__ __forceinline__ T vb_elem(const vb_u4 (&c)[NV], int e)
{
    unsigned w[4 * NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        w[4 * v] = c[v].x;
        w[4 * v + 1] = c[v].y;
        w[4 * v + 2] = c[v].z;
        w[4 * v + 3] = c[v].w;
    }
    constexpr int ES = (int)sizeof(TI);
    if constexpr (ES == 8) {
        const unsigned long long b = (unsigned long long)w[2 * e] | ((unsigned long long)w[2 * e + 1] << 32);
        return (T)__builtin_bit_cast(double, b);
    } else if constexpr (ES == 4) {
        return (T)__builtin_bit_cast(float, w[e]);
    } else if constexpr (ES == 2) {
        TI x;
        x.v = (unsigned short)(w[e >> 1] >> (16 * (e & 1)));
        return (T)dec(x);
    } else {
        // OCP E4M3 -> binary32 by the hardware conversion (exact; the
        // E4M3 NaN codes give NaN), two bytes of a dword per instruction
        const int word = (int)w[e >> 2];
        const auto f2 = (e & 2) ? __builtin_amdgcn_cvt_pk_f32_fp8(word, true)
                                : __builtin_amdgcn_cvt_pk_f32_fp8(word, false);
        return (T)f2[e & 1];
    }
}

// Largest value of x over the wave, x being uniform within each team of D
// lanes: one lane read per team (scalar reads, no LDS round trip).
template <int D>
__device__ __forceinline__ int team_max(int x)
{
    int r = 0;
#pragma unroll
    for (int j = 0; j < 64 / D; ++j) {
        const int y = __builtin_amdgcn_readlane(x, j * D);
        r = y > r ? y : r;
    }
    return r;
}

// Value of x held by lane L of this lane's team of D lanes, by DPP (no LDS):
// D = 16, a team is a DPP row: row broadcast of lane L; D = 8, two teams per
// row: broadcasts of lanes L and 8 + L into banks 0-1 and 2-3; D = 4, a team
// is a quad: quad permute [L, L, L, L].
template <int D, int L>
__device__ __forceinline__ int team_bcast_u32(int x)
{
    if constexpr (D == 16) {
        return __builtin_amdgcn_mov_dpp(x, 0x150 + L, 0xF, 0xF, false);
    } else if constexpr (D == 8) {
        const int lo = __builtin_amdgcn_update_dpp(0, x, 0x150 + L, 0xF, 0x3, false);
        return __builtin_amdgcn_update_dpp(lo, x, 0x150 + 8 + L, 0xF, 0xC, false);
    } else {
        return __builtin_amdgcn_mov_dpp(x, L * 0x55, 0xF, 0xF, false);
    }
}

template <int D, int L>
__device__ __forceinline__ float team_bcast(float x)
{
    return __builtin_bit_cast(float, team_bcast_u32<D, L>(__builtin_bit_cast(int, x)));
}

template <int D, int L>
__device__ __forceinline__ double team_bcast(double x)
{
    const long long v = __builtin_bit_cast(long long, x);
    const int lo = team_bcast_u32<D, L>((int)v);
    const int hi = team_bcast_u32<D, L>((int)(v >> 32));
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// Teams of 16 (one DPP row): the broadcast fused into the FMA
// (v_fmac_*_dpp with row_newbcast), sixteen per asm statement.  Each
// statement starts with two wait states, the hazard of a DPP read of a
// register a VALU op has just written; the statements write only acc.
#define SBG_FMA16C(I, X) "v_fmac_" SBG_FSFX "_dpp %" #I ", %" #X ", %32 row_newbcast:%33 row_mask:0xf bank_mask:0xf\n"
#define SBG_FMA16R(I) "v_fmac_" SBG_FSFX "_dpp %" #I ", %16, %17 row_newbcast:" #I " row_mask:0xf bank_mask:0xf\n"
#define SBG_FMA16_BODYC                                                                                      \
    "s_nop 1\n" SBG_FMA16C(0, 16) SBG_FMA16C(1, 17) SBG_FMA16C(2, 18) SBG_FMA16C(3, 19) SBG_FMA16C(4, 20)   \
        SBG_FMA16C(5, 21) SBG_FMA16C(6, 22) SBG_FMA16C(7, 23) SBG_FMA16C(8, 24) SBG_FMA16C(9, 25)           \
            SBG_FMA16C(10, 26) SBG_FMA16C(11, 27) SBG_FMA16C(12, 28) SBG_FMA16C(13, 29) SBG_FMA16C(14, 30)  \
                SBG_FMA16C(15, 31)
#define SBG_FMA16_BODYR                                                                                      \
    "s_nop 1\n" SBG_FMA16R(0) SBG_FMA16R(1) SBG_FMA16R(2) SBG_FMA16R(3) SBG_FMA16R(4) SBG_FMA16R(5)         \
        SBG_FMA16R(6) SBG_FMA16R(7) SBG_FMA16R(8) SBG_FMA16R(9) SBG_FMA16R(10) SBG_FMA16R(11) SBG_FMA16R(12) \
            SBG_FMA16R(13) SBG_FMA16R(14) SBG_FMA16R(15)
#define SBG_ACC16                                                                                            \
    "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3]), "+v"(acc[4]), "+v"(acc[5]), "+v"(acc[6]),       \
        "+v"(acc[7]), "+v"(acc[8]), "+v"(acc[9]), "+v"(acc[10]), "+v"(acc[11]), "+v"(acc[12]), "+v"(acc[13]), \
        "+v"(acc[14]), "+v"(acc[15])
#define SBG_CA16                                                                                             \
    "v"(ca[0]), "v"(ca[1]), "v"(ca[2]), "v"(ca[3]), "v"(ca[4]), "v"(ca[5]), "v"(ca[6]), "v"(ca[7]),         \
        "v"(ca[8]), "v"(ca[9]), "v"(ca[10]), "v"(ca[11]), "v"(ca[12]), "v"(ca[13]), "v"(ca[14]), "v"(ca[15])

// acc[i] += bcast_L(ca[i]) b (AC) or acc[i] += bcast_i(x) b (x = entry L of
// the lane's row of op(A)), for the sixteen i.
template <int L>
__device__ __forceinline__ void fma16_col(float (&acc)[16], const float (&ca)[16], float b)
{
#define SBG_FSFX "f32"
    asm(SBG_FMA16_BODYC : SBG_ACC16 : SBG_CA16, "v"(b), "i"(L));
#undef SBG_FSFX
}
template <int L>
__device__ __forceinline__ void fma16_col(double (&acc)[16], const double (&ca)[16], double b)
{
#define SBG_FSFX "f64"
    asm(SBG_FMA16_BODYC : SBG_ACC16 : SBG_CA16, "v"(b), "i"(L));
#undef SBG_FSFX
}
__device__ __forceinline__ void fma16_row(float (&acc)[16], float x, float b)
{
#define SBG_FSFX "f32"
    asm(SBG_FMA16_BODYR : SBG_ACC16 : "v"(x), "v"(b));
#undef SBG_FSFX
}
__device__ __forceinline__ void fma16_row(double (&acc)[16], double x, double b)
{
#define SBG_FSFX "f64"
    asm(SBG_FMA16_BODYR : SBG_ACC16 : "v"(x), "v"(b));
#undef SBG_FSFX
}
#undef SBG_FMA16C
#undef SBG_FMA16R
#undef SBG_FMA16_BODYC
#undef SBG_FMA16_BODYR
#undef SBG_ACC16
#undef SBG_CA16

// acc[i] += op(A)(i, L) op(B)(L, j) on lane j of a team: op(A)'s column L is
// lane L's column (AC) or entry L of every lane's row (otherwise).
template <typename T, int D, bool AC, int L, int... I>
__device__ __forceinline__ void vbt_dpp_l(T (&acc)[D], const T (&ca)[D], T b, std::integer_sequence<int, I...>)
{
    if constexpr (D == 16) {
        if constexpr (AC) fma16_col<L>(acc, ca, b);
        else fma16_row(acc, ca[L], b);
    } else if constexpr (AC) {
        ((acc[I] = team_fma<T>(team_bcast<D, L>(ca[I]), b, acc[I])), ...);
    } else {
        ((acc[I] = team_fma<T>(team_bcast<D, I>(ca[L]), b, acc[I])), ...);
    }
}

template <typename T, int D, bool AC, int... L>
__device__ __forceinline__ void vbt_dpp_k(T (&acc)[D], const T (&ca)[D], const T (&bv)[D],
                                          std::integer_sequence<int, L...>)
{
    (vbt_dpp_l<T, D, AC, L>(acc, ca, bv[L], std::make_integer_sequence<int, D>{}), ...);
}

// The matrix a team serves, read from the caller's arrays in two stages so
// that the reads of the next step overlap the current one: vbt_load issues
// the reads of the sizes, leading dimensions, pointers and scales (a team
// past the batch re-reads the last matrix; a null pointer or scale array is
// read at a valid address and the value replaced later), vbt_check turns
// them into the matrix (checks, rejection).
struct VbtRaw {
    const void* A;
    const void* B;
    const void* C;
    int m, n, k, lda, ldb, ldc;
    float sa, sb;
    bool in;
};

struct VbtMat {
    const void* A;
    const void* B;
    void* C;
    int m, n, k, lda, ldb, ldc;
    float scale;
    bool valid;   // inside the batch and accepted
    bool bad;     // inside the batch and rejected: skipped and counted
};

template <typename T>
__device__ __forceinline__ VbtRaw vbt_load(const GemmArgs<T>& a, int64_t p)
{
    VbtRaw r;
    r.in = p < a.batch;
    const int64_t q = r.in ? p : a.batch - 1;
    const void* const* carr = reinterpret_cast<const void* const*>(a.Carr);
    r.m = a.dm[q];
    r.n = a.dn[q];
    r.k = a.dk[q];
    r.lda = a.dlda[q];
    r.ldb = a.dldb[q];
    r.ldc = a.dldc[q];
    r.A = *(a.Aarr ? a.Aarr + q : carr + q);
    r.B = *(a.Barr ? a.Barr + q : carr + q);
    r.C = carr[q];
    r.sa = *(a.scaleA ? a.scaleA + q : reinterpret_cast<const float*>(a.dm + q));
    r.sb = *(a.scaleB ? a.scaleB + q : reinterpret_cast<const float*>(a.dm + q));
    return r;
}

template <typename T>
__device__ __forceinline__ VbtMat vbt_check(const GemmArgs<T>& a, const VbtRaw& w)
{
    VbtMat r;
    r.m = w.m;
    r.n = w.n;
    r.k = w.k;
    r.lda = w.lda;
    r.ldb = w.ldb;
    r.ldc = w.ldc;
    r.A = a.Aarr ? w.A : nullptr;
    r.B = a.Barr ? w.B : nullptr;
    r.C = const_cast<void*>(w.C);
    r.scale = a.scaleA ? w.sa * w.sb : 1.0f;
    const int rowsA = a.a_trans ? r.k : r.m;
    const int rowsB = a.b_trans ? r.n : r.k;
    r.bad = w.in && (r.m < 0 || r.n < 0 || r.k < 0 || r.m > a.max_m || r.n > a.max_n || r.k > a.max_k ||
                     r.lda < (rowsA > 1 ? rowsA : 1) || r.ldb < (rowsB > 1 ? rowsB : 1) || r.ldc < (r.m > 1 ? r.m : 1));
    r.valid = w.in && !r.bad && r.m > 0 && r.n > 0;
    if (!r.valid) r.m = r.n = r.k = 0;
    return r;
}

// One wave step: TPW = 64 / D teams, one matrix each.  AC / BC: op(A) /
// op(B) is N (stored columns are operand columns) rather than T (stored
// columns are operand rows).
template <typename T, typename TI, int D, bool AC, bool BC>
__device__ __forceinline__ void vbt_step(const VbtMat& rec, const T& alpha, const T& beta, bool a0, bool b0,
                                         unsigned char* lds_wave)
{
    constexpr int ESI = (int)sizeof(TI);
    constexpr int ESC = (int)sizeof(T);
    constexpr int NVI = (D * ESI + 15) / 16;   // 16-byte slots of an input column
    constexpr int NVC = (D * ESC + 15) / 16;   // and of a C column
    const int lane = threadIdx.x & 63;
    const int team = lane / D, t = lane - team * D;
    const bool valid = rec.valid;
    const int m = rec.m, n = rec.n, k = rec.k;
    const int base = team * D;
    // stored columns of this lane: A column ta (la elements), B column tb (lb), C column tc (m)
    const int la = AC ? m : k, na = AC ? k : m;
    const int lb = BC ? k : n, nb = BC ? n : k;
    const bool has_a = !a0 && k > 0;               // A, B read at all for this matrix
    const int ta = t < na ? t : 0, tb = t < nb ? t : 0, tc = t < n ? t : 0;
    const GBy cC = gby(rec.C) + (int64_t)tc * rec.ldc * ESC;
    // matrices whose A and B are not read load from their C column instead
    const GBy cA = has_a ? gby(rec.A) + (int64_t)ta * rec.lda * ESI : cC;
    const GBy cB = has_a ? gby(rec.B) + (int64_t)tb * rec.ldb * ESI : cC;
    const int LA_ = has_a ? (la > 0 ? la : 1) * ESI : ESC;
    const int LB_ = has_a ? (lb > 0 ? lb : 1) * ESI : ESC;
    const int LC_ = m * ESC;

    VbCol<NVI> ra, rb;
    VbCol<NVC> rc;
    vb_issue<NVI>(ra, cA, LA_);
    vb_issue<NVI>(rb, cB, LB_);
    if (!b0) vb_issue<NVC>(rc, cC, LC_);
    const int kw = team_max<D>(valid && has_a ? k : 0);
#pragma unroll
    for (int v = 0; v < NVI; ++v) {
        __asm__ volatile("" ::"v"(ra.s[v]), "v"(rb.s[v]));
    }
    __asm__ volatile("" ::"v"(ra.t0), "v"(rb.t0));
    if constexpr (NVI == 1) __asm__ volatile("" ::"v"(ra.t1), "v"(rb.t1));
    if (!b0) {
        // C's registers live before the compute too, so its loads stay with A's and B's
#pragma unroll
        for (int v = 0; v < NVC; ++v) __asm__ volatile("" ::"v"(rc.s[v]));
        __asm__ volatile("" ::"v"(rc.t0));
        if constexpr (NVC == 1) __asm__ volatile("" ::"v"(rc.t1));
    }

    vb_u4 xa[NVI], xb[NVI];
    vb_fix<NVI, (ESI < 4)>(xa, ra, cA, LA_);
    vb_fix<NVI, (ESI < 4)>(xb, rb, cB, LB_);
    // decoded columns, zero past their length and for columns past the matrix
    const bool okA = valid && has_a && t < na;
    const bool okB = valid && has_a && t < nb;
    T ca[D], cb[D];
#pragma unroll
    for (int e = 0; e < D; ++e) {
        const T va = vb_elem<T, TI, NVI>(xa, e);
        const T vb = vb_elem<T, TI, NVI>(xb, e);
        ca[e] = (okA && e < la) ? va : T(0);
        cb[e] = (okB && e < lb) ? vb : T(0);
    }
    // C column (when beta != 0) re-aligned before the compute, so that its
    // raw registers are free during it
    vb_u4 xc[NVC];
    if (!b0) vb_fix<NVC, false>(xc, rc, cC, LC_);
    T acc[D];
#pragma unroll
    for (int i = 0; i < D; ++i) acc[i] = T(0);
    T* wl = reinterpret_cast<T*>(lds_wave);
    T* bl = wl + 64 * D;
    if (kw > 0) {
        T bv[D];
        if (BC) {
#pragma unroll
            for (int l = 0; l < D; ++l) bv[l] = cb[l];
        } else {
            // lane t holds row t of op(B): column t of op(B) through LDS
            vstore<T, D>(bl + lane * D, cb);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
            for (int l = 0; l < D; ++l) bv[l] = bl[(base + l) * D + t];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
#define SBG_VBT_CASE(KK) \
    case KK: vbt_dpp_k<T, D, AC>(acc, ca, bv, std::make_integer_sequence<int, KK>{}); break;
        switch (kw) {
            SBG_VBT_CASE(1)
            SBG_VBT_CASE(2)
            SBG_VBT_CASE(3)
            SBG_VBT_CASE(4)
            default:
                if constexpr (D >= 8) {
                    switch (kw) {
                        SBG_VBT_CASE(5)
                        SBG_VBT_CASE(6)
                        SBG_VBT_CASE(7)
                        SBG_VBT_CASE(8)
                        default:
                            if constexpr (D == 16) {
                                switch (kw) {
                                    SBG_VBT_CASE(9)
                                    SBG_VBT_CASE(10)
                                    SBG_VBT_CASE(11)
                                    SBG_VBT_CASE(12)
                                    SBG_VBT_CASE(13)
                                    SBG_VBT_CASE(14)
                                    SBG_VBT_CASE(15)
                                    SBG_VBT_CASE(16)
                                    default: break;
                                }
                            }
                            break;
                    }
                }
                break;
        }
#undef SBG_VBT_CASE
    }
    // the epilogue
    using R = typename Tr<T>::R;
    const R ar = (R)alpha * (R)rec.scale, br = (R)beta;
    vb_u4 oc[NVC];
    T outv[4 * NVC * 4 / ESC];
#pragma unroll
    for (int e = 0; e < D; ++e) {
        const T cin = b0 ? T(0) : vb_elem<T, T, NVC>(xc, e);
        outv[e] = axpby<T>(ar, R(0), br, R(0), a0, b0, acc[e], R(0), cin);
    }
#pragma unroll
    for (int e = D; e < 16 * NVC / ESC; ++e) outv[e] = T(0);
    __builtin_memcpy(oc, outv, 16 * NVC);
    if (valid && t < n) {
        GByw col = (GByw)cC;
        using GU = __attribute__((address_space(1))) vb_u4u*;
        if (LC_ >= 16) {
            const int nfull = LC_ >> 4;
#pragma unroll
            for (int v = 0; v < NVC; ++v)
                if (v < nfull) *reinterpret_cast<GU>(col + 16 * v) = oc[v];
            if (LC_ & 15) {
                // the vector ending at the column's end, read back from the
                // lane's own op(A) slot (D elements of T = the column's size;
                // free once every lane of the wave has passed the compute)
                using LA = __attribute__((address_space(3))) vb_u4*;
                using LU = __attribute__((address_space(3))) vb_u4u*;
                LBy carea = lby(lds_wave) + lane * D * ESC;
#pragma unroll
                for (int v = 0; v < NVC; ++v) *reinterpret_cast<LA>(carea + 16 * v) = oc[v];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                const vb_u4 last = *reinterpret_cast<LU>(carea + (LC_ - 16));
                *reinterpret_cast<GU>(col + (LC_ - 16)) = last;
            }
        } else {
#pragma unroll
            for (int e = 0; e < D; ++e)
                if (e < m) st1<T>(reinterpret_cast<__attribute__((address_space(1))) T*>(col) + e, outv[e]);
        }
    }
}

// Bytes of LDS per wave: the C tail vectors and, for T / C op(B), its rows
// (D elements of T per lane each).
template <typename T, int D, bool BC>
struct VbtLds {
    static constexpr int bytes = 64 * D * (int)sizeof(T) * (BC ? 1 : 2);
};

// Persistent kernel over the batch in its own order: wave step grp serves
// matrices grp TPW .. grp TPW + TPW - 1.  Single-precision variants are held
// to 128 registers, so four waves fit on each SIMD.
template <typename T, typename TI, int D, bool AC, bool BC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1)))
void gemm_vbteam_kernel(const GemmArgs<T> a)
{
    using L = VbtLds<T, D, BC>;
    constexpr int TPW = 64 / D;
    __shared__ __attribute__((aligned(16))) unsigned char lds[4 * L::bytes];
    unsigned char* lw = lds + (threadIdx.x >> 6) * L::bytes;
    const int lane = threadIdx.x & 63;
    T alpha, beta;
    load_scalars(a, alpha, beta);
    const bool a0 = is_zero(alpha), b0 = is_zero(beta);
    const int64_t groups = (a.batch + TPW - 1) / TPW;
    const int64_t W = (int64_t)gridDim.x * 4;
    int nbad = 0;
    int64_t grp = xcd_wave_index(a.xcd_chunk);
    if (grp < groups) {
        VbtRaw raw = vbt_load(a, grp * TPW + lane / D);
        // the first reads complete before the loop, so that at its head the
        // wait covers only the reads issued one step earlier
        __asm__ volatile("" ::"v"(raw.m), "v"(raw.n), "v"(raw.k), "v"(raw.lda), "v"(raw.ldb), "v"(raw.ldc));
        __asm__ volatile("" ::"v"(raw.A), "v"(raw.B), "v"(raw.C), "v"(raw.sa), "v"(raw.sb));
        for (; grp < groups; grp += W) {
            const VbtMat mt = vbt_check(a, raw);
            // the next step's matrix is read while this one runs (the last
            // step re-reads its own: the address stays branch-free)
            const int64_t nx = grp + W < groups ? grp + W : grp;
            raw = vbt_load(a, nx * TPW + lane / D);
            nbad += (mt.bad && lane % D == 0) ? 1 : 0;   // counted once per team
            vbt_step<T, TI, D, AC, BC>(mt, alpha, beta, a0, b0, lw);
        }
    }
    if (nbad) atomicAdd(&a.ws[3], nbad);
}

template <typename T, typename TI, int D, bool AC, bool BC>
hipError_t launch_vbteam_variant(GemmArgs<T> a, hipStream_t stream)
{
    auto kern = gemm_vbteam_kernel<T, TI, D, AC, BC>;
    const int64_t steps = (a.batch + 64 / D - 1) / (64 / D);
    const int64_t grid = persistent_grid(kern, steps, a);
    if (VbDescribe& ds = vb_describe(); ds.buf) {
        const auto tf = [](bool b) { return b ? "true" : "false"; };
        snprintf(ds.buf, ds.len,
                 "kernel=void sbg::gemm_vbteam_kernel<%s, %s, %d, %s, %s>(sbg::GemmArgs<%s>) grid=%lld units=%lld",
                 TypeName<T>::s, TypeName<TI>::s, D, tf(AC), tf(BC), TypeName<T>::s, (long long)grid,
                 (long long)steps);
        return hipSuccess;
    }
    // the header (word 3: rejected matrices) starts at zero
    hipLaunchKernelGGL(vb_zero_kernel, dim3(1), dim3(64), 0, stream, a.ws);
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(256), 0, stream, a);
    return hipGetLastError();
}

template <typename T, typename TI, int D>
hipError_t launch_vbteam_d(const GemmArgs<T>& a, hipStream_t stream)
{
    const bool ac = !a.a_trans, bc = !a.b_trans;
    if (ac) return bc ? launch_vbteam_variant<T, TI, D, true, true>(a, stream)
                      : launch_vbteam_variant<T, TI, D, true, false>(a, stream);
    return bc ? launch_vbteam_variant<T, TI, D, false, true>(a, stream)
              : launch_vbteam_variant<T, TI, D, false, false>(a, stream);
}

// Team variable-size path (real types, binary32 / binary64 C, plain mode):
// no binning; the team size is the size class of the declared bounds
// max(max_m, max_n, max_k), and the op letters pick the variant
// (conjugation does not apply to real data).
template <typename T, typename TI>
hipError_t launch_vbteam(const GemmArgs<T>& a, hipStream_t stream)
{
    const int D = size_class(a.max_m, a.max_n, a.max_k);
    if (D <= 4) return launch_vbteam_d<T, TI, 4>(a, stream);
    if (D <= 8) return launch_vbteam_d<T, TI, 8>(a, stream);
    return launch_vbteam_d<T, TI, 16>(a, stream);
}

}  // namespace sbg
