// Building blocks shared by the batched-GEMM kernels (gfx950): element types,
// the 16x16x4 MFMA wrappers with their result layouts, narrow-type decoding,
// the BF16x3 split, and the tile routine that multiplies 16/D packed small
// matrices held by one wavefront (see gemm_direct.h for the design notes).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "sbg_internal.h"

namespace sbg {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// ---- storage types of the narrow input formats ----------------------------
struct bf16_t { unsigned short v; };   // bfloat16: upper half of a binary32
struct f16_t { unsigned short v; };    // IEEE binary16
struct e4m3_t { unsigned char v; };    // OCP 8-bit float E4M3 ("fn": no inf, max 448)

template <typename T> struct Tr;
template <> struct Tr<float>   { using R = float;  static constexpr bool cplx = false; };
template <> struct Tr<double>  { using R = double; static constexpr bool cplx = false; };
template <> struct Tr<float2>  { using R = float;  static constexpr bool cplx = true; };
template <> struct Tr<double2> { using R = double; static constexpr bool cplx = true; };

// 16x16x4 MFMA per real type, with the row held by result register r of lane
// group g (the column is always the lane index mod 16).
template <typename R> struct Mfma;
template <> struct Mfma<float> {
    using acc_t = f32x4;
    static constexpr bool rows_contig = true;
    static constexpr bool swap = false;
    static __device__ __forceinline__ int row(int g, int r) { return 4 * g + r; }
    static __device__ __forceinline__ acc_t run(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <> struct Mfma<double> {
    using acc_t = f64x4;
    static constexpr bool rows_contig = false;
    // The f64 result rows of a lane are 4 apart; feeding op(B) as the MFMA's
    // first operand and op(A) as its second makes the accumulator hold C^T,
    // so the 16 lanes of a group hold 16 consecutive rows of one C column
    // (128 contiguous bytes per store instruction and group).
    static constexpr bool swap = true;
    static __device__ __forceinline__ int row(int g, int r) { return 4 * r + g; }
    static __device__ __forceinline__ acc_t run(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

template <typename T> __device__ __forceinline__ typename Tr<T>::R re_of(const T& v);
template <typename T> __device__ __forceinline__ typename Tr<T>::R im_of(const T& v);
template <> __device__ __forceinline__ float re_of<float>(const float& v) { return v; }
template <> __device__ __forceinline__ double re_of<double>(const double& v) { return v; }
template <> __device__ __forceinline__ float re_of<float2>(const float2& v) { return v.x; }
template <> __device__ __forceinline__ double re_of<double2>(const double2& v) { return v.x; }
template <> __device__ __forceinline__ float im_of<float>(const float&) { return 0.f; }
template <> __device__ __forceinline__ double im_of<double>(const double&) { return 0.0; }
template <> __device__ __forceinline__ float im_of<float2>(const float2& v) { return v.y; }
template <> __device__ __forceinline__ double im_of<double2>(const double2& v) { return v.y; }

template <typename T> __device__ __forceinline__ T make_val(typename Tr<T>::R re, typename Tr<T>::R im);
template <> __device__ __forceinline__ float make_val<float>(float re, float) { return re; }
template <> __device__ __forceinline__ double make_val<double>(double re, double) { return re; }
template <> __device__ __forceinline__ float2 make_val<float2>(float re, float im) { return make_float2(re, im); }
template <> __device__ __forceinline__ double2 make_val<double2>(double re, double im) { return make_double2(re, im); }

template <typename T>
__device__ __forceinline__ bool is_zero(const T& v) {
    return re_of<T>(v) == 0 && im_of<T>(v) == 0;
}

// ---- decoding of stored input elements into the compute type -------------
// bfloat16 -> binary32: the 16 stored bits are the high half.
__device__ __forceinline__ float dec(bf16_t x) { return __uint_as_float(((unsigned)x.v) << 16); }
// binary16 -> binary32 (exact; hardware conversion).
__device__ __forceinline__ float dec(f16_t x) {
    _Float16 h;
    __builtin_memcpy(&h, &x.v, 2);
    return (float)h;
}
// OCP E4M3 -> binary32, exact: sign, 4-bit exponent (bias 7), 3-bit fraction;
// exponent 0 is subnormal (fraction * 2^-9); S.1111.111 is NaN.
__device__ __forceinline__ float dec(e4m3_t x) {
    const unsigned b = x.v;
    const unsigned s = (b & 0x80u) << 24;
    const unsigned e = (b >> 3) & 0xFu;
    const unsigned f = b & 0x7u;
    float v;
    if (e == 0xFu && f == 0x7u)
        v = __uint_as_float(0x7FC00000u);
    else if (e == 0)
        v = (float)f * 0x1p-9f;
    else
        v = __uint_as_float(((e + 120u) << 23) | (f << 20));
    return __uint_as_float(__float_as_uint(v) | s);
}
__device__ __forceinline__ float dec(float x) { return x; }
__device__ __forceinline__ double dec(double x) { return x; }
__device__ __forceinline__ float2 dec(float2 x) { return x; }
__device__ __forceinline__ double2 dec(double2 x) { return x; }

// Round a binary32 value to the nearest bfloat16 (ties to even), returned as a
// binary32 holding that bfloat16 value.  Finite inputs only.
__device__ __forceinline__ float round_bf16(float x) {
    const unsigned u = __float_as_uint(x);
    const unsigned bias = 0x7FFFu + ((u >> 16) & 1u);
    return __uint_as_float((u + bias) & 0xFFFF0000u);
}

// Read CNT consecutive elements starting at p as one (element-aligned) access.
template <typename X, int CNT, typename P>
__device__ __forceinline__ void vload(X (&v)[CNT], P p) {
    __builtin_memcpy(v, p, sizeof(X) * CNT);
}
template <typename X, int CNT, typename P>
__device__ __forceinline__ void vstore(P p, const X (&v)[CNT]) {
    __builtin_memcpy(p, v, sizeof(X) * CNT);
}
// One element through a pointer of any address space (vector structs have no
// assignment from address-space-qualified objects).
template <typename X, typename P>
__device__ __forceinline__ X ld1(P p) {
    X v;
    __builtin_memcpy(&v, p, sizeof(X));
    return v;
}
template <typename X, typename P>
__device__ __forceinline__ void st1(P p, const X& v) {
    __builtin_memcpy(p, &v, sizeof(X));
}

// Pointers in a named address space: 1 = global memory (the direct and
// variable-size kernels), 3 = LDS (the staged kernel).  Matrix pointers that
// the kernels read from memory (pointer arrays, var-size records) would
// otherwise be generic, and generic accesses compile to flat instructions
// (counted against both the vector-memory and the LDS counters).
template <typename X, int AS> struct SpacePtr;
template <typename X> struct SpacePtr<X, 1> { using type = __attribute__((address_space(1))) X*; };
template <typename X> struct SpacePtr<X, 3> { using type = __attribute__((address_space(3))) X*; };
template <int AS, typename X>
__device__ __forceinline__ typename SpacePtr<X, AS>::type in_space(X* p)
{
    return (typename SpacePtr<X, AS>::type)p;
}

// Epilogue of one entry: alpha * acc + beta * c (real or complex), with the
// special cases alpha == 0 (acc unused) and beta == 0 (c unused).
// a b + c in the precision of R (no promotion of binary32 operands).
__device__ __forceinline__ float fma_r(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_r(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T>
__device__ __forceinline__ T axpby(typename Tr<T>::R ar, typename Tr<T>::R ai, typename Tr<T>::R br,
                                   typename Tr<T>::R bi, bool a0, bool b0, typename Tr<T>::R accr,
                                   typename Tr<T>::R acci, const T& c)
{
    using R = typename Tr<T>::R;
    const R cr = re_of<T>(c), ci = im_of<T>(c);
    if (!Tr<T>::cplx) {
        R o;
        if (a0)
            o = b0 ? R(0) : br * cr;
        else if (b0)
            o = ar * accr;
        else
            o = fma_r(ar, accr, br * cr);
        return make_val<T>(o, R(0));
    }
    R tr = 0, ti = 0;
    if (!b0) {
        tr = fma_r(br, cr, -(bi * ci));
        ti = fma_r(br, ci, bi * cr);
    }
    if (!a0) {
        tr = fma_r(ar, accr, fma_r(-ai, acci, tr));
        ti = fma_r(ar, acci, fma_r(ai, accr, ti));
    }
    return make_val<T>(tr, ti);
}

// One lane's view of the matrix it serves in a tile.  Output register r of
// the lane holds C(i, j) with (i, j) = (orow[r], ij), or (ij, orow[r]) when
// the MFMA operands are swapped.
template <typename T, typename TI, int AS = 1>
struct LaneMat {
    typename SpacePtr<const TI, AS>::type A;
    typename SpacePtr<const TI, AS>::type B;
    typename SpacePtr<T, AS>::type C;
    int m, n, k;
    int64_t lda, ldb, ldc;
    float scale;   // sA * sB for scaled narrow inputs, 1 otherwise
    bool valid;
    // A vector of the k-contiguous operand (or of C's rows) may run up to 3
    // elements past the end of this matrix's row: set only when those
    // elements lie inside the caller's buffer (a later matrix of the same
    // strided batch); the extra elements are masked, never used or stored.
    bool overA, overB, overC;
};

// Per-lane constants of the packed tile layout.
template <int D, typename R>
struct LaneGeom {
    int g, c, sel, ij, kk0;
    bool keep[4];
    int orow[4];
    __device__ __forceinline__ LaneGeom() {
        const int lane = threadIdx.x & 63;
        g = lane >> 4;
        c = lane & 15;
        sel = c / D;
        ij = c % D;
        kk0 = (D / 4) * g;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int Rr = Mfma<R>::row(g, r);
            keep[r] = (Rr / D) == sel;
            orow[r] = Rr % D;
        }
    }
};

struct Scalars {
    bool a0, b0;
};

// Raw operand registers of U tiles (stored format, not yet decoded), so that
// the loads of one group can be in flight while another group computes.
template <typename T, typename TI, int D, int U>
struct TileRegs {
    TI va[U][D / 4];
    TI vb[U][D / 4];
    T cin[U][4];
};

// Issue the loads of U tiles: op(A) row ij and op(B) column ij of the lane's
// matrix at k-indices kk0 .. kk0+KB-1, and the lane's C entries when
// beta != 0.  Nothing here waits for the data.
//
// The loads are branch-free: every lane of a live tile issues the same
// loads, an entry outside its matrix reading the matrix's first element
// instead (tile_finish masks it to zero, or never stores it), and nothing is
// zero-filled here.  A register written under a lane mask while loads into it
// are in flight for other lanes forces the compiler to wait for every load
// of the wave; without masks the loads of all U tiles stay in flight
// together.  The caller's pointers must be valid whenever the tile is live
// (tiles past the batch carry a valid matrix's pointers with valid = false),
// except A and B when alpha == 0 or k == 0 (then they are not read).
//
// CALL: every tile loads its C entries (independent tiles); false: only the
// first (the U tiles are k-chunks of one output block).
template <typename T, typename TI, int D, int U, bool ACONT, bool BCONT, int AS, bool CALL = true>
__device__ __forceinline__ void tile_load(const LaneMat<T, TI, AS> (&mats)[U], const LaneGeom<D, typename Tr<T>::R>& L,
                                          bool a0, bool b0, TileRegs<T, TI, D, U>& t)
{
    using M = Mfma<typename Tr<T>::R>;
    constexpr int KB = D / 4;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const LaneMat<T, TI, AS>& mt = mats[u];
        const bool row_ok = L.ij < mt.m;
        const bool col_ok = L.ij < mt.n;
        // vector loads of the k-contiguous operands when k is a multiple of
        // the lane's k-run (each run then whole or past k) or the run may be
        // over-read, scalars otherwise; decided by a wave vote, so the choice
        // is uniform even when the lanes serve matrices of different sizes
        const bool kvec = (mt.k % KB) == 0;
        const bool vecA = __all(kvec || mt.overA);
        const bool vecB = __all(kvec || mt.overB);
        const bool vecC = __all((mt.m & 3) == 0 || mt.overC);
        if (!a0 && mt.k > 0) {
            if (ACONT) {
                const auto src = mt.A + L.ij * mt.lda + L.kk0;
                if (vecA) {
                    vload<TI, KB>(t.va[u], (row_ok && L.kk0 < mt.k) ? src : mt.A);
                } else {
#pragma unroll
                    for (int kb = 0; kb < KB; ++kb)
                        t.va[u][kb] = ld1<TI>((row_ok && L.kk0 + kb < mt.k) ? src + kb : mt.A);
                }
            } else {
#pragma unroll
                for (int kb = 0; kb < KB; ++kb)
                    t.va[u][kb] = ld1<TI>((row_ok && L.kk0 + kb < mt.k) ? mt.A + L.ij + (L.kk0 + kb) * mt.lda : mt.A);
            }
            if (BCONT) {
                const auto src = mt.B + L.ij * mt.ldb + L.kk0;
                if (vecB) {
                    vload<TI, KB>(t.vb[u], (col_ok && L.kk0 < mt.k) ? src : mt.B);
                } else {
#pragma unroll
                    for (int kb = 0; kb < KB; ++kb)
                        t.vb[u][kb] = ld1<TI>((col_ok && L.kk0 + kb < mt.k) ? src + kb : mt.B);
                }
            } else {
#pragma unroll
                for (int kb = 0; kb < KB; ++kb)
                    t.vb[u][kb] = ld1<TI>((col_ok && L.kk0 + kb < mt.k) ? mt.B + L.ij + (L.kk0 + kb) * mt.ldb : mt.B);
            }
        }
        if (!b0 && (CALL || u == 0)) {
            if (M::swap) {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    t.cin[u][r] = ld1<T>((row_ok && L.keep[r] && L.orow[r] < mt.n) ? mt.C + L.ij + L.orow[r] * mt.ldc
                                                                                    : mt.C);
            } else {
                // rows 4g'..4g'+3 of the lane's column: a vector when m is a
                // multiple of 4 (each lane's rows whole or past m)
                const auto cb = mt.C + L.ij * mt.ldc;
                if (M::rows_contig && vecC) {
                    vload<T, 4>(t.cin[u], (col_ok && L.keep[0] && L.orow[0] < mt.m) ? cb + L.orow[0] : mt.C);
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        t.cin[u][r] = ld1<T>((col_ok && L.keep[r] && L.orow[r] < mt.m) ? cb + L.orow[r] : mt.C);
                }
            }
        }
    }
}

// MFMA steps of one tile: the lane's op(A) row and op(B) column entries
// (stored format in va, vb; decoded here, masked to exact zeros outside the
// matrix or when !live) multiplied into acc_r (and acc_i for complex types).
// MODE 0: plain; MODE 1: BF16x3 (each binary32 operand split into bf16
// hi + lo; hi*hi + hi*lo + lo*hi accumulated in binary32).
template <typename T, typename TI, int MODE, int D, int AS>
__device__ __forceinline__ void tile_mma(const LaneMat<T, TI, AS>& mt, const LaneGeom<D, typename Tr<T>::R>& L,
                                         bool live, float a_conj, float b_conj, const TI (&va)[D / 4],
                                         const TI (&vb)[D / 4], typename Mfma<typename Tr<T>::R>::acc_t& acc_r,
                                         typename Mfma<typename Tr<T>::R>::acc_t& acc_i)
{
    using R = typename Tr<T>::R;
    using M = Mfma<R>;
    constexpr bool CPLX = Tr<T>::cplx;
    constexpr int KB = D / 4;
    const bool row_ok = L.ij < mt.m;
    const bool col_ok = L.ij < mt.n;
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
        // masked entries stay exact zeros (never a NaN from memory)
        const bool oka = live && row_ok && (L.kk0 + kb) < mt.k;
        const bool okb = live && col_ok && (L.kk0 + kb) < mt.k;
        const T da = oka ? dec(va[kb]) : make_val<T>(R(0), R(0));
        const T db = okb ? dec(vb[kb]) : make_val<T>(R(0), R(0));
        const R xar = re_of<T>(da), xbr = re_of<T>(db);
        const R xai = CPLX ? im_of<T>(da) * (R)a_conj : R(0);
        const R xbi = CPLX ? im_of<T>(db) * (R)b_conj : R(0);
        if (MODE == 1) {
            const R ah = (R)round_bf16((float)xar);
            const R al = (R)round_bf16((float)(xar - ah));
            const R bh = (R)round_bf16((float)xbr);
            const R bl = (R)round_bf16((float)(xbr - bh));
            acc_r = M::run(ah, bh, acc_r);
            acc_r = M::run(ah, bl, acc_r);
            acc_r = M::run(al, bh, acc_r);
        } else if (M::swap) {
            acc_r = M::run(xbr, xar, acc_r);
            if (CPLX) {
                acc_r = M::run(xbi, -xai, acc_r);
                acc_i = M::run(xbi, xar, acc_i);
                acc_i = M::run(xbr, xai, acc_i);
            }
        } else {
            acc_r = M::run(xar, xbr, acc_r);
            if (CPLX) {
                acc_r = M::run(-xai, xbi, acc_r);
                acc_i = M::run(xar, xbi, acc_i);
                acc_i = M::run(xai, xbr, acc_i);
            }
        }
    }
}

// Epilogue of one tile: C = alpha acc + beta C (cin: the lane's C entries as
// loaded) for the entries the lane keeps, written back to the matrix.
template <typename T, typename TI, int D, int AS>
__device__ __forceinline__ void tile_store(const LaneMat<T, TI, AS>& mt, const LaneGeom<D, typename Tr<T>::R>& L,
                                           const T& alpha, const T& beta, bool a0, bool b0,
                                           const typename Mfma<typename Tr<T>::R>::acc_t& acc_r,
                                           const typename Mfma<typename Tr<T>::R>::acc_t& acc_i, const T (&cin)[4])
{
    using R = typename Tr<T>::R;
    using M = Mfma<R>;
    constexpr bool CPLX = Tr<T>::cplx;
    const bool row_ok = L.ij < mt.m;
    const bool col_ok = L.ij < mt.n;
    const bool lane_ok = M::swap ? row_ok : col_ok;
    if (!(mt.valid && lane_ok)) return;
    // scaled narrow inputs: alpha * sA * sB applied as (alpha sA sB) * acc
    R ar = re_of<T>(alpha);
    const R ai = im_of<T>(alpha);
    const R br = re_of<T>(beta), bi = im_of<T>(beta);
    if (!CPLX && mt.scale != 1.0f) ar = ar * (R)mt.scale;
    T out[4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
        out[r] = axpby<T>(ar, ai, br, bi, a0, b0, acc_r[r], acc_i[r], cin[r]);
    if (M::swap) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (L.keep[r] && L.orow[r] < mt.n) st1<T>(mt.C + L.ij + L.orow[r] * mt.ldc, out[r]);
    } else {
        const auto cb = mt.C + L.ij * mt.ldc;
        if (M::rows_contig && L.keep[0] && (L.orow[0] + 3) < mt.m) {
            vstore<T, 4>(cb + L.orow[0], out);
        } else {
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (L.keep[r] && L.orow[r] < mt.m) st1<T>(cb + L.orow[r], out[r]);
        }
    }
}

// Decode, multiply (MFMA steps) and write back U tiles whose loads were
// issued by tile_load.
template <typename T, typename TI, int MODE, int D, int U, int AS>
__device__ __forceinline__ void tile_finish(const LaneMat<T, TI, AS> (&mats)[U], const LaneGeom<D, typename Tr<T>::R>& L,
                                            const T& alpha, const T& beta, bool a0, bool b0, float a_conj,
                                            float b_conj, const TileRegs<T, TI, D, U>& t)
{
    using acc_t = typename Mfma<typename Tr<T>::R>::acc_t;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const LaneMat<T, TI, AS>& mt = mats[u];
        acc_t acc_r = {0, 0, 0, 0};
        acc_t acc_i = {0, 0, 0, 0};
        // The MFMA chain runs whatever alpha is (with alpha == 0 every operand
        // is masked to zero): a branch around it separates the last MFMA from
        // the accumulator reads below by a block boundary, across which the
        // required wait states were found missing (reads of the last
        // accumulator row returned stale values).
        tile_mma<T, TI, MODE, D, AS>(mt, L, mt.valid && !a0, a_conj, b_conj, t.va[u], t.vb[u], acc_r, acc_i);
        tile_store<T, TI, D, AS>(mt, L, alpha, beta, a0, b0, acc_r, acc_i, t.cin[u]);
    }
}

// U tiles of one wavefront: all loads first, then the MFMA steps and epilogues.
template <typename T, typename TI, int MODE, int D, int U, bool ACONT, bool BCONT, int AS>
__device__ __forceinline__ void tile_group(const LaneMat<T, TI, AS> (&mats)[U], const LaneGeom<D, typename Tr<T>::R>& L,
                                           const T& alpha, const T& beta, bool a0, bool b0, float a_conj,
                                           float b_conj)
{
    TileRegs<T, TI, D, U> t;
    tile_load<T, TI, D, U, ACONT, BCONT>(mats, L, a0, b0, t);
    tile_finish<T, TI, MODE, D, U>(mats, L, alpha, beta, a0, b0, a_conj, b_conj, t);
}

// Tiles per wave per step: keep roughly 3-6 KB of operand loads in flight per
// wave whatever the element size and size class.
template <typename T, int D> struct Unroll {
    static constexpr int per_tile = 3 * 16 * D * (int)sizeof(T);   // A, B, C of the packed tile
    static constexpr int value = per_tile >= 6144 ? 1 : (per_tile >= 3072 ? 2 : 4);
};

// XCD-aware position of this wave in a persistent grid (gridDim.x % 8 == 0):
// each XCD takes runs of `chunk` consecutive work units.
__device__ __forceinline__ int64_t xcd_wave_index(int64_t chunk)
{
    const int64_t local = (int64_t)(blockIdx.x >> 3) * 4 + (threadIdx.x >> 6);
    const int64_t xcd = blockIdx.x & 7;
    return ((local / chunk) * 8 + xcd) * chunk + (local % chunk);
}

}  // namespace sbg
