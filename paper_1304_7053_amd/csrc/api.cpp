// C-ABI entry points of include/sbg.h: argument checking in BLAS (xerbla)
// order, quick returns, decoding of the op characters (Sec. 2) and of the
// storage rule of Sec. 5 into element strides, then one kernel launch.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdlib>
#include <mutex>
#include <unordered_map>
#include <string>
#include <vector>

#include "sbg.h"
#include "sbg_internal.h"

namespace sbg {

static thread_local sbg_scalar_mode_t tl_scalar_mode = SBG_SCALAR_HOST;
static thread_local int tl_last_invalid = 0;

int device_cu_count()
{
    static std::mutex mu;
    static std::vector<int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    std::lock_guard<std::mutex> lock(mu);
    if ((int)cache.size() <= dev) cache.resize(dev + 1, 0);
    if (cache[dev] == 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        cache[dev] = cus;
    }
    return cache[dev];
}

int resident_blocks_per_cu(const void* kernel)
{
    static std::mutex mu;
    static std::unordered_map<const void*, int> cache;
    {
        std::lock_guard<std::mutex> lock(mu);
        auto it = cache.find(kernel);
        if (it != cache.end()) return it->second;
    }
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, 256, 0) != hipSuccess || nb <= 0) nb = 1;
    std::lock_guard<std::mutex> lock(mu);
    cache[kernel] = nb;
    return nb;
}

Tuning& tuning_mut()
{
    static Tuning t = [] {
        Tuning v{0, 0, 2, 2048, 8192, false, 0, 0, 0, 1, 0};
        const auto env = [](const char* name, int lo, int hi, int& dst) {
            if (const char* e = std::getenv(name)) {
                const int x = std::atoi(e);
                if (x >= lo && x <= hi) dst = x;
            }
        };
        env("SBG_WG_PER_CU", 0, 32, v.wg_per_cu);
        env("SBG_XCD_CHUNK", 0, 1 << 20, v.xcd_chunk);
        env("SBG_STAGED", 0, 2, v.staged);
        env("SBG_TILE_BYTES", 256, 1 << 20, v.tile_bytes);
        env("SBG_TILE_BYTES16", 256, 1 << 20, v.tile_bytes16);
        env("SBG_PATH", 0, 3, v.path);
        env("SBG_UNROLL", 0, 8, v.unroll);
        env("SBG_GRID", 0, 1 << 20, v.grid);
        env("SBG_TABLE", 0, 1, v.table);
        env("SBG_BLOCKED", 0, 2, v.blocked);
        if (const char* e = std::getenv("SBG_PIPELINE")) v.pipeline = std::atoi(e) != 0;
        return v;
    }();
    return t;
}

const Tuning& tuning() { return tuning_mut(); }

VbDescribe& vb_describe()
{
    thread_local VbDescribe d;
    return d;
}

namespace {

enum Op { OP_N, OP_T, OP_C, OP_R, OP_BAD };

Op decode_op(char c)
{
    switch (c) {
    case 'N': case 'n': return OP_N;
    case 'T': case 't': return OP_T;
    case 'C': case 'c': return OP_C;
    case 'R': case 'r': return OP_R;
    default: return OP_BAD;
    }
}

bool transposes(Op o) { return o == OP_T || o == OP_C; }
bool conjugates(Op o) { return o == OP_C || o == OP_R; }

template <typename T> struct Scal;
template <> struct Scal<float> {
    using api_t = float;
    static float get(const float* p) { return *p; }
    static bool zero(float v) { return v == 0.f; }
    static bool one(float v) { return v == 1.f; }
};
template <> struct Scal<double> {
    using api_t = double;
    static double get(const double* p) { return *p; }
    static bool zero(double v) { return v == 0.0; }
    static bool one(double v) { return v == 1.0; }
};
template <> struct Scal<float2> {
    using api_t = sbg_cfloat;
    static float2 get(const sbg_cfloat* p) { return make_float2(p->re, p->im); }
    static bool zero(float2 v) { return v.x == 0.f && v.y == 0.f; }
    static bool one(float2 v) { return v.x == 1.f && v.y == 0.f; }
};
template <> struct Scal<double2> {
    using api_t = sbg_cdouble;
    static double2 get(const sbg_cdouble* p) { return make_double2(p->re, p->im); }
    static bool zero(double2 v) { return v.x == 0.0 && v.y == 0.0; }
    static bool one(double2 v) { return v.x == 1.0 && v.y == 0.0; }
};

// When non-null, run() stops after validation and writes the name of the
// kernel it would launch here instead of launching (thread-local).
thread_local char* tl_describe_buf = nullptr;
thread_local int tl_describe_len = 0;

sbg_status_t reject(int pos)
{
    tl_last_invalid = pos;
    return SBG_INVALID_VALUE;
}

// Common checks and launch for both batch forms.  `pos` gives the 1-based
// argument positions of (alpha, A, lda, B, ldb, beta, C, ldc, batch) in the
// public signature; strided-only arguments are checked by the caller.
struct Pos { int alpha, A, lda, B, ldb, beta, C, ldc, batch; };

// Validates in argument order and fills args; `launch` is false on a quick
// return.  Strides (strided form) are checked at positions lda+1, ldb+1, ldc+1.
template <typename T>
sbg_status_t prepare(char transa, char transb, int m, int n, int k,
                     const typename Scal<T>::api_t* alpha, const void* A, int lda,
                     const void* B, int ldb, const typename Scal<T>::api_t* beta,
                     const void* C, int ldc, int64_t batch, const Pos& pos,
                     GemmArgs<T>& args, bool& launch,
                     const int64_t* strides /* strideA, strideB, strideC or null */,
                     bool any_size /* sizes above 16 (the sub-blocked kernel) accepted */)
{
    launch = false;
    tl_last_invalid = 0;
    const Op oa = decode_op(transa), ob = decode_op(transb);
    if (oa == OP_BAD) return reject(1);
    if (ob == OP_BAD) return reject(2);
    if (m < 0) return reject(3);
    if (n < 0) return reject(4);
    if (k < 0) return reject(5);
    if (!alpha) return reject(pos.alpha);
    const bool host = tl_scalar_mode == SBG_SCALAR_HOST;
    T al{}, be{};
    if (host) al = Scal<T>::get(alpha);
    const bool need_ab = !host || (!Scal<T>::zero(al) && k > 0);
    const int rowsA = transposes(oa) ? k : m;
    const int rowsB = transposes(ob) ? n : k;
    const bool nonempty = m > 0 && n > 0 && batch > 0;
    if (need_ab && nonempty && !A) return reject(pos.A);
    if (lda < (rowsA > 1 ? rowsA : 1)) return reject(pos.lda);
    if (strides && strides[0] < 0) return reject(pos.lda + 1);
    if (need_ab && nonempty && !B) return reject(pos.B);
    if (ldb < (rowsB > 1 ? rowsB : 1)) return reject(pos.ldb);
    if (strides && strides[1] < 0) return reject(pos.ldb + 1);
    if (!beta) return reject(pos.beta);
    if (nonempty && !C) return reject(pos.C);
    if (ldc < (m > 1 ? m : 1)) return reject(pos.ldc);
    if (strides && (strides[2] < 0 || (batch > 1 && strides[2] < (int64_t)ldc * n)))
        return reject(pos.ldc + 1);
    if (batch < 0) return reject(pos.batch);
    if (!any_size && (m > 16 || n > 16 || k > 16)) return SBG_NOT_SUPPORTED;

    if (!nonempty) return SBG_OK;
    if (host) {
        be = Scal<T>::get(beta);
        if ((Scal<T>::zero(al) || k == 0) && Scal<T>::one(be)) return SBG_OK;
    }

    args.m = m;
    args.n = n;
    args.k = k;
    args.lda = lda;
    args.ldb = ldb;
    args.ldc = ldc;
    args.a_trans = transposes(oa);
    args.b_trans = transposes(ob);
    args.a_conj = conjugates(oa) ? -1.f : 1.f;
    args.b_conj = conjugates(ob) ? -1.f : 1.f;
    args.batch = batch;
    if (host) {
        args.alpha = al;
        args.beta = be;
        args.alpha_dev = nullptr;
        args.beta_dev = nullptr;
    } else {
        args.alpha = T{};
        args.beta = T{};
        args.alpha_dev = reinterpret_cast<const T*>(alpha);
        args.beta_dev = reinterpret_cast<const T*>(beta);
    }
    launch = true;
    return SBG_OK;
}

template <typename T>
sbg_status_t launch_plain(GemmArgs<T>& args, bool pointer_form, void* stream)
{
    if (tl_describe_buf) {
        describe_gemm<T>(args, pointer_form, tl_describe_buf, tl_describe_len);
        return SBG_OK;
    }
    hipError_t e = launch_gemm<T>(args, pointer_form, reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? SBG_OK : SBG_HIP_ERROR;
}

template <typename T>
sbg_status_t strided(char ta, char tb, int m, int n, int k, const typename Scal<T>::api_t* alpha,
                     const void* A, int lda, int64_t sA, const void* B, int ldb, int64_t sB,
                     const typename Scal<T>::api_t* beta, void* C, int ldc, int64_t sC,
                     int64_t batch, void* stream)
{
    GemmArgs<T> a{};
    a.A = A;
    a.B = B;
    a.C = static_cast<T*>(C);
    a.strideA = sA;
    a.strideB = sB;
    a.strideC = sC;
    const int64_t strides[3] = {sA, sB, sC};
    static const Pos pos = {6, 7, 8, 10, 11, 13, 14, 15, 17};
    bool launch = false;
    const sbg_status_t st = prepare<T>(ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, batch, pos, a,
                                       launch, strides, true);
    if (st != SBG_OK || !launch) return st;
    return launch_plain<T>(a, false, stream);
}

template <typename T>
sbg_status_t pointers(char ta, char tb, int m, int n, int k, const typename Scal<T>::api_t* alpha,
                      const void* Aarr, int lda, const void* Barr, int ldb,
                      const typename Scal<T>::api_t* beta, const void* Carr, int ldc,
                      int64_t batch, void* stream)
{
    GemmArgs<T> a{};
    a.Aarr = static_cast<const void* const*>(Aarr);
    a.Barr = static_cast<const void* const*>(Barr);
    a.Carr = static_cast<T* const*>(const_cast<void*>(Carr));
    static const Pos pos = {6, 7, 8, 9, 10, 11, 12, 13, 14};
    bool launch = false;
    const sbg_status_t st = prepare<T>(ta, tb, m, n, k, alpha, Aarr, lda, Barr, ldb, beta, Carr, ldc, batch, pos,
                                       a, launch, nullptr, true);
    if (st != SBG_OK || !launch) return st;
    return launch_plain<T>(a, true, stream);
}


// Common argument checks of the variable-size forms.  Positions: 1 transa,
// 2 transb, 3 d_m, 4 d_n, 5 d_k, 6 max_m, 7 max_n, 8 max_k, 9 alpha, 10 Aarray,
// 11 d_lda, then `extra` (1 for the scaleA of the _ex form), B..., beta, C...,
// batch, workspace, workspace_bytes.
struct VbPos { int alpha, A, lda, scaleA, B, ldb, scaleB, beta, C, ldc, batch, ws, wsb; };

template <typename T>
sbg_status_t vb_run(char transa, char transb, const int* dm, const int* dn, const int* dk, int max_m, int max_n,
                    int max_k, const void* alpha, const void* Aarr, const int* dlda, const float* scaleA,
                    const void* Barr, const int* dldb, const float* scaleB, const void* beta, const void* Carr,
                    const int* dldc, int64_t batch, void* ws, size_t ws_bytes, const VbPos& pos,
                    GemmArgs<T>& args, bool& launch, bool scales_required)
{
    launch = false;
    tl_last_invalid = 0;
    const Op oa = decode_op(transa), ob = decode_op(transb);
    if (oa == OP_BAD) return reject(1);
    if (ob == OP_BAD) return reject(2);
    const bool nonempty_b = batch > 0;
    if (nonempty_b && !dm) return reject(3);
    if (nonempty_b && !dn) return reject(4);
    if (nonempty_b && !dk) return reject(5);
    if (max_m < 0) return reject(6);
    if (max_n < 0) return reject(7);
    if (max_k < 0) return reject(8);
    if (!alpha) return reject(pos.alpha);
    const bool host = tl_scalar_mode == SBG_SCALAR_HOST;
    T al{}, be{};
    if (host) al = Scal<T>::get(static_cast<const typename Scal<T>::api_t*>(alpha));
    const bool nonempty = nonempty_b && max_m > 0 && max_n > 0;
    const bool need_ab = nonempty && (!host || (!Scal<T>::zero(al) && max_k > 0));
    if (need_ab && !Aarr) return reject(pos.A);
    if (nonempty && !dlda) return reject(pos.lda);
    if (pos.scaleA && ((scaleA == nullptr) != (scaleB == nullptr) || (scales_required && need_ab && !scaleA)))
        return reject(pos.scaleA);
    if (need_ab && !Barr) return reject(pos.B);
    if (nonempty && !dldb) return reject(pos.ldb);
    if (pos.scaleB && scales_required && need_ab && !scaleB) return reject(pos.scaleB);
    if (!beta) return reject(pos.beta);
    if (nonempty && !Carr) return reject(pos.C);
    if (nonempty && !dldc) return reject(pos.ldc);
    if (batch < 0 || batch > 0x7FFFFFFF) return reject(pos.batch);
    if (nonempty && (!ws || (reinterpret_cast<uintptr_t>(ws) & 15))) return reject(pos.ws);
    if (max_m > 16 || max_n > 16 || max_k > 16) return SBG_NOT_SUPPORTED;
    if (!nonempty) return SBG_OK;
    if (ws_bytes < vb_workspace_bytes(batch)) return SBG_WORKSPACE_TOO_SMALL;
    if (host) {
        be = Scal<T>::get(static_cast<const typename Scal<T>::api_t*>(beta));
        if ((Scal<T>::zero(al) || max_k == 0) && Scal<T>::one(be)) return SBG_OK;
    }
    args.dm = dm;
    args.dn = dn;
    args.dk = dk;
    args.dlda = dlda;
    args.dldb = dldb;
    args.dldc = dldc;
    args.max_m = max_m;
    args.max_n = max_n;
    args.max_k = max_k;
    args.ws = static_cast<int*>(ws);
    args.Aarr = static_cast<const void* const*>(Aarr);
    args.Barr = static_cast<const void* const*>(Barr);
    args.Carr = static_cast<T* const*>(const_cast<void*>(Carr));
    args.scaleA = scaleA;
    args.scaleB = scaleB;
    args.a_trans = transposes(oa);
    args.b_trans = transposes(ob);
    args.a_conj = conjugates(oa) ? -1.f : 1.f;
    args.b_conj = conjugates(ob) ? -1.f : 1.f;
    args.batch = batch;
    if (host) {
        args.alpha = al;
        args.beta = be;
        args.alpha_dev = nullptr;
        args.beta_dev = nullptr;
    } else {
        args.alpha_dev = static_cast<const T*>(alpha);
        args.beta_dev = static_cast<const T*>(beta);
    }
    launch = true;
    return SBG_OK;
}

template <typename T>
sbg_status_t vbatched(char ta, char tb, const int* dm, const int* dn, const int* dk, int max_m, int max_n, int max_k,
                      const void* alpha, const void* Aarr, const int* dlda, const void* Barr, const int* dldb,
                      const void* beta, const void* Carr, const int* dldc, int64_t batch, void* ws,
                      size_t ws_bytes, void* stream)
{
    GemmArgs<T> a{};
    static const VbPos pos = {9, 10, 11, 0, 12, 13, 0, 14, 15, 16, 17, 18, 19};
    bool launch = false;
    sbg_status_t st = vb_run<T>(ta, tb, dm, dn, dk, max_m, max_n, max_k, alpha, Aarr, dlda, nullptr, Barr, dldb,
                                nullptr, beta, Carr, dldc, batch, ws, ws_bytes, pos, a, launch, false);
    if (st != SBG_OK || !launch) return st;
    hipError_t e = launch_vbatched<T>(a, reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? SBG_OK : SBG_HIP_ERROR;
}

bool ab_type_ok(int t) { return t >= 0 && t <= 3; }

template <typename T> T real_val(double v);
template <> float real_val<float>(double v) { return (float)v; }
template <> double real_val<double>(double v) { return v; }
template <> float2 real_val<float2>(double v) { return make_float2((float)v, 0.f); }
template <> double2 real_val<double2>(double v) { return make_double2(v, 0.0); }

// Batched GEMV, y_p <- alpha op(A_p) x_p + beta y_p, in the paper's strided
// interface (its Sec. 9 proposes the interface for other BLAS routines,
// formulated on batched GEMM), run as one batched GEMM:
//  * op N with incy == 1: y is an m' x 1 matrix C; x the k x 1 matrix B
//    (incx == 1) or the transpose of a 1 x k matrix with leading dimension
//    incx;
//  * otherwise y^T = alpha x^T op(A)^T + beta y^T, a 1 x m' matrix with
//    leading dimension incy; op(A)^T is A read with the other op ('T' for
//    'N', 'N' for 'T', conjugated 'N' for 'C').  For op T and C this reads A
//    as the right operand with its k index contiguous (measured faster than
//    A as a k-contiguous left operand: 0.40 against 0.25 of HBM peak, f32).
// Positions: 1 trans, 2 m, 3 n, 4 alpha, 5 A, 6 lda, 7 strideA, 8 x, 9 incx,
// 10 stridex, 11 beta, 12 y, 13 incy, 14 stridey, 15 batch_count.
template <typename T>
sbg_status_t gemv(char trans, int m, int n, const typename Scal<T>::api_t* alpha, const void* A, int lda,
                  int64_t sA, const void* x, int incx, int64_t sx, const typename Scal<T>::api_t* beta, void* y,
                  int incy, int64_t sy, int64_t batch, void* stream)
{
    tl_last_invalid = 0;
    const Op op = decode_op(trans);
    if (op == OP_BAD || op == OP_R) return reject(1);
    if (m < 0) return reject(2);
    if (n < 0) return reject(3);
    if (!alpha) return reject(4);
    const bool host = tl_scalar_mode == SBG_SCALAR_HOST;
    T al{}, be{};
    if (host) al = Scal<T>::get(alpha);
    const int rows = op == OP_N ? m : n, cols = op == OP_N ? n : m;
    const bool nonempty = m > 0 && n > 0 && batch > 0;
    const bool need_ax = !host || !Scal<T>::zero(al);
    if (need_ax && nonempty && !A) return reject(5);
    if (lda < (m > 1 ? m : 1)) return reject(6);
    if (sA < 0) return reject(7);
    if (need_ax && nonempty && !x) return reject(8);
    if (incx < 1) return reject(9);
    if (sx < 0) return reject(10);
    if (!beta) return reject(11);
    if (nonempty && !y) return reject(12);
    if (incy < 1) return reject(13);
    // output vectors may not overlap
    if (sy < 0 || (batch > 1 && rows > 0 && sy < (int64_t)(rows - 1) * incy + 1)) return reject(14);
    if (batch < 0) return reject(15);
    // BLAS quick returns: an empty A leaves y untouched
    if (!nonempty) return SBG_OK;
    if (host) {
        be = Scal<T>::get(beta);
        if (Scal<T>::zero(al) && Scal<T>::one(be)) return SBG_OK;
    }
    GemmArgs<T> g{};
    g.k = cols;
    if (incy == 1 && op == OP_N) {
        g.m = rows;
        g.n = 1;
        g.A = A;
        g.lda = lda;
        g.strideA = sA;
        g.a_trans = op != OP_N;
        g.a_conj = op == OP_C ? -1.f : 1.f;
        g.B = x;
        g.b_trans = incx != 1;
        g.ldb = incx != 1 ? incx : (cols > 1 ? cols : 1);
        g.strideB = sx;
        g.b_conj = 1.f;
        g.ldc = rows;
    } else {
        g.m = 1;
        g.n = rows;
        g.A = x;
        g.a_trans = incx == 1;
        g.lda = incx == 1 ? (cols > 1 ? cols : 1) : incx;
        g.strideA = sx;
        g.a_conj = 1.f;
        g.B = A;
        g.ldb = lda;
        g.strideB = sA;
        g.b_trans = op == OP_N;
        g.b_conj = op == OP_C ? -1.f : 1.f;
        g.ldc = incy;
    }
    g.C = static_cast<T*>(y);
    g.strideC = sy;
    g.batch = batch;
    if (host) {
        g.alpha = al;
        g.beta = be;
    } else {
        g.alpha_dev = reinterpret_cast<const T*>(alpha);
        g.beta_dev = reinterpret_cast<const T*>(beta);
    }
    return launch_plain<T>(g, false, stream);
}

// Batched TRSM in the strided interface: side L solves op(A_p) X_p =
// alpha B_p, side R X_p op(A_p) = alpha B_p, with A_p triangular (uplo) and
// unit or non-unit diagonal; X_p overwrites B_p.  Formulated on batched GEMM
// as the paper suggests (Sec. 9): with the triangular order s <= 16 one
// launch of the substitution kernel; larger s is cut into diagonal blocks of
// 16 -- B is first scaled by alpha (a GEMM with k = 0), then each diagonal
// block is solved by the substitution kernel and the remaining rows (side L)
// or columns (side R) of B are updated by one batched GEMM with the solved
// block (alpha = -1, beta = 1).
// Positions: 1 side, 2 uplo, 3 transa, 4 diag, 5 m, 6 n, 7 alpha, 8 A, 9 lda,
// 10 strideA, 11 B, 12 ldb, 13 strideB, 14 batch_count.
template <typename T>
sbg_status_t getrf(int n, void* A, int lda, int64_t sA, int* ipiv, int64_t sP, int* info, int64_t batch,
                   void* stream)
{
    tl_last_invalid = 0;
    if (n < 0) return reject(1);
    if (n > 32) return SBG_NOT_SUPPORTED;
    const bool nonempty = n > 0 && batch > 0;
    if (nonempty && !A) return reject(2);
    if (lda < (n > 1 ? n : 1)) return reject(3);
    if (sA < 0 || (batch > 1 && sA < (int64_t)lda * n)) return reject(4);
    if (nonempty && !ipiv) return reject(5);
    if (sP < 0 || (batch > 1 && sP < n)) return reject(6);
    if (batch > 0 && !info) return reject(7);
    if (batch < 0) return reject(8);
    if (batch == 0) return SBG_OK;
    GetrfArgs<T> g{};
    g.n = n;
    g.A = static_cast<T*>(A);
    g.lda = lda;
    g.strideA = sA;
    g.ipiv = ipiv;
    g.strideP = sP;
    g.info = info;
    g.batch = batch;
    // n == 0 still launches: every info[p] is set to 0
    return launch_getrf<T>(g, reinterpret_cast<hipStream_t>(stream)) == hipSuccess ? SBG_OK : SBG_HIP_ERROR;
}

template <typename T>
sbg_status_t trsm(char side, char uplo, char transa, char diag, int m, int n,
                  const typename Scal<T>::api_t* alpha, const void* A, int lda, int64_t sA, void* B, int ldb,
                  int64_t sB, int64_t batch, void* stream)
{
    tl_last_invalid = 0;
    const bool left = side == 'L' || side == 'l';
    if (!left && side != 'R' && side != 'r') return reject(1);
    const bool up = uplo == 'U' || uplo == 'u';
    if (!up && uplo != 'L' && uplo != 'l') return reject(2);
    const Op op = decode_op(transa);
    if (op == OP_BAD || op == OP_R) return reject(3);
    const bool unit = diag == 'U' || diag == 'u';
    if (!unit && diag != 'N' && diag != 'n') return reject(4);
    if (m < 0) return reject(5);
    if (n < 0) return reject(6);
    if (!alpha) return reject(7);
    const bool host = tl_scalar_mode == SBG_SCALAR_HOST;
    T al{};
    if (host) al = Scal<T>::get(alpha);
    const int s = left ? m : n;
    const bool nonempty = m > 0 && n > 0 && batch > 0;
    if (nonempty && (!host || !Scal<T>::zero(al)) && !A) return reject(8);
    if (lda < (s > 1 ? s : 1)) return reject(9);
    if (sA < 0) return reject(10);
    if (nonempty && !B) return reject(11);
    if (ldb < (m > 1 ? m : 1)) return reject(12);
    if (sB < 0 || (batch > 1 && sB < (int64_t)ldb * n)) return reject(13);
    if (batch < 0) return reject(14);
    if (!nonempty) return SBG_OK;
    const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    T* Bp = static_cast<T*>(B);
    const T* Ap = static_cast<const T*>(A);
    // M, the matrix applied to each right-hand-side vector: op(A) for side L,
    // op(A)^T for side R; M(i, l) = A[l + lda i] when eff_trans
    const bool op_lower = (!up) == (op == OP_N);
    const bool lower = left ? op_lower : !op_lower;
    const bool eff_trans = left ? op != OP_N : op == OP_N;
    const bool conj = op == OP_C;
    TrsmArgs<T> t{};
    t.lower = lower;
    t.eff_trans = eff_trans;
    t.conj = conj;
    t.unit = unit;
    t.lda = lda;
    t.strideA = sA;
    t.strideB = sB;
    t.batch = batch;
    t.nv = left ? n : m;
    t.vec_elem = left ? 1 : ldb;     // element i of a vector
    t.vec_step = left ? ldb : 1;     // the next vector
    if (s <= 16) {
        t.size = s;
        t.A = Ap;
        t.B = Bp;
        if (host) t.alpha = al;
        else t.alpha_dev = reinterpret_cast<const T*>(alpha);
        return launch_trsm_small<T>(t, st) == hipSuccess ? SBG_OK : SBG_HIP_ERROR;
    }
    // B <- alpha B: C = alpha * 0 + beta C with k = 0 and beta = the caller's alpha
    {
        GemmArgs<T> g{};
        g.m = m;
        g.n = n;
        g.k = 0;
        g.A = Bp;
        g.B = Bp;
        g.lda = ldb;
        g.ldb = 1;
        g.ldc = ldb;
        g.C = Bp;
        g.strideC = sB;
        g.batch = batch;
        g.a_conj = g.b_conj = 1.f;
        g.alpha = real_val<T>(1.0);
        if (host) g.beta = al;
        else g.beta_dev = reinterpret_cast<const T*>(alpha);
        if (launch_gemm<T>(g, false, st) != hipSuccess) return SBG_HIP_ERROR;
        if (host && Scal<T>::zero(al)) return SBG_OK;   // B = 0; A not read
    }
    const int nb = (s + 15) / 16;
    for (int q = 0; q < nb; ++q) {
        const int b = lower ? q : nb - 1 - q;          // block in solve order
        const int r0 = 16 * b, rs = s - r0 < 16 ? s - r0 : 16;
        // the diagonal block: M(r0.., r0..) and the vectors' entries r0..
        t.size = rs;
        t.A = Ap + r0 + (int64_t)lda * r0;
        t.B = Bp + (left ? r0 : (int64_t)ldb * r0);
        t.alpha = real_val<T>(1.0);
        t.alpha_dev = nullptr;
        if (launch_trsm_small<T>(t, st) != hipSuccess) return SBG_HIP_ERROR;
        // the rest of the vectors' entries: after the block (lower M) or before it
        const int e0 = lower ? r0 + rs : 0;
        const int ecnt = lower ? s - (r0 + rs) : r0;
        if (ecnt == 0) continue;
        // M(e0.., r0..) as a stored sub-matrix: element (i, l) at
        // A[(e0 + i) + lda (r0 + l)], or A[(r0 + l) + lda (e0 + i)] when eff_trans
        const T* Mblk = eff_trans ? Ap + r0 + (int64_t)lda * e0 : Ap + e0 + (int64_t)lda * r0;
        GemmArgs<T> g{};
        g.batch = batch;
        g.alpha = real_val<T>(-1.0);
        g.beta = real_val<T>(1.0);
        g.strideA = left ? sA : sB;
        g.strideB = left ? sB : sA;
        g.strideC = sB;
        g.ldc = ldb;
        g.k = rs;
        if (left) {
            // B(e0.., :) -= M(e0.., r0..) X(r0.., :)
            g.m = ecnt;
            g.n = n;
            g.A = Mblk;
            g.lda = lda;
            g.a_trans = eff_trans;
            g.a_conj = conj ? -1.f : 1.f;
            g.B = Bp + r0;
            g.ldb = ldb;
            g.b_trans = false;
            g.b_conj = 1.f;
            g.C = Bp + e0;
        } else {
            // B(:, e0..) -= X(:, r0..) M(e0.., r0..)^T
            g.m = m;
            g.n = ecnt;
            g.A = Bp + (int64_t)ldb * r0;
            g.lda = ldb;
            g.a_trans = false;
            g.a_conj = 1.f;
            g.B = Mblk;
            g.ldb = lda;
            g.b_trans = !eff_trans;
            g.b_conj = conj ? -1.f : 1.f;
            g.C = Bp + (int64_t)ldb * e0;
        }
        if (launch_gemm<T>(g, false, st) != hipSuccess) return SBG_HIP_ERROR;
    }
    return SBG_OK;
}

// The variable-size mixed-precision call with a given workspace (positions of
// the workspace arguments in pos).
sbg_status_t vb_ex(char transa, char transb, const int* d_m, const int* d_n, const int* d_k, int max_m, int max_n,
                   int max_k, const float* alpha, const void* const* Aarray, const int* d_lda, const float* scaleA,
                   const void* const* Barray, const int* d_ldb, const float* scaleB, const float* beta,
                   float* const* Carray, const int* d_ldc, int64_t batch_count, sbg_datatype_t ab_type,
                   sbg_compute_mode_t mode, void* workspace, size_t workspace_bytes, const VbPos& pos, void* stream)
{
    GemmArgs<float> a{};
    bool launch = false;
    sbg_status_t st = vb_run<float>(transa, transb, d_m, d_n, d_k, max_m, max_n, max_k, alpha, Aarray, d_lda,
                                    scaleA, Barray, d_ldb, scaleB, beta, Carray, d_ldc, batch_count, workspace,
                                    workspace_bytes, pos, a, launch, ab_type == SBG_R_8F_E4M3);
    if (st != SBG_OK) return st;
    if (!ab_type_ok((int)ab_type)) return reject(20);
    if (mode != SBG_MODE_PLAIN && mode != SBG_MODE_BF16X3) return reject(21);
    if (mode == SBG_MODE_BF16X3 && ab_type != SBG_R_32F) return reject(21);
    if (!launch) return SBG_OK;
    hipError_t e = launch_gemm_ex(a, (int)ab_type, (int)mode, 2, reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? SBG_OK : SBG_HIP_ERROR;
}

}  // namespace
}  // namespace sbg

using sbg::pointers;
using sbg::strided;

extern "C" {

sbg_status_t sbg_sgemv_strided_batched(char trans, int m, int n, const float* alpha, const float* A, int lda,
    int64_t strideA, const float* x, int incx, int64_t stridex, const float* beta, float* y, int incy,
    int64_t stridey, int64_t batch_count, void* stream)
{
    return sbg::gemv<float>(trans, m, n, alpha, A, lda, strideA, x, incx, stridex, beta, y, incy, stridey,
                            batch_count, stream);
}

sbg_status_t sbg_sgetrf_strided_batched(int n, float* A, int lda, int64_t strideA, int* ipiv, int64_t strideP,
                                        int* info, int64_t batch_count, void* stream)
{
    return sbg::getrf<float>(n, A, lda, strideA, ipiv, strideP, info, batch_count, stream);
}

sbg_status_t sbg_dgetrf_strided_batched(int n, double* A, int lda, int64_t strideA, int* ipiv, int64_t strideP,
                                        int* info, int64_t batch_count, void* stream)
{
    return sbg::getrf<double>(n, A, lda, strideA, ipiv, strideP, info, batch_count, stream);
}

sbg_status_t sbg_strsm_strided_batched(char side, char uplo, char transa, char diag, int m, int n,
    const float* alpha, const float* A, int lda, int64_t strideA, float* B, int ldb, int64_t strideB,
    int64_t batch_count, void* stream)
{
    return sbg::trsm<float>(side, uplo, transa, diag, m, n, alpha, A, lda, strideA, B, ldb, strideB, batch_count,
                            stream);
}

sbg_status_t sbg_dgemv_strided_batched(char trans, int m, int n, const double* alpha, const double* A, int lda,
    int64_t strideA, const double* x, int incx, int64_t stridex, const double* beta, double* y, int incy,
    int64_t stridey, int64_t batch_count, void* stream)
{
    return sbg::gemv<double>(trans, m, n, alpha, A, lda, strideA, x, incx, stridex, beta, y, incy, stridey,
                            batch_count, stream);
}

sbg_status_t sbg_dtrsm_strided_batched(char side, char uplo, char transa, char diag, int m, int n,
    const double* alpha, const double* A, int lda, int64_t strideA, double* B, int ldb, int64_t strideB,
    int64_t batch_count, void* stream)
{
    return sbg::trsm<double>(side, uplo, transa, diag, m, n, alpha, A, lda, strideA, B, ldb, strideB, batch_count,
                            stream);
}

sbg_status_t sbg_cgemv_strided_batched(char trans, int m, int n, const sbg_cfloat* alpha, const sbg_cfloat* A, int lda,
    int64_t strideA, const sbg_cfloat* x, int incx, int64_t stridex, const sbg_cfloat* beta, sbg_cfloat* y, int incy,
    int64_t stridey, int64_t batch_count, void* stream)
{
    return sbg::gemv<float2>(trans, m, n, alpha, A, lda, strideA, x, incx, stridex, beta, y, incy, stridey,
                            batch_count, stream);
}

sbg_status_t sbg_ctrsm_strided_batched(char side, char uplo, char transa, char diag, int m, int n,
    const sbg_cfloat* alpha, const sbg_cfloat* A, int lda, int64_t strideA, sbg_cfloat* B, int ldb, int64_t strideB,
    int64_t batch_count, void* stream)
{
    return sbg::trsm<float2>(side, uplo, transa, diag, m, n, alpha, A, lda, strideA, B, ldb, strideB, batch_count,
                            stream);
}

sbg_status_t sbg_zgemv_strided_batched(char trans, int m, int n, const sbg_cdouble* alpha, const sbg_cdouble* A, int lda,
    int64_t strideA, const sbg_cdouble* x, int incx, int64_t stridex, const sbg_cdouble* beta, sbg_cdouble* y, int incy,
    int64_t stridey, int64_t batch_count, void* stream)
{
    return sbg::gemv<double2>(trans, m, n, alpha, A, lda, strideA, x, incx, stridex, beta, y, incy, stridey,
                            batch_count, stream);
}

sbg_status_t sbg_ztrsm_strided_batched(char side, char uplo, char transa, char diag, int m, int n,
    const sbg_cdouble* alpha, const sbg_cdouble* A, int lda, int64_t strideA, sbg_cdouble* B, int ldb, int64_t strideB,
    int64_t batch_count, void* stream)
{
    return sbg::trsm<double2>(side, uplo, transa, diag, m, n, alpha, A, lda, strideA, B, ldb, strideB, batch_count,
                            stream);
}

sbg_status_t sbg_sgemm_strided_batched(char ta, char tb, int m, int n, int k, const float* alpha,
    const float* A, int lda, int64_t sA, const float* B, int ldb, int64_t sB, const float* beta,
    float* C, int ldc, int64_t sC, int64_t batch, void* stream)
{
    return strided<float>(ta, tb, m, n, k, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, stream);
}

sbg_status_t sbg_dgemm_strided_batched(char ta, char tb, int m, int n, int k, const double* alpha,
    const double* A, int lda, int64_t sA, const double* B, int ldb, int64_t sB, const double* beta,
    double* C, int ldc, int64_t sC, int64_t batch, void* stream)
{
    return strided<double>(ta, tb, m, n, k, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, stream);
}

sbg_status_t sbg_cgemm_strided_batched(char ta, char tb, int m, int n, int k, const sbg_cfloat* alpha,
    const sbg_cfloat* A, int lda, int64_t sA, const sbg_cfloat* B, int ldb, int64_t sB,
    const sbg_cfloat* beta, sbg_cfloat* C, int ldc, int64_t sC, int64_t batch, void* stream)
{
    return strided<float2>(ta, tb, m, n, k, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, stream);
}

sbg_status_t sbg_zgemm_strided_batched(char ta, char tb, int m, int n, int k, const sbg_cdouble* alpha,
    const sbg_cdouble* A, int lda, int64_t sA, const sbg_cdouble* B, int ldb, int64_t sB,
    const sbg_cdouble* beta, sbg_cdouble* C, int ldc, int64_t sC, int64_t batch, void* stream)
{
    return strided<double2>(ta, tb, m, n, k, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, stream);
}

sbg_status_t sbg_sgemm_batched(char ta, char tb, int m, int n, int k, const float* alpha,
    const float* const* A, int lda, const float* const* B, int ldb, const float* beta,
    float* const* C, int ldc, int64_t batch, void* stream)
{
    return pointers<float>(ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, batch, stream);
}

sbg_status_t sbg_dgemm_batched(char ta, char tb, int m, int n, int k, const double* alpha,
    const double* const* A, int lda, const double* const* B, int ldb, const double* beta,
    double* const* C, int ldc, int64_t batch, void* stream)
{
    return pointers<double>(ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, batch, stream);
}

sbg_status_t sbg_cgemm_batched(char ta, char tb, int m, int n, int k, const sbg_cfloat* alpha,
    const sbg_cfloat* const* A, int lda, const sbg_cfloat* const* B, int ldb, const sbg_cfloat* beta,
    sbg_cfloat* const* C, int ldc, int64_t batch, void* stream)
{
    return pointers<float2>(ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, batch, stream);
}

sbg_status_t sbg_zgemm_batched(char ta, char tb, int m, int n, int k, const sbg_cdouble* alpha,
    const sbg_cdouble* const* A, int lda, const sbg_cdouble* const* B, int ldb, const sbg_cdouble* beta,
    sbg_cdouble* const* C, int ldc, int64_t batch, void* stream)
{
    return pointers<double2>(ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, batch, stream);
}

size_t sbg_vbatched_workspace_size(int64_t batch_count)
{
    return sbg::vb_workspace_bytes(batch_count);
}

#define SBG_VB_ENTRY(NAME, T, API_T)                                                                   \
    sbg_status_t NAME(char ta, char tb, const int* d_m, const int* d_n, const int* d_k, int max_m,    \
                      int max_n, int max_k, const API_T* alpha, const API_T* const* Aarray,            \
                      const int* d_lda, const API_T* const* Barray, const int* d_ldb, const API_T* beta, \
                      API_T* const* Carray, const int* d_ldc, int64_t batch_count, void* workspace,     \
                      size_t workspace_bytes, void* stream)                                             \
    {                                                                                                   \
        return sbg::vbatched<T>(ta, tb, d_m, d_n, d_k, max_m, max_n, max_k, alpha, Aarray, d_lda,      \
                                Barray, d_ldb, beta, Carray, d_ldc, batch_count, workspace,             \
                                workspace_bytes, stream);                                               \
    }
SBG_VB_ENTRY(sbg_sgemm_vbatched, float, float)
SBG_VB_ENTRY(sbg_dgemm_vbatched, double, double)
SBG_VB_ENTRY(sbg_cgemm_vbatched, float2, sbg_cfloat)
SBG_VB_ENTRY(sbg_zgemm_vbatched, double2, sbg_cdouble)
#undef SBG_VB_ENTRY

sbg_status_t sbg_gemm_strided_batched_ex(char transa, char transb, int m, int n, int k, const float* alpha,
    const void* A, int lda, int64_t strideA, const float* scaleA, const void* B, int ldb, int64_t strideB,
    const float* scaleB, const float* beta, float* C, int ldc, int64_t strideC, int64_t batch_count,
    sbg_datatype_t ab_type, sbg_compute_mode_t mode, void* stream)
{
    // positions: 1 transa 2 transb 3 m 4 n 5 k 6 alpha 7 A 8 lda 9 strideA 10 scaleA 11 B 12 ldb
    // 13 strideB 14 scaleB 15 beta 16 C 17 ldc 18 strideC 19 batch_count 20 ab_type 21 mode
    // (the GEMM arguments are checked first, then scales, type and mode)
    sbg::GemmArgs<float> a{};
    a.A = A;
    a.B = B;
    a.C = C;
    a.strideA = strideA;
    a.strideB = strideB;
    a.strideC = strideC;
    const int64_t strides[3] = {strideA, strideB, strideC};
    static const sbg::Pos pos = {6, 7, 8, 11, 12, 15, 16, 17, 19};
    bool launch = false;
    const sbg_status_t st = sbg::prepare<float>(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                                                batch_count, pos, a, launch, strides, false);
    if (st != SBG_OK) return st;
    if ((scaleA == nullptr) != (scaleB == nullptr)) return sbg::reject(scaleA ? 14 : 10);
    if (ab_type == SBG_R_8F_E4M3 && !scaleA) return sbg::reject(10);
    if (!sbg::ab_type_ok((int)ab_type)) return sbg::reject(20);
    if (mode != SBG_MODE_PLAIN && mode != SBG_MODE_BF16X3) return sbg::reject(21);
    if (mode == SBG_MODE_BF16X3 && ab_type != SBG_R_32F) return sbg::reject(21);
    if (!launch) return SBG_OK;
    a.scaleA = scaleA;
    a.scaleB = scaleB;
    hipError_t e = sbg::launch_gemm_ex(a, (int)ab_type, (int)mode, 0, reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? SBG_OK : SBG_HIP_ERROR;
}


sbg_status_t sbg_gemm_vbatched_ex(char transa, char transb, const int* d_m, const int* d_n, const int* d_k,
    int max_m, int max_n, int max_k, const float* alpha, const void* const* Aarray, const int* d_lda,
    const float* scaleA, const void* const* Barray, const int* d_ldb, const float* scaleB, const float* beta,
    float* const* Carray, const int* d_ldc, int64_t batch_count, sbg_datatype_t ab_type, sbg_compute_mode_t mode,
    void* workspace, size_t workspace_bytes, void* stream)
{
    // positions: 1-8 as sbg_?gemm_vbatched, 9 alpha 10 Aarray 11 d_lda 12 scaleA 13 Barray 14 d_ldb
    // 15 scaleB 16 beta 17 Carray 18 d_ldc 19 batch_count 20 ab_type 21 mode 22 workspace 23 workspace_bytes
    static const sbg::VbPos pos = {9, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19, 22, 23};
    return sbg::vb_ex(transa, transb, d_m, d_n, d_k, max_m, max_n, max_k, alpha, Aarray, d_lda, scaleA, Barray,
                      d_ldb, scaleB, beta, Carray, d_ldc, batch_count, ab_type, mode, workspace, workspace_bytes,
                      pos, stream);
}

sbg_status_t sbg_gemm_vbatched_ex_noalloc(char transa, char transb, const int* d_m, const int* d_n,
    const int* d_k, int max_m, int max_n, int max_k, const float* alpha, const void* const* Aarray,
    const int* d_lda, const float* scaleA, const void* const* Barray, const int* d_ldb, const float* scaleB,
    const float* beta, float* const* Carray, const int* d_ldc, int64_t batch_count, sbg_datatype_t ab_type,
    sbg_compute_mode_t mode, void* stream)
{
    // the library's scratch replaces the workspace (never null, 256-byte
    // aligned); a batch above SBG_NOALLOC_MAX_BATCH finds it too small
    void* ws = nullptr;
    size_t ws_bytes = 0;
    if (sbg::noalloc_scratch(&ws, &ws_bytes) != hipSuccess) return SBG_HIP_ERROR;
    static const sbg::VbPos pos = {9, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19, 0, 0};
    return sbg::vb_ex(transa, transb, d_m, d_n, d_k, max_m, max_n, max_k, alpha, Aarray, d_lda, scaleA, Barray,
                      d_ldb, scaleB, beta, Carray, d_ldc, batch_count, ab_type, mode, ws, ws_bytes, pos, stream);
}

sbg_status_t sbg_quantize_e4m3_strided_batched(int rows, int cols, const float* X, int ldx, int64_t strideX,
    unsigned char* Q, int ldq, int64_t strideQ, float* scales, int64_t batch_count, void* stream)
{
    sbg::tl_last_invalid = 0;
    if (rows < 0) return sbg::reject(1);
    if (cols < 0) return sbg::reject(2);
    const bool nonempty = rows > 0 && cols > 0 && batch_count > 0;
    if (nonempty && !X) return sbg::reject(3);
    if (ldx < (rows > 1 ? rows : 1)) return sbg::reject(4);
    if (strideX < 0 || (batch_count > 1 && strideX < (int64_t)ldx * cols && strideX != 0)) return sbg::reject(5);
    if (nonempty && !Q) return sbg::reject(6);
    if (ldq < (rows > 1 ? rows : 1)) return sbg::reject(7);
    if (strideQ < 0 || (batch_count > 1 && strideQ < (int64_t)ldq * cols)) return sbg::reject(8);
    if (batch_count > 0 && !scales) return sbg::reject(9);
    if (batch_count < 0) return sbg::reject(10);
    if (rows > 16 || cols > 16) return SBG_NOT_SUPPORTED;
    if (batch_count == 0) return SBG_OK;
    sbg::QuantArgs q{};
    q.rows = rows;
    q.cols = cols;
    q.X = X;
    q.ldx = ldx;
    q.strideX = strideX;
    q.Q = Q;
    q.ldq = ldq;
    q.strideQ = strideQ;
    q.scales = scales;
    q.batch = batch_count;
    hipError_t e = sbg::launch_quant_e4m3(q, false, reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? SBG_OK : SBG_HIP_ERROR;
}

sbg_status_t sbg_quantize_e4m3_vbatched(const int* d_rows, const int* d_cols, int max_rows, int max_cols,
    const float* const* Xarray, const int* d_ldx, unsigned char* const* Qarray, const int* d_ldq, float* scales,
    int64_t batch_count, void* stream)
{
    sbg::tl_last_invalid = 0;
    const bool nonempty = batch_count > 0;
    if (nonempty && !d_rows) return sbg::reject(1);
    if (nonempty && !d_cols) return sbg::reject(2);
    if (max_rows < 0) return sbg::reject(3);
    if (max_cols < 0) return sbg::reject(4);
    if (nonempty && !Xarray) return sbg::reject(5);
    if (nonempty && !d_ldx) return sbg::reject(6);
    if (nonempty && !Qarray) return sbg::reject(7);
    if (nonempty && !d_ldq) return sbg::reject(8);
    if (nonempty && !scales) return sbg::reject(9);
    if (batch_count < 0) return sbg::reject(10);
    if (max_rows > 16 || max_cols > 16) return SBG_NOT_SUPPORTED;
    if (!nonempty) return SBG_OK;
    sbg::QuantArgs q{};
    q.drows = d_rows;
    q.dcols = d_cols;
    q.max_rows = max_rows;
    q.max_cols = max_cols;
    q.Xarr = Xarray;
    q.dldx = d_ldx;
    q.Qarr = Qarray;
    q.dldq = d_ldq;
    q.scales = scales;
    q.batch = batch_count;
    hipError_t e = sbg::launch_quant_e4m3(q, true, reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? SBG_OK : SBG_HIP_ERROR;
}

int sbg_describe_strided(char prefix, char transa, char transb, int m, int n, int k, int lda,
                         int64_t strideA, int ldb, int64_t strideB, int ldc, int64_t strideC,
                         int64_t batch_count, char* buf, int buflen)
{
    if (!buf || buflen <= 0) return -1;
    buf[0] = 0;
    // fake, never dereferenced operand addresses: the describe path returns
    // before any launch
    const double one[2] = {1.0, 0.0}, half[2] = {0.5, 0.0};
    const float onef[2] = {1.f, 0.f}, halff[2] = {0.5f, 0.f};
    void* fake = reinterpret_cast<void*>(static_cast<uintptr_t>(256));
    sbg::tl_describe_buf = buf;
    sbg::tl_describe_len = buflen;
    sbg_status_t st = SBG_INVALID_VALUE;
    switch (prefix) {
    case 's': st = sbg_sgemm_strided_batched(transa, transb, m, n, k, onef, (const float*)fake, lda, strideA,
                   (const float*)fake, ldb, strideB, halff, (float*)fake, ldc, strideC, batch_count, nullptr); break;
    case 'd': st = sbg_dgemm_strided_batched(transa, transb, m, n, k, one, (const double*)fake, lda, strideA,
                   (const double*)fake, ldb, strideB, half, (double*)fake, ldc, strideC, batch_count, nullptr); break;
    case 'c': st = sbg_cgemm_strided_batched(transa, transb, m, n, k, (const sbg_cfloat*)onef,
                   (const sbg_cfloat*)fake, lda, strideA, (const sbg_cfloat*)fake, ldb, strideB,
                   (const sbg_cfloat*)halff, (sbg_cfloat*)fake, ldc, strideC, batch_count, nullptr); break;
    case 'z': st = sbg_zgemm_strided_batched(transa, transb, m, n, k, (const sbg_cdouble*)one,
                   (const sbg_cdouble*)fake, lda, strideA, (const sbg_cdouble*)fake, ldb, strideB,
                   (const sbg_cdouble*)half, (sbg_cdouble*)fake, ldc, strideC, batch_count, nullptr); break;
    default: break;
    }
    sbg::tl_describe_buf = nullptr;
    sbg::tl_describe_len = 0;
    return st == SBG_OK && buf[0] ? 0 : -1;
}

int sbg_describe_vbatched(char prefix, char transa, char transb, int max_m, int max_n, int max_k,
                          int64_t batch_count, sbg_datatype_t ab_type, sbg_compute_mode_t mode, char* buf,
                          int buflen)
{
    if (!buf || buflen <= 0) return -1;
    buf[0] = 0;
    if (prefix != 's' && (ab_type != SBG_R_32F || mode != SBG_MODE_PLAIN)) return -1;
    // fake, never dereferenced device addresses (16-byte aligned): the
    // describe path returns before any launch
    void* fake = reinterpret_cast<void*>(static_cast<uintptr_t>(256));
    const int* di = static_cast<const int*>(fake);
    const double one[2] = {1.5, 0.0}, half[2] = {0.5, 0.0};
    const float onef[2] = {1.5f, 0.f}, halff[2] = {0.5f, 0.f};
    const size_t big = ~size_t(0);
    sbg::VbDescribe& ds = sbg::vb_describe();
    ds.buf = buf;
    ds.len = buflen;
    sbg_status_t st = SBG_INVALID_VALUE;
    switch (prefix) {
    case 's':
        st = sbg_gemm_vbatched_ex(transa, transb, di, di, di, max_m, max_n, max_k, onef,
                                  static_cast<const void* const*>(fake), di, static_cast<const float*>(fake),
                                  static_cast<const void* const*>(fake), di, static_cast<const float*>(fake), halff,
                                  static_cast<float* const*>(fake), di, batch_count, ab_type, mode, fake, big,
                                  nullptr);
        break;
    case 'd':
        st = sbg_dgemm_vbatched(transa, transb, di, di, di, max_m, max_n, max_k, one,
                                static_cast<const double* const*>(fake), di, static_cast<const double* const*>(fake),
                                di, half, static_cast<double* const*>(fake), di, batch_count, fake, big, nullptr);
        break;
    case 'c':
        st = sbg_cgemm_vbatched(transa, transb, di, di, di, max_m, max_n, max_k,
                                reinterpret_cast<const sbg_cfloat*>(onef),
                                static_cast<const sbg_cfloat* const*>(fake), di,
                                static_cast<const sbg_cfloat* const*>(fake), di,
                                reinterpret_cast<const sbg_cfloat*>(halff), static_cast<sbg_cfloat* const*>(fake), di,
                                batch_count, fake, big, nullptr);
        break;
    case 'z':
        st = sbg_zgemm_vbatched(transa, transb, di, di, di, max_m, max_n, max_k,
                                reinterpret_cast<const sbg_cdouble*>(one),
                                static_cast<const sbg_cdouble* const*>(fake), di,
                                static_cast<const sbg_cdouble* const*>(fake), di,
                                reinterpret_cast<const sbg_cdouble*>(half), static_cast<sbg_cdouble* const*>(fake),
                                di, batch_count, fake, big, nullptr);
        break;
    default: break;
    }
    ds.buf = nullptr;
    ds.len = 0;
    return st == SBG_OK && buf[0] ? 0 : -1;
}

namespace {
struct Knob {
    const char* name;
    int lo, hi;
    int sbg::Tuning::*field;
};
const Knob kKnobs[] = {
    {"wg_per_cu", 0, 32, &sbg::Tuning::wg_per_cu},
    {"xcd_chunk", 0, 1 << 20, &sbg::Tuning::xcd_chunk},
    {"staged", 0, 2, &sbg::Tuning::staged},
    {"tile_bytes", 256, 1 << 20, &sbg::Tuning::tile_bytes},
    {"tile_bytes16", 256, 1 << 20, &sbg::Tuning::tile_bytes16},
    {"path", 0, 3, &sbg::Tuning::path},
    {"unroll", 0, 8, &sbg::Tuning::unroll},
    {"grid", 0, 1 << 20, &sbg::Tuning::grid},
    {"table", 0, 1, &sbg::Tuning::table},
    {"blocked", 0, 2, &sbg::Tuning::blocked},
};
}  // namespace

int sbg_set_tuning(const char* key, int value)
{
    if (!key) return -1;
    sbg::Tuning& t = sbg::tuning_mut();
    const std::string k(key);
    if (k == "pipeline") {
        const int old = t.pipeline ? 1 : 0;
        t.pipeline = value != 0;
        return old;
    }
    for (const Knob& kn : kKnobs) {
        if (k == kn.name) {
            if (value < kn.lo || value > kn.hi) return -1;
            const int old = t.*kn.field;
            t.*kn.field = value;
            return old;
        }
    }
    return -1;
}

int sbg_get_tuning(const char* key)
{
    if (!key) return -1;
    const sbg::Tuning& t = sbg::tuning();
    const std::string k(key);
    if (k == "pipeline") return t.pipeline ? 1 : 0;
    for (const Knob& kn : kKnobs)
        if (k == kn.name) return t.*kn.field;
    return -1;
}

int sbg_tuned_table_info(char* buf, int buflen)
{
    return sbg::tuned_table_info(buf, buflen);
}

void sbg_set_scalar_mode(sbg_scalar_mode_t mode)
{
    sbg::tl_scalar_mode = (mode == SBG_SCALAR_DEVICE) ? SBG_SCALAR_DEVICE : SBG_SCALAR_HOST;
}

sbg_scalar_mode_t sbg_get_scalar_mode(void) { return sbg::tl_scalar_mode; }

int sbg_last_invalid_arg(void) { return sbg::tl_last_invalid; }

const char* sbg_status_string(sbg_status_t s)
{
    switch (s) {
    case SBG_OK: return "success";
    case SBG_INVALID_VALUE: return "invalid argument (see sbg_last_invalid_arg)";
    case SBG_NOT_SUPPORTED: return "not supported (a size above 16)";
    case SBG_HIP_ERROR: return "HIP runtime error at launch";
    case SBG_WORKSPACE_TOO_SMALL: return "workspace too small";
    }
    return "unknown status";
}

int sbg_version(void) { return 100; }

}  // extern "C"
