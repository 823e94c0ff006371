// Host-only driver for the C-ABI layer (paper_1304_7053_amd/csrc/api.cpp:
// argument validation, quick returns, scalar classes, kernel planning),
// built with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_abi_fuzz.py and linked against stubs in place of the kernel
// launchers and the HIP runtime, so it runs without a GPU.  Every entry point
// is called with seeded random arguments drawn from boundary values: negative
// and huge sizes, leading dimensions and strides up to INT64_MAX, batch counts
// up to 2^62, null and misaligned pointers, invalid op characters, NaN and
// zero scalars.  Any out-of-bounds access, signed overflow or other undefined
// behaviour aborts the run.  The driver also checks that every call returns a
// defined status, that a rejected call names an argument position, and that
// an accepted call reached a launcher only with sizes inside the documented
// limits.  Prints "abi fuzz ok <calls> <accepted>" on success.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <type_traits>

#include "sbg.h"
#include "sbg_internal.h"

// ---- stubs: the HIP runtime calls the host layer makes ----------------------
extern "C" {
hipError_t hipGetDevice(int*) { return hipErrorNoDevice; }
hipError_t hipDeviceGetAttribute(int*, hipDeviceAttribute_t, int) { return hipErrorNoDevice; }
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* nb, const void*, int, size_t)
{
    *nb = 4;
    return hipSuccess;
}
}

// ---- stubs: the launchers (kernel translation units) -------------------------
namespace {
long g_launches = 0;
bool g_bad = false;

template <typename T>
void check_gemm(const sbg::GemmArgs<T>& a)
{
    ++g_launches;
    if (a.m < 0 || a.n < 0 || a.k < 0 || a.batch < 0) g_bad = true;
}
}  // namespace

namespace sbg {
template <> hipError_t launch_gemm<float>(const GemmArgs<float>& a, bool, hipStream_t) { check_gemm(a); return hipSuccess; }
template <> hipError_t launch_gemm<double>(const GemmArgs<double>& a, bool, hipStream_t) { check_gemm(a); return hipSuccess; }
template <> hipError_t launch_gemm<float2>(const GemmArgs<float2>& a, bool, hipStream_t) { check_gemm(a); return hipSuccess; }
template <> hipError_t launch_gemm<double2>(const GemmArgs<double2>& a, bool, hipStream_t) { check_gemm(a); return hipSuccess; }
template <> int describe_gemm<float>(const GemmArgs<float>&, bool, char* b, int n) { return snprintf(b, n, "stub"); }
template <> int describe_gemm<double>(const GemmArgs<double>&, bool, char* b, int n) { return snprintf(b, n, "stub"); }
template <> int describe_gemm<float2>(const GemmArgs<float2>&, bool, char* b, int n) { return snprintf(b, n, "stub"); }
template <> int describe_gemm<double2>(const GemmArgs<double2>&, bool, char* b, int n) { return snprintf(b, n, "stub"); }
template <> hipError_t launch_vbatched<float>(const GemmArgs<float>& a, hipStream_t) { check_gemm(a); return hipSuccess; }
template <> hipError_t launch_vbatched<double>(const GemmArgs<double>& a, hipStream_t) { check_gemm(a); return hipSuccess; }
template <> hipError_t launch_vbatched<float2>(const GemmArgs<float2>& a, hipStream_t) { check_gemm(a); return hipSuccess; }
template <> hipError_t launch_vbatched<double2>(const GemmArgs<double2>& a, hipStream_t) { check_gemm(a); return hipSuccess; }
hipError_t launch_gemm_ex(const GemmArgs<float>& a, int, int, int, hipStream_t) { check_gemm(a); return hipSuccess; }
template <> hipError_t launch_getrf<float>(const GetrfArgs<float>& g, hipStream_t)
{
    ++g_launches;
    if (g.n < 0 || g.n > 32 || g.batch < 0) g_bad = true;
    return hipSuccess;
}
template <> hipError_t launch_getrf<double>(const GetrfArgs<double>& g, hipStream_t)
{
    ++g_launches;
    if (g.n < 0 || g.n > 32 || g.batch < 0) g_bad = true;
    return hipSuccess;
}
hipError_t launch_quant_e4m3(const QuantArgs& q, bool, hipStream_t)
{
    ++g_launches;
    if (q.batch < 0) g_bad = true;
    return hipSuccess;
}
template <> hipError_t launch_trsm_small<float>(const TrsmArgs<float>& t, hipStream_t) { ++g_launches; if (t.size > 16) g_bad = true; return hipSuccess; }
template <> hipError_t launch_trsm_small<double>(const TrsmArgs<double>& t, hipStream_t) { ++g_launches; if (t.size > 16) g_bad = true; return hipSuccess; }
template <> hipError_t launch_trsm_small<float2>(const TrsmArgs<float2>& t, hipStream_t) { ++g_launches; if (t.size > 16) g_bad = true; return hipSuccess; }
template <> hipError_t launch_trsm_small<double2>(const TrsmArgs<double2>& t, hipStream_t) { ++g_launches; if (t.size > 16) g_bad = true; return hipSuccess; }
size_t vb_workspace_bytes(int64_t batch) { return batch < 0 ? 0 : (size_t)(64 + 144 * (uint64_t)batch); }
hipError_t noalloc_scratch(void** p, size_t* bytes)
{
    *p = nullptr;
    *bytes = 0;
    return hipErrorNoDevice;
}
}  // namespace sbg

// ---- random arguments ------------------------------------------------------------
namespace {
uint64_t g_seed = 13047053;
uint64_t rnd()
{
    g_seed = g_seed * 6364136223846793005ull + 1442695040888963407ull;
    return g_seed >> 17;
}
template <typename X, size_t N>
X pick(const X (&v)[N]) { return v[rnd() % N]; }

int rint_()
{
    static const int v[] = {std::numeric_limits<int>::min(), -7, -1, 0, 0, 1, 1, 2, 3, 4, 7, 8, 9, 15, 16, 16, 17,
                            31, 32, 33, 63, 64, 65, 100, 1000, 46341, 1 << 30, std::numeric_limits<int>::max()};
    return rnd() % 4 == 0 ? (int)(rnd() % 80) - 5 : pick(v);
}
int64_t r64()
{
    static const int64_t v[] = {std::numeric_limits<int64_t>::min(), -1, 0, 0, 1, 16, 256, 257, 1000, 65536,
                                (int64_t)1 << 31, (int64_t)1 << 40, (int64_t)1 << 62, std::numeric_limits<int64_t>::max()};
    return rnd() % 3 == 0 ? (int64_t)(rnd() % 5000) - 10 : pick(v);
}
int64_t rbatch()
{
    static const int64_t v[] = {-5, -1, 0, 1, 2, 3, 100, 100000, (int64_t)1 << 31, (int64_t)1 << 40, (int64_t)1 << 62};
    return pick(v);
}
char rop()
{
    static const char v[] = {'N', 'T', 'C', 'R', 'n', 't', 'c', 'r', 'X', '\0', 'L', 'U'};
    return pick(v);
}
char rside() { static const char v[] = {'L', 'R', 'l', 'r', 'N', 'X'}; return pick(v); }
char ruplo() { static const char v[] = {'L', 'U', 'l', 'u', 'N', 'X'}; return pick(v); }
char rdiag() { static const char v[] = {'N', 'U', 'n', 'u', 'T', 'X'}; return pick(v); }

// pointers: null, small fake device addresses (never dereferenced by the host
// layer), misaligned ones
alignas(64) unsigned char g_dummy[4096];
void* rptr()
{
    switch (rnd() % 5) {
        case 0: return nullptr;
        case 1: return g_dummy + 1;
        default: return g_dummy + 64 * (rnd() % 8);
    }
}
template <typename S>
const S* rscalar(S* store)
{
    static const double v[] = {0.0, 1.0, -0.5, 2.0, NAN, INFINITY};
    const double x = pick(v), y = pick(v);
    if constexpr (std::is_same<S, float>::value) *store = (float)x;
    else if constexpr (std::is_same<S, double>::value) *store = x;
    else if constexpr (std::is_same<S, sbg_cfloat>::value) { store->re = (float)x; store->im = (float)y; }
    else { store->re = x; store->im = y; }
    return rnd() % 16 == 0 ? nullptr : store;
}

long g_calls = 0, g_ok = 0;
void account(sbg_status_t st)
{
    ++g_calls;
    if (st == SBG_OK) {
        ++g_ok;
        return;
    }
    if (st != SBG_INVALID_VALUE && st != SBG_NOT_SUPPORTED && st != SBG_HIP_ERROR && st != SBG_WORKSPACE_TOO_SMALL) {
        std::printf("undefined status %d\n", (int)st);
        std::exit(3);
    }
    if (st == SBG_INVALID_VALUE && sbg_last_invalid_arg() <= 0) {
        std::printf("rejected call without an argument position\n");
        std::exit(4);
    }
}

// a leading dimension or stride that is usually consistent with its matrix
// (so the call gets past validation) and sometimes at the edge of int / int64
int ld_for(int rows)
{
    static const int pad[] = {0, 0, 1, 3, 16};
    const int r = rows > 1 ? rows : 1;
    return rnd() % 8 == 0 ? std::numeric_limits<int>::max() - (int)(rnd() % 4) : r + pick(pad);
}
int64_t stride_for(int64_t ld, int cols)
{
    const int64_t base = ld * (cols > 1 ? cols : 1);
    switch (rnd() % 8) {
        case 0: return 0;
        case 1: return (int64_t)1 << 62;
        case 2: return std::numeric_limits<int64_t>::max() - (int64_t)(rnd() % 4);
        default: return base + (int64_t)(rnd() % 5);
    }
}
template <typename S>
void strided_gemm(sbg_status_t (*f)(char, char, int, int, int, const S*, const S*, int, int64_t, const S*, int,
                                    int64_t, const S*, S*, int, int64_t, int64_t, void*))
{
    S al, be;
    if (rnd() % 2) {
        account(f(rop(), rop(), rint_(), rint_(), rint_(), rscalar(&al), (const S*)rptr(), rint_(), r64(),
                  (const S*)rptr(), rint_(), r64(), rscalar(&be), (S*)rptr(), rint_(), r64(), rbatch(), nullptr));
        return;
    }
    // consistent shapes: exercises the accepted paths' address arithmetic
    static const char ops[] = {'N', 'T', 'C'};
    static const int sz[] = {0, 1, 5, 16, 17, 33, 64, 65, 100};
    const char ta = pick(ops), tb = pick(ops);
    const int m = pick(sz), n = pick(sz), k = pick(sz);
    const int ra = ta == 'N' ? m : k, ca = ta == 'N' ? k : m;
    const int rb = tb == 'N' ? k : n, cb = tb == 'N' ? n : k;
    const int lda = ld_for(ra), ldb = ld_for(rb), ldc = ld_for(m);
    static const int64_t batches[] = {1, 2, 3, 1000, (int64_t)1 << 31, (int64_t)1 << 40, (int64_t)1 << 62};
    account(f(ta, tb, m, n, k, rscalar(&al), (const S*)(g_dummy + 64), lda, stride_for(lda, ca),
              (const S*)(g_dummy + 128), ldb, stride_for(ldb, cb), rscalar(&be), (S*)(g_dummy + 256), ldc,
              stride_for(ldc, n), pick(batches), nullptr));
}
template <typename S>
void pointer_gemm(sbg_status_t (*f)(char, char, int, int, int, const S*, const S* const*, int, const S* const*,
                                    int, const S*, S* const*, int, int64_t, void*))
{
    S al, be;
    account(f(rop(), rop(), rint_(), rint_(), rint_(), rscalar(&al), (const S* const*)rptr(), rint_(),
              (const S* const*)rptr(), rint_(), rscalar(&be), (S* const*)rptr(), rint_(), rbatch(), nullptr));
}
template <typename S>
void var_gemm(sbg_status_t (*f)(char, char, const int*, const int*, const int*, int, int, int, const S*,
                                const S* const*, const int*, const S* const*, const int*, const S*, S* const*,
                                const int*, int64_t, void*, size_t, void*))
{
    S al, be;
    account(f(rop(), rop(), (const int*)rptr(), (const int*)rptr(), (const int*)rptr(), rint_(), rint_(), rint_(),
              rscalar(&al), (const S* const*)rptr(), (const int*)rptr(), (const S* const*)rptr(),
              (const int*)rptr(), rscalar(&be), (S* const*)rptr(), (const int*)rptr(), rbatch(), rptr(),
              (size_t)r64(), nullptr));
}
template <typename S>
void gemv(sbg_status_t (*f)(char, int, int, const S*, const S*, int, int64_t, const S*, int, int64_t, const S*, S*,
                            int, int64_t, int64_t, void*))
{
    S al, be;
    account(f(rop(), rint_(), rint_(), rscalar(&al), (const S*)rptr(), rint_(), r64(), (const S*)rptr(), rint_(),
              r64(), rscalar(&be), (S*)rptr(), rint_(), r64(), rbatch(), nullptr));
}
template <typename S>
void trsm(sbg_status_t (*f)(char, char, char, char, int, int, const S*, const S*, int, int64_t, S*, int, int64_t,
                            int64_t, void*))
{
    S al;
    account(f(rside(), ruplo(), rop(), rdiag(), rint_(), rint_(), rscalar(&al), (const S*)rptr(), rint_(), r64(),
              (S*)rptr(), rint_(), r64(), rbatch(), nullptr));
}
template <typename S>
void getrf(sbg_status_t (*f)(int, S*, int, int64_t, int*, int64_t, int*, int64_t, void*))
{
    account(f(rint_(), (S*)rptr(), rint_(), r64(), (int*)rptr(), r64(), (int*)rptr(), rbatch(), nullptr));
}
}  // namespace

int main()
{
    char buf[512];
    for (int it = 0; it < 60000; ++it) {
        if (it % 1000 == 0) sbg_set_scalar_mode(rnd() % 2 ? SBG_SCALAR_DEVICE : SBG_SCALAR_HOST);
        switch (rnd() % 22) {
            case 0: strided_gemm<float>(sbg_sgemm_strided_batched); break;
            case 1: strided_gemm<double>(sbg_dgemm_strided_batched); break;
            case 2: strided_gemm<sbg_cfloat>(sbg_cgemm_strided_batched); break;
            case 3: strided_gemm<sbg_cdouble>(sbg_zgemm_strided_batched); break;
            case 4: pointer_gemm<float>(sbg_sgemm_batched); break;
            case 5: pointer_gemm<sbg_cdouble>(sbg_zgemm_batched); break;
            case 6: var_gemm<float>(sbg_sgemm_vbatched); break;
            case 7: var_gemm<sbg_cfloat>(sbg_cgemm_vbatched); break;
            case 8: {
                float al, be;
                account(sbg_gemm_strided_batched_ex(rop(), rop(), rint_(), rint_(), rint_(), rscalar(&al), rptr(),
                                                    rint_(), r64(), (const float*)rptr(), rptr(), rint_(), r64(),
                                                    (const float*)rptr(), rscalar(&be), (float*)rptr(), rint_(), r64(),
                                                    rbatch(), (sbg_datatype_t)(rnd() % 7 - 1),
                                                    (sbg_compute_mode_t)(rnd() % 4 - 1), nullptr));
                break;
            }
            case 9: {
                float al, be;
                account(sbg_gemm_vbatched_ex(rop(), rop(), (const int*)rptr(), (const int*)rptr(), (const int*)rptr(),
                                             rint_(), rint_(), rint_(), rscalar(&al), (const void* const*)rptr(),
                                             (const int*)rptr(), (const float*)rptr(), (const void* const*)rptr(),
                                             (const int*)rptr(), (const float*)rptr(), rscalar(&be),
                                             (float* const*)rptr(), (const int*)rptr(), rbatch(),
                                             (sbg_datatype_t)(rnd() % 7 - 1), (sbg_compute_mode_t)(rnd() % 4 - 1),
                                             rptr(), (size_t)r64(), nullptr));
                break;
            }
            case 10: {
                float al, be;
                account(sbg_gemm_vbatched_ex_noalloc(rop(), rop(), (const int*)rptr(), (const int*)rptr(),
                                                     (const int*)rptr(), rint_(), rint_(), rint_(), rscalar(&al),
                                                     (const void* const*)rptr(), (const int*)rptr(),
                                                     (const float*)rptr(), (const void* const*)rptr(),
                                                     (const int*)rptr(), (const float*)rptr(), rscalar(&be),
                                                     (float* const*)rptr(), (const int*)rptr(), rbatch(),
                                                     (sbg_datatype_t)(rnd() % 7 - 1),
                                                     (sbg_compute_mode_t)(rnd() % 4 - 1), nullptr));
                break;
            }
            case 11:
                account(sbg_quantize_e4m3_strided_batched(rint_(), rint_(), (const float*)rptr(), rint_(), r64(),
                                                          (unsigned char*)rptr(), rint_(), r64(), (float*)rptr(),
                                                          rbatch(), nullptr));
                break;
            case 12:
                account(sbg_quantize_e4m3_vbatched((const int*)rptr(), (const int*)rptr(), rint_(), rint_(),
                                                   (const float* const*)rptr(), (const int*)rptr(),
                                                   (unsigned char* const*)rptr(), (const int*)rptr(),
                                                   (float*)rptr(), rbatch(), nullptr));
                break;
            case 13: gemv<float>(sbg_sgemv_strided_batched); break;
            case 14: gemv<sbg_cdouble>(sbg_zgemv_strided_batched); break;
            case 15: trsm<float>(sbg_strsm_strided_batched); break;
            case 16: trsm<double>(sbg_dtrsm_strided_batched); break;
            case 17: trsm<sbg_cfloat>(sbg_ctrsm_strided_batched); break;
            case 18: getrf<float>(sbg_sgetrf_strided_batched); break;
            case 19: getrf<double>(sbg_dgetrf_strided_batched); break;
            case 20:
                sbg_describe_strided("sdczx"[rnd() % 5], rop(), rop(), rint_(), rint_(), rint_(), rint_(), r64(),
                                     rint_(), r64(), rint_(), r64(), rbatch(), buf, (int)(rnd() % 3 == 0 ? 0 : 512));
                ++g_calls;
                break;
            default:
                sbg_vbatched_workspace_size(rbatch());
                sbg_status_string((sbg_status_t)(rnd() % 9 - 2));
                ++g_calls;
                break;
        }
        if (g_bad) {
            std::printf("a launcher was reached with out-of-range sizes (call %d)\n", it);
            return 5;
        }
    }
    sbg_set_scalar_mode(SBG_SCALAR_HOST);
    std::printf("abi fuzz ok %ld %ld (launches %ld)\n", g_calls, g_ok, g_launches);
    return 0;
}
