// Mixed-precision instances (binary32 accumulation and C): bf16, fp16 and
// fp8-e4m3 inputs, and the BF16x3 split mode on binary32 inputs, for the
// strided, pointer-array and variable-size forms.
#include "gemm_vbatched.h"

namespace sbg {

namespace {

template <typename TI, int MODE>
hipError_t run_form(const GemmArgs<float>& a, int form, hipStream_t s)
{
    if (form == 2) return launch_vbatched_t<float, TI, MODE>(a, s);
    return launch_direct<float, TI, MODE>(a, form == 1, s);
}

}  // namespace

hipError_t launch_gemm_ex(const GemmArgs<float>& a, int ab_type, int mode, int form, hipStream_t s)
{
    if (mode == 1) return run_form<float, 1>(a, form, s);   // BF16x3 on binary32 inputs
    switch (ab_type) {
    case 1: return run_form<bf16_t, 0>(a, form, s);
    case 2: return run_form<f16_t, 0>(a, form, s);
    case 3: return run_form<e4m3_t, 0>(a, form, s);
    default: break;
    }
    // binary32 inputs, plain mode: the S kernels themselves
    if (form == 2) return launch_vbatched<float>(a, s);
    return launch_direct<float, float, 0>(a, form == 1, s);
}

}  // namespace sbg
