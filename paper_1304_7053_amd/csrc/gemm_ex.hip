// Mixed-precision dispatch (binary32 accumulation and C): bf16, fp16 and
// fp8-e4m3 inputs, and the BF16x3 split mode on binary32 inputs, for the
// strided, pointer-array and variable-size forms.  The instances live in
// one translation unit per input format (gemm_ex_*.hip) to build in parallel.
#include "sbg_internal.h"

namespace sbg {

hipError_t launch_ex_bf16(const GemmArgs<float>& a, int form, hipStream_t s);
hipError_t launch_ex_f16(const GemmArgs<float>& a, int form, hipStream_t s);
hipError_t launch_ex_e4m3(const GemmArgs<float>& a, int form, hipStream_t s);
hipError_t launch_ex_split3(const GemmArgs<float>& a, int form, hipStream_t s);

hipError_t launch_gemm_ex(const GemmArgs<float>& a, int ab_type, int mode, int form, hipStream_t s)
{
    if (mode == 1) return launch_ex_split3(a, form, s);   // BF16x3 on binary32 inputs
    switch (ab_type) {
    case 1: return launch_ex_bf16(a, form, s);
    case 2: return launch_ex_f16(a, form, s);
    case 3: return launch_ex_e4m3(a, form, s);
    default: break;
    }
    // binary32 inputs, plain mode: the S kernels themselves
    if (form == 2) return launch_vbatched<float>(a, s);
    return launch_gemm<float>(a, form == 1, s);
}

}  // namespace sbg
