// Mixed-precision kernel instances: A and B stored as float, mode 1 (see gemm_ex.hip).
#include "gemm_vbatched.h"
#include "gemm_staged.h"

namespace sbg {

hipError_t launch_ex_split3(const GemmArgs<float>& a, int form, hipStream_t s)
{
    if (form == 2) return launch_vbatched_t<float, float, 1>(a, s);
    return launch_direct<float, float, 1>(a, form == 1, s);
}

}  // namespace sbg
