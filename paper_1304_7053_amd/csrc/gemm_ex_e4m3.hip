// Mixed-precision kernel instances: A and B stored as e4m3_t, mode 0 (see gemm_ex.hip).
#include "gemm_vbatched.h"
#include "gemm_vbteam.h"
#include "gemm_staged.h"

namespace sbg {

hipError_t launch_ex_e4m3(const GemmArgs<float>& a, int form, hipStream_t s)
{
    if (form == 2) return launch_vbatched_t<float, e4m3_t, 0>(a, s);
    return launch_direct<float, e4m3_t, 0>(a, form == 1, s);
}

}  // namespace sbg
