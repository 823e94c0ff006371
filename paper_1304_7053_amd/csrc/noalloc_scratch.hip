// Device scratch of the allocation-free variable-size entry point
// (sbg_gemm_vbatched_ex_noalloc): the binning workspace of up to
// SBG_NOALLOC_MAX_BATCH matrices, held by every GPU the library runs on until
// the process ends.  Host code never uses the array's name as an address: the
// device address comes from hipGetSymbolAddress, once per device, with that
// device current.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "gemm_vbatched.h"

namespace sbg {

constexpr size_t NOALLOC_SCRATCH_BYTES = vbatched_workspace_bytes(SBG_NOALLOC_MAX_BATCH);

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

hipError_t noalloc_scratch(void** ptr, size_t* bytes)
{
    static std::mutex mu;
    static std::vector<void*> addr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(mu);
    if ((int)addr.size() <= dev) addr.resize(dev + 1, nullptr);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    *bytes = NOALLOC_SCRATCH_BYTES;
    return hipSuccess;
}

}  // namespace sbg
