// Fixed device scratch for the entry point that allocates nothing
// (mm_keyswitch_noalloc): a file-scope device array, one copy per GPU, whose
// address is looked up once per device with that device current.
//
// In host code the name `scratch` is only a host-side stand-in for the symbol;
// kernels receive the device address returned by hipGetSymbolAddress instead.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "kernels.hpp"

namespace mm {
namespace dev {

static __device__ __align__(256) uint64_t scratch[NOALLOC_SCRATCH_BYTES / sizeof(uint64_t)];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex scratch_lock;
void *scratch_ptr[MAX_DEVICES] = {};
}  // namespace

hipError_t noalloc_scratch_init(int device, void **out)
{
    *out = nullptr;
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(scratch_lock);
    if (!scratch_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        scratch_ptr[device] = p;
    }
    *out = scratch_ptr[device];
    return hipSuccess;
}

}  // namespace dev
}  // namespace mm
