// Device scratch for the entry point that allocates nothing
// (nvsm_reconstruct_noalloc): a fixed array in the library's device data,
// one copy per GPU, present from the first look-up until the process ends.
//
// In host code the name `scratch` stands for the array but is not its
// device address.  scratch_setup looks the address up once per device
// (with that device current) and keeps it; everything else uses the kept
// address: it is what the kernels receive as their workspace.
#include <hip/hip_runtime.h>

#include <mutex>

#include "scratch.hpp"

static __device__ __align__(256) unsigned char scratch[nvsm::SCRATCH_BYTES];

namespace nvsm {

namespace {
std::mutex g_mu;
void *g_ptr[SCRATCH_MAX_DEVICES] = {};
}  // namespace

hipError_t scratch_setup(int device) {
    if (device < 0 || device >= SCRATCH_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_ptr[device]) return hipSuccess;
    int prev = 0;
    hipError_t e = hipGetDevice(&prev);
    if (e != hipSuccess) return e;
    if ((e = hipSetDevice(device)) != hipSuccess) return e;
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    const hipError_t r = hipSetDevice(prev);
    if (e != hipSuccess) return e;
    if (r != hipSuccess) return r;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[device] = p;
    return hipSuccess;
}

void *scratch_address(int device) {
    if (device < 0 || device >= SCRATCH_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    return g_ptr[device];
}

}  // namespace nvsm
