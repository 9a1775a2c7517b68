// Fixed device workspace of navsim_rp_propose_noalloc: one array per device,
// part of the library's code object, so the entry point that uses it never
// allocates.  Host code must not pass `scratch` itself to a kernel (in host
// code the name is a stand-in, not a device address): rp_scratch_address()
// looks the array's device address up once per device and every user takes
// that pointer.
#include <hip/hip_runtime.h>

#include <mutex>

#include "rp_scratch.hpp"

static __device__ __align__(256) unsigned char scratch[navsim::kRpScratchBytes];

namespace navsim {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_addr[kMaxDevices] = {};

}  // namespace

hipError_t rp_scratch_address(int device, void **out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_addr[device] = p;
    }
    *out = g_addr[device];
    return hipSuccess;
}

}  // namespace navsim
