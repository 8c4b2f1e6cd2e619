// Fixed device workspace for the entry points that must not allocate
// (bido_inner_solve_noalloc): one file-scope array per GPU, sized once at
// build time.  Host code never passes the array's name to a kernel (in host
// code it is only a stand-in for the symbol); it looks up the array's device
// address once per device with hipGetSymbolAddress and hands that out.
#include <hip/hip_runtime.h>

#include <mutex>

#include "launch.h"

namespace bido {

namespace {

static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
double* g_ptr[MAX_DEVICES] = {};

}  // namespace

hipError_t noalloc_scratch(int device, double** ptr) {
    *ptr = nullptr;
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) {
            e = hipSetDevice(device);
            if (e != hipSuccess) return e;
        }
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) hipSetDevice(cur);
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[device] = static_cast<double*>(p);
    }
    *ptr = g_ptr[device];
    return hipSuccess;
}

}  // namespace bido
