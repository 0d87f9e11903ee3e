// Fixed device workspace for the entry points that must not allocate.
//
// `scratch` is a file-scope device array: every GPU the library runs on holds
// its own copy (at its own address) until the process ends.  Host code never
// passes the array's name to a kernel or a copy (on the host that name is a
// stand-in, not a device address); it asks the runtime for the device
// address once per device, with that device current, and uses that pointer.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.h"

namespace qs {

namespace {

__device__ __align__(256) double scratch[kNoAllocScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};

}  // namespace

hipError_t noalloc_scratch(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

}  // namespace qs
