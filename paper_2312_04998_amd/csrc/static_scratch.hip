// Library-held scratch for the allocation-free VJP entry point
// (ac_vjp_static): the per-workgroup partial sums of dL/dlog alpha live in a
// file-scope device array instead of memory the network allocates. Each GPU
// holds its own copy for the life of the process; host code reaches it only
// through the device address looked up here, once per device.
#include <hip/hip_runtime.h>

#include <mutex>

#include "devnet.h"

namespace ac {

static __device__ __align__(256) double scratch[size_t(VJP_STATIC_ROWS) * VJP_STATIC_NR];

hipError_t vjp_static_scratch(double **ptr) {
  constexpr int MAX_DEVICES = 64;
  static std::mutex mu;
  static double *addr[MAX_DEVICES] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = static_cast<double *>(p);
  }
  *ptr = addr[dev];
  return hipSuccess;
}

}  // namespace ac
