// The library's own device scratch array, for dsrg_df_energy_noalloc: the
// workspace of an energy call held in a file-scope device array instead of a
// caller buffer, for callers that cannot allocate device memory.
//
// Each GPU the library runs on holds its own copy of the array (its address
// differs per device) from the loading of the code object until the process
// ends. Host code never passes the array's name to a kernel: the name is a
// host-side stand-in, not a device address. The device address is looked up
// once per device with hipGetSymbolAddress, with that device current, and
// kept; kernels receive that pointer as their workspace argument.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"

namespace dsrg {

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch(void **ptr) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[dev] = p;
  }
  *ptr = g_ptr[dev];
  return hipSuccess;
}

}  // namespace dsrg
