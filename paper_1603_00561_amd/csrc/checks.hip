// The per-device sign check word of DSRG_OPT_CHECK_SIGNS: bit 0 is set by a
// CCVV work item whose contribution to E_CCVV came out positive or NaN
// (impossible when every denominator e_i + e_j - e_a - e_b of Eq. expensive is
// negative, so a set bit flags orbital energies out of order, NaN inputs or
// a fault in the kernels).
//
// As for any file-scope device variable, each GPU holds its own copy and the
// name is only a host-side stand-in: the device address is looked up once per
// device with hipGetSymbolAddress, with that device current, and passed to the
// kernels as an argument.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"

namespace dsrg {

static __device__ unsigned sign_check_word;

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned *g_ptr[kMaxDevices] = {};
}  // namespace

hipError_t sign_check_ptr(unsigned **ptr) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(sign_check_word));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[dev] = static_cast<unsigned *>(p);
  }
  *ptr = g_ptr[dev];
  return hipSuccess;
}

hipError_t sign_check_read(unsigned *word) {
  unsigned *p = nullptr;
  hipError_t e = sign_check_ptr(&p);
  if (e != hipSuccess) return e;
  if ((e = hipDeviceSynchronize()) != hipSuccess) return e;
  if ((e = hipMemcpy(word, p, sizeof(unsigned), hipMemcpyDeviceToHost)) != hipSuccess) return e;
  const unsigned zero = 0;
  return hipMemcpy(p, &zero, sizeof(unsigned), hipMemcpyHostToDevice);
}

}  // namespace dsrg
