// The fixed device scratch of shh_homogenize_noalloc: a file-scope device
// array that every GPU the library runs on holds until the process ends.
//
// In host code `scratch` names a host-side shadow, not device memory: its
// device address is looked up once per device, with that device current, and
// only that address is ever handed to kernels or copies.
#include <hip/hip_runtime.h>

#include <mutex>

#include "shellhom.h"

namespace {

__device__ __align__(256) unsigned char scratch[SHH_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void *g_addr[MAX_DEVICES] = {};

}  // namespace

namespace shh {

// Device address of the current device's copy of `scratch`; the first call on
// a device resolves it (hipGetSymbolAddress) and keeps it.
int noalloc_scratch(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return SHH_HIP_ERROR;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_addr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SHH_HIP_ERROR;
    g_addr[dev] = p;
  }
  *out = g_addr[dev];
  return SHH_OK;
}

}  // namespace shh
