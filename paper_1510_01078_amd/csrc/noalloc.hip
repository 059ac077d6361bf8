// Reconstruction without a caller workspace and without any allocation: the
// workspace lives in a fixed device array of the library (one per GPU the
// library runs on, held until the process ends), for callers that cannot
// allocate device memory at the time of the call.
#include <hip/hip_runtime.h>

#include <mutex>

#include "pat_nufft.h"
#include "plan_internal.hpp"

using namespace patint;

namespace {

// The library's scratch workspace. In host code `scratch` names a host-side
// stand-in, not device memory: its device address is taken once per device
// with hipGetSymbolAddress and only that address is used.
static __device__ __align__(256) unsigned char scratch[PAT_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;

// Device address of this device's scratch array, looked up on the first call
// with `dev` current; nullptr if the lookup failed.
void* scratch_address(int dev) {
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    addr[dev] = p;
  }
  return addr[dev];
}

}  // namespace

extern "C" pat_status pat_reconstruct_noalloc(pat_plan* P, const void* g, void* f, void* stream) {
  if (!P || !g || !f) return PAT_ERR_INVALID_ARGUMENT;
  size_t need = 0;
  const pat_status st = nufft_plan_workspace_size(P, &need);
  if (st != PAT_OK) return st;
  if (need > size_t(PAT_NOALLOC_SCRATCH_BYTES)) return PAT_ERR_WORKSPACE_TOO_LARGE;
  void* ws = nullptr;
  {
    DeviceGuard guard(P->device);
    if (!guard.ok) return PAT_ERR_HIP;
    ws = scratch_address(P->device);
  }
  if (!ws) return PAT_ERR_HIP;
  // every stage writes what the next one reads, so nothing in the scratch
  // needs clearing between calls
  return pat_reconstruct(P, g, f, ws, stream);
}
