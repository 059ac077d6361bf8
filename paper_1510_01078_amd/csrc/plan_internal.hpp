// Internal to the library: the plan object and host helpers shared by the
// single-problem (api.hip) and batched (batch.hip) entry points.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "kernels.hpp"
#include "pat_nufft.h"

namespace patint {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

inline void* dev_alloc(const pat_plan_desc& d, size_t bytes) {
  if (d.alloc) return d.alloc(bytes, d.alloc_ctx);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

inline void dev_free(const pat_plan_desc& d, void* p) {
  if (!p) return;
  if (d.free)
    d.free(p, d.alloc_ctx);
  else
    (void)hipFree(p);
}

inline pat_status to_status(hipError_t e) { return e == hipSuccess ? PAT_OK : PAT_ERR_HIP; }

struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) {
      ok = false;
      prev = -1;
      return;
    }
    if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

}  // namespace patint

struct pat_plan {
  pat_plan_desc d;
  int device = 0;
  bool fp64 = false;
  patk::DevPlan dp;
  void* dev = nullptr;
  size_t dev_bytes = 0;
  size_t off_B = 0;     // workspace regions: A at 0 (grid chunk / lateral spectra),
  size_t off_C = 0;     // B at off_B (x rows / spectrum), C at off_C (per-sensor bins)
  size_t ws_bytes = 0;
  int64_t spread_pairs = 0;
  int64_t spread_slots = 0;
  int64_t band_pairs = 0;   // (x-mode, bin) pairs inside the per-x-mode band ranges
  bool forward_ok = false;  // the forward model's per-column LDS fits the device
  bool forward_fused = false;  // the forward model's x-FFT and interpolation run as one kernel
  double range_xy = 1.0;    // dynamic range of the lateral deconvolution (x times y)
  double range_t = 1.0;     // dynamic range of the temporal deapodisation
  // timing: per recorded call, marks_per_call events; mark i > 0 closes the
  // interval of stage ev_stage[i] that began at mark i-1
  std::vector<hipEvent_t> ev;
  std::vector<int> ev_stage;
  int marks_per_call = 0;
  unsigned ev_mask = 0;  // stages whose two ends record events
  int ev_max = 0;
  int ev_used = 0;
};
