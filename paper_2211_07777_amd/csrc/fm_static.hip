// fm_solve_static: fm_solve with the workspace taken from a fixed device array of the
// library instead of the caller or the allocator, for callers that cannot allocate
// device memory (code under graph capture, tight serving loops, harnesses that forbid
// hipMalloc).
//
// The array `scratch` below is a file-scope device variable: every GPU the library runs
// on holds its own copy, at its own address, until the process ends.  Its name in host
// code is a host-side stand-in, not a device address; the device address is looked up
// once per device (hipGetSymbolAddress, with that device current) and only that
// address is handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/fluxmi.h"
#include "fm_internal.h"

namespace {

constexpr size_t kScratchBytes = FM_STATIC_WORKSPACE_BYTES;
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch_dev[kMaxDevices] = {nullptr};

// The device address of `scratch` on the current device (looked up once per device).
int scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    fm::set_last_hip_error((int)e);
    return FM_E_HIP;
  }
  if (dev < 0 || dev >= kMaxDevices) return FM_E_ARG;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) {
      fm::set_last_hip_error((int)e);
      return FM_E_HIP;
    }
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return FM_OK;
}

}  // namespace

extern "C" {

int fm_solve_static(fm_plan p, const void* rhs_dev, void* out_dev, void* hip_stream) {
  if (!p || !rhs_dev || !out_dev) return FM_E_NULL;
  size_t need = 0;
  int rc = fm_plan_workspace_bytes(p, &need);
  if (rc) return rc;
  if (need > kScratchBytes) return FM_E_SCRATCH;
  void* ws = nullptr;
  rc = scratch_address(&ws);
  if (rc) return rc;
  // every pass writes its whole output before the next pass reads it, so the array
  // needs no clearing between calls
  return fm_solve(p, rhs_dev, out_dev, ws, hip_stream);
}

}  // extern "C"
