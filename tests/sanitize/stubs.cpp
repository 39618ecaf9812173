// Device-side entry points of the library replaced by stubs, so that the host planning
// code (fm_plan.cpp) links into a sanitizer build without device code.  Planning and the
// host-only entry points never reach them.
#include <hip/hip_runtime.h>

#include "../../paper_2211_07777_amd/csrc/fm_pass.h"

namespace fm {
template <typename T>
hipError_t launch_pass(const PassDesc&, const PassDesc*, const void*, void*, hipStream_t) {
  return hipErrorNotSupported;
}
template <typename T>
hipError_t launch_pass_batched(int, const PassDesc*, const int*, int, int, int, hipStream_t) {
  return hipErrorNotSupported;
}
template <typename T> hipError_t launch_twiddles(void*, int, hipStream_t) { return hipErrorNotSupported; }
template <typename T> hipError_t launch_stage_twiddles(void*, int, hipStream_t) { return hipErrorNotSupported; }
template <typename T> hipError_t launch_wave_twiddles(void*, int, int, hipStream_t) { return hipErrorNotSupported; }
template <typename T>
hipError_t launch_green_final(void*, const double*, const int[3], const int[3], const int[3], double, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_green_sample(double*, const GreenGen&, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_lgf(double*, double*, double*, const LgfGen&, hipStream_t) { return hipErrorNotSupported; }
template <typename T> hipError_t launch_curl_real(const CurlReal&, hipStream_t) { return hipErrorNotSupported; }
template hipError_t launch_curl_real<float>(const CurlReal&, hipStream_t);
template hipError_t launch_curl_real<double>(const CurlReal&, hipStream_t);
bool is_fast_len(int M) {
  for (int m : kFastLens)
    if (m == M) return true;
  return false;
}
template hipError_t launch_pass<float>(const PassDesc&, const PassDesc*, const void*, void*, hipStream_t);
template hipError_t launch_pass<double>(const PassDesc&, const PassDesc*, const void*, void*, hipStream_t);
template hipError_t launch_pass_batched<float>(int, const PassDesc*, const int*, int, int, int, hipStream_t);
template hipError_t launch_pass_batched<double>(int, const PassDesc*, const int*, int, int, int, hipStream_t);
template hipError_t launch_twiddles<float>(void*, int, hipStream_t);
template hipError_t launch_twiddles<double>(void*, int, hipStream_t);
template hipError_t launch_stage_twiddles<float>(void*, int, hipStream_t);
template hipError_t launch_stage_twiddles<double>(void*, int, hipStream_t);
template hipError_t launch_wave_twiddles<float>(void*, int, int, hipStream_t);
template hipError_t launch_wave_twiddles<double>(void*, int, int, hipStream_t);
template hipError_t launch_green_final<float>(void*, const double*, const int[3], const int[3], const int[3], double, hipStream_t);
template hipError_t launch_green_final<double>(void*, const double*, const int[3], const int[3], const int[3], double, hipStream_t);
}  // namespace fm
