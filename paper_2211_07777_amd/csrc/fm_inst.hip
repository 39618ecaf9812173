// One (precision, length class) instantiation of the pass kernels, compiled once per
// pair with -DFM_T=<float|double> -DFM_MC=<length, or kRtShort / kRtLong for the
// runtime-length kernels>.
#include <cstdlib>

#include "fm_device.h"
#include "fm_launch.h"
#include "fm_wave.h"

#ifndef FM_T
#error "FM_T must be defined"
#endif
#ifndef FM_MC
#error "FM_MC must be defined"
#endif

namespace fm {

template <auto K>
static hipError_t allow_full_lds() {
  // let the kernel use the full LDS of a gfx950 workgroup (set once per kernel)
  static hipError_t once = hipFuncSetAttribute(reinterpret_cast<const void*>(K),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
  return once;
}

// Fused complex passes in the per-wavefront kernel with E values per lane: d.B /
// wave_lines(M, E) wavefronts per workgroup, one workgroup per tile.  Three-component
// (curl) lines of 16 values per lane are built in FP32, and in FP64 for 1024-point lines
// only; 32 values per lane (one LDS exchange per transform up to 1024 points) for FP32
// Poisson lines only (three components, or FP64, would not fit the registers).
template <int KIND, int E>
static hipError_t launch_wave_e(const PassDesc& d, const PassDesc* dev, const void* in, void* out,
                                hipStream_t st) {
  if constexpr (wave_length(FM_MC, E) &&
                ((KIND == K_F_C2C && (E != 32 || sizeof(FM_T) == 4)) ||
                 (KIND == K_F_CURL && E != 32 && (sizeof(FM_T) == 4 || E == 8 || FM_MC == 1024)))) {
    const int threads = 64 * (d.B / wave_lines(FM_MC, E));
    if (threads < 64 || threads > kThreads) return hipErrorInvalidValue;
    if (d.lds_bytes > kSoftLds) {
      const hipError_t e = allow_full_lds<&wave_pass_kernel<FM_T, FM_MC, KIND, E>>();
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((wave_pass_kernel<FM_T, FM_MC, KIND, E>), dim3(d.tiles), dim3(threads),
                       d.lds_bytes, st, dev, in, out);
    return hipGetLastError();
  } else {
    (void)d; (void)dev; (void)in; (void)out; (void)st;
    return hipErrorInvalidValue;
  }
}

// Plain passes in the per-wavefront kernel: four wavefronts per workgroup, a persistent
// grid of as many workgroups as can be resident at once (each loops over its tiles).
template <int KIND, int E>
static hipError_t launch_wave_plain_e(const PassDesc& d, const PassDesc* dev, const void* in,
                                      void* out, hipStream_t st) {
  if constexpr (wave_length(FM_MC, E) && KIND >= K_C2C_F && KIND <= K_R2R) {
    constexpr auto kern = &wave_plain_kernel<FM_T, FM_MC, KIND, E>;
    if (d.lds_bytes > kSoftLds) {
      const hipError_t e = allow_full_lds<kern>();
      if (e != hipSuccess) return e;
    }
    static int resident[kMaxLds / 256 + 1] = {0};
    const int slot = d.lds_bytes / 256;
    if (resident[slot] == 0) {
      int per_cu = 0, dev_id = 0, cus = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kThreads, d.lds_bytes) != hipSuccess ||
          per_cu < 1)
        per_cu = 1;
      if (hipGetDevice(&dev_id) != hipSuccess ||
          hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev_id) != hipSuccess || cus < 1)
        cus = 256;
      resident[slot] = per_cu * cus;
    }
    const int grid = d.tiles < resident[slot] ? d.tiles : resident[slot];
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), d.lds_bytes, st, dev, in, out);
    return hipGetLastError();
  } else {
    (void)d; (void)dev; (void)in; (void)out; (void)st;
    return hipErrorInvalidValue;
  }
}

template <int KIND>
static hipError_t launch_wave(const PassDesc& d, const PassDesc* dev, const void* in, void* out,
                              hipStream_t st) {
  if constexpr (fused_of(KIND)) {
    if (d.wave == 16) return launch_wave_e<KIND, 16>(d, dev, in, out, st);
    if (d.wave == 8) return launch_wave_e<KIND, 8>(d, dev, in, out, st);
    if (d.wave == 32) return launch_wave_e<KIND, 32>(d, dev, in, out, st);
  } else {
    if (d.wave == 16) return launch_wave_plain_e<KIND, 16>(d, dev, in, out, st);
    if (d.wave == 8) return launch_wave_plain_e<KIND, 8>(d, dev, in, out, st);
  }
  return hipErrorInvalidValue;
}

template <int KIND>
static hipError_t launch_kind(const PassDesc& d, const PassDesc* dev, const void* in, void* out,
                              hipStream_t st) {
  if constexpr (KIND == K_F_C2C || KIND == K_F_CURL || (KIND >= K_C2C_F && KIND <= K_R2R)) {
    if (d.wave) return launch_wave<KIND>(d, dev, in, out, st);
  }
  static const bool persistent = [] {
    const char* e = std::getenv("FLUXMI_PERSISTENT");
    return e == nullptr || std::atoi(e) != 0;
  }();
  if constexpr (pipelined_kernel((int)sizeof(FM_T), FM_MC)) {
    // twiddle tables staged in LDS: the pipelined kernel, on a persistent grid (as many
    // workgroups as can be resident at once, each looping over tiles) or one tile each
    if (d.lds_tabs) {
      if (d.lds_bytes > kSoftLds) {
        const hipError_t e = allow_full_lds<&pass_kernel<FM_T, FM_MC, KIND, 1>>();
        if (e != hipSuccess) return e;
      }
      static int resident[kMaxLds / 256 + 1] = {0};
      const int slot = d.lds_bytes / 256;
      if (resident[slot] == 0) {
        int per_cu = 0, dev_id = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pass_kernel<FM_T, FM_MC, KIND, 1>,
                                                          kThreads, d.lds_bytes) != hipSuccess ||
            per_cu < 1)
          per_cu = 1;
        if (hipGetDevice(&dev_id) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev_id) != hipSuccess ||
            cus < 1)
          cus = 256;
        resident[slot] = per_cu * cus;
      }
      const int grid = (!persistent || !d.persist || d.tiles < resident[slot]) ? d.tiles : resident[slot];
      hipLaunchKernelGGL((pass_kernel<FM_T, FM_MC, KIND, 1>), dim3(grid), dim3(kThreads), d.lds_bytes,
                         st, dev, in, out);
      return hipGetLastError();
    }
  }
  // one tile per workgroup, tables read from global memory
  if (d.lds_bytes > kSoftLds) {
    const hipError_t e = allow_full_lds<&pass_kernel<FM_T, FM_MC, KIND, 0>>();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((pass_kernel<FM_T, FM_MC, KIND, 0>), dim3(d.tiles), dim3(kThreads), d.lds_bytes,
                     st, dev, in, out);
  return hipGetLastError();
}

template <>
hipError_t launch_len<FM_T, FM_MC>(const PassDesc& d, const PassDesc* dev, const void* in,
                                   void* out, hipStream_t st) {
  switch (d.kind) {
    case K_C2C_F: return launch_kind<K_C2C_F>(d, dev, in, out, st);
    case K_C2C_I: return launch_kind<K_C2C_I>(d, dev, in, out, st);
    case K_R2C: return launch_kind<K_R2C>(d, dev, in, out, st);
    case K_C2R: return launch_kind<K_C2R>(d, dev, in, out, st);
    case K_R2R: return launch_kind<K_R2R>(d, dev, in, out, st);
    case K_F_C2C: return launch_kind<K_F_C2C>(d, dev, in, out, st);
    case K_F_CURL: return launch_kind<K_F_CURL>(d, dev, in, out, st);
    case K_F_R2C: return launch_kind<K_F_R2C>(d, dev, in, out, st);
    case K_F_R2R: return launch_kind<K_F_R2R>(d, dev, in, out, st);
    default: return hipErrorInvalidValue;
  }
}

template <>
hipError_t launch_len_batched<FM_T, FM_MC>(const PassDesc* ds, const int* prefix, int n,
                                           int total_tiles, int lds_bytes, hipStream_t st) {
#ifdef FM_NO_BATCHED
  // the one-launch batched kernels exist in FP64 only; FP32 batches run plan by plan
  (void)ds; (void)prefix; (void)n; (void)total_tiles; (void)lds_bytes; (void)st;
  return hipErrorNotSupported;
#else
  if (lds_bytes > kSoftLds) {
    const hipError_t e = allow_full_lds<&pass_kernel_batched<FM_T, FM_MC>>();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((pass_kernel_batched<FM_T, FM_MC>), dim3(total_tiles), dim3(kThreads),
                     lds_bytes, st, ds, prefix, n);
  return hipGetLastError();
#endif
}

}  // namespace fm
