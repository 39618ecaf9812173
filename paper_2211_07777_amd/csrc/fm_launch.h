// Per-length pass launchers.  Each (precision, length class) pair is compiled in its
// own object from fm_inst.hip; length classes kRtShort / kRtLong are the runtime-length
// kernels (kRtLong only in FP64).
#pragma once
#include <hip/hip_runtime.h>

#include "fm_pass.h"

namespace fm {

// d: host copy (grid, LDS); dev: the same descriptor in device memory
template <typename T, int MC>
hipError_t launch_len(const PassDesc& d, const PassDesc* dev, const void* in, void* out,
                      hipStream_t st);

template <typename T, int MC>
hipError_t launch_len_batched(const PassDesc* ds, const int* prefix, int n, int total_tiles,
                              int lds_bytes, hipStream_t st);

#define FM_DECLARE_LEN(T, MC)                                                                  \
  template <>                                                                                  \
  hipError_t launch_len<T, MC>(const PassDesc& d, const PassDesc* dev, const void* in, void* out, \
                               hipStream_t st);                                                 \
  template <>                                                                                  \
  hipError_t launch_len_batched<T, MC>(const PassDesc* ds, const int* prefix, int n,            \
                                       int total_tiles, int lds_bytes, hipStream_t st);
#define FM_DECLARE_PREC(T)                                                                    \
  FM_DECLARE_LEN(T, 0)                                                                        \
  FM_DECLARE_LEN(T, 32)                                                                       \
  FM_DECLARE_LEN(T, 48)                                                                       \
  FM_DECLARE_LEN(T, 64)                                                                       \
  FM_DECLARE_LEN(T, 96)                                                                       \
  FM_DECLARE_LEN(T, 128)                                                                      \
  FM_DECLARE_LEN(T, 192)                                                                      \
  FM_DECLARE_LEN(T, 256)                                                                      \
  FM_DECLARE_LEN(T, 384)                                                                      \
  FM_DECLARE_LEN(T, 512)                                                                      \
  FM_DECLARE_LEN(T, 768)                                                                      \
  FM_DECLARE_LEN(T, 1024)                                                                     \
  FM_DECLARE_LEN(T, 2048)                                                                     \
  FM_DECLARE_LEN(T, 4096)
FM_DECLARE_PREC(float)
FM_DECLARE_PREC(double)
FM_DECLARE_LEN(double, 1)  // kRtLong: FP64 lines longer than kMaxFastLen64
#undef FM_DECLARE_PREC
#undef FM_DECLARE_LEN

}  // namespace fm
