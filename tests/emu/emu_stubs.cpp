// Length classes the emulated replay does not compile (its grids need none of them):
// their launchers report hipErrorNotSupported, so a plan that reaches one fails loudly.
#include <hip/hip_runtime.h>

#include "../../paper_2211_07777_amd/csrc/fm_launch.h"

namespace fm {
#define FM_EMU_STUB(T, MC)                                                                          \
  template <>                                                                                       \
  hipError_t launch_len<T, MC>(const PassDesc&, const PassDesc*, const void*, void*, hipStream_t) { \
    return hipErrorNotSupported;                                                                    \
  }                                                                                                 \
  template <>                                                                                       \
  hipError_t launch_len_batched<T, MC>(const PassDesc*, const int*, int, int, int, hipStream_t) {   \
    return hipErrorNotSupported;                                                                    \
  }
#define FM_EMU_STUBS(T) \
  FM_EMU_STUB(T, 192)   \
  FM_EMU_STUB(T, 256)   \
  FM_EMU_STUB(T, 384)   \
  FM_EMU_STUB(T, 512)   \
  FM_EMU_STUB(T, 768)   \
  FM_EMU_STUB(T, 1024)  \
  FM_EMU_STUB(T, 2048)  \
  FM_EMU_STUB(T, 4096)
FM_EMU_STUBS(float)
FM_EMU_STUBS(double)
FM_EMU_STUB(double, 1)
}  // namespace fm
