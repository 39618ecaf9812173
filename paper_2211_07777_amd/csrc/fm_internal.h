// Library-internal entry points shared by the host sources of libfluxmi (not part of
// the C ABI and not exported by name from the header).
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/fluxmi.h"

namespace fm {

// The status code fm_last_hip_error reports for the calling thread.
void set_last_hip_error(int e);

// fm_plan_create whose generation (twiddles, Green's spectrum) is enqueued on `st`
// without waiting for it.  *ready receives an event that completes with the generation:
// solves with the plan on any other stream must wait for it first, and
// plan_generation_done must be called once it has completed (it releases the
// generation's temporaries).  fm_plan_destroy waits for it by itself.
int plan_create_deferred(fm_plan* out, const int n[3], const double h[3], const int bc[3][2],
                         int layout, int green, int prec, int kind, int ncomp, hipStream_t st,
                         hipEvent_t* ready);
void plan_generation_done(fm_plan p);

}  // namespace fm
