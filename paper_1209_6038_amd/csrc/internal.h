// Calls between the library's own translation units (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/rt.h"

// The network half of rt_surrogate_infer, gate included and no exact
// fallback: rows the gate accepts get their predicted exit in y5, status
// RT_RAY_EXITED and fallback 0; the others get fallback 1 and keep y5 and
// status. d is the geometry of the cloaks (r1, r2, z0, z1). Any n >= 0 (the
// rows go through the network in batches of at most 2^24). Asynchronous on s.
__attribute__((visibility("hidden"))) int surrogate_predict_gated(rt_model model, const rt_cloak_desc &d,
                                                                  int64_t n, int64_t ld, const float *x6,
                                                                  float *y5, uint8_t *fallback,
                                                                  int32_t *status, hipStream_t s);

// RT_OK if the model lives on the current device and has a calibrated trust
// map (what surrogate_predict_gated needs); sets the error message otherwise.
__attribute__((visibility("hidden"))) int surrogate_check_ready(rt_model model);

// The exit error that the model's calibration bounds for an accepted
// prediction (the trust map's tolerance, in units of r2 for position and
// radians for direction).
__attribute__((visibility("hidden"))) double surrogate_exit_tolerance(rt_model model);
