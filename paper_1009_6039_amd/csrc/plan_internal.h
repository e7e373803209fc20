// Entry points of the solver plan shared with other parts of the library (not part of
// the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include "ma_ot.h"

// theta_q = Lbar^{-1} sigma_q (Section 4.2) for `count` FP32 fields of side n and one
// averaged operator abar[5]: one upload of the pair table and three launches for all
// fields.  sigma_q is only read; theta_q receives the mean-zero result.  Asynchronous.
int plan_lbar_inverse_many(ma_plan* plan, int n, int count, const float* const* sigma, const double* abar,
                           float* const* theta, hipStream_t stream);
