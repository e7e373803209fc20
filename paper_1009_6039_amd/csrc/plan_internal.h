// Entry points of the solver plan shared with other parts of the library (not part of
// the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include "common.h"
#include "ma_ot.h"

// theta_q = Lbar^{-1} sigma_q (Section 4.2) for `count` FP32 fields of side n and one
// averaged operator abar[5]: one upload of the pair table and three launches for all
// fields.  sigma_q is only read; theta_q receives the mean-zero result.  Asynchronous.
int plan_lbar_inverse_many(ma_plan* plan, int n, int count, const float* const* sigma, const double* abar,
                           float* const* theta, hipStream_t stream);

// What the autotuner needs of a plan whose first `npairs` pair slots hold synthetic
// fields of side n (pair state: solving, GMRES running, unit Krylov scales).
struct TunerView {
  LaunchCtx ctx;
  int n, npairs;
  const float2* tw;
  PairDesc desc0;  // host copy of pair 0's descriptor
};
// times the variants of each pass and writes the fastest verified ones into t
int tune_passes(const TunerView& view, ma_tuning* t, hipStream_t stream);
// 1 and t->variant filled if the cache file holds an entry for this device, library
// build, n, npairs and restart length m; 0 otherwise
int tune_cache_lookup(const char* path, int n, int npairs, int m, ma_tuning* t);
void tune_cache_store(const char* path, int n, int npairs, int m, const ma_tuning& t);
