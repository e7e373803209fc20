// Host-side launchers of the device kernels (one call per size class).
#pragma once
#include <hip/hip_ext.h>

#include "common.h"

// Optional start/stop events stamped at the kernel's own start and end
// (hipExtLaunchKernelGGL), used by the timing hook.
struct TimedLaunch {
  hipEvent_t start = nullptr, stop = nullptr;
};
#define MA_LAUNCH(ev, kernel, grid, block, st, ...)                                           \
  do {                                                                                        \
    if ((ev).start)                                                                           \
      hipExtLaunchKernelGGL(kernel, grid, block, 0, st, (ev).start, (ev).stop, 0, __VA_ARGS__); \
    else                                                                                      \
      hipLaunchKernelGGL(kernel, grid, block, 0, st, __VA_ARGS__);                            \
  } while (0)

// pass modes
enum : int {
  PA_INIT = 0,     // v0 = (r + translation) / tau, stored as V[0]
  PA_PLAIN = 1,    // V[0] as written by the restart kernel
  PA_ARNOLDI = 2,  // Gram-Schmidt update of V[jn] against V[0..jn-1]
  PA_RECOVER = 3,  // sigma = x + sum y_l v_l
  PA_STEP = 4,     // V[0] as given (single-step entry points)
};
enum : int { PB_MATVEC = 0, PB_RECOVER = 1, PB_FORWARD = 2 };
enum : int { PC_MATVEC = 0, PC_RECOVER = 1, PC_THETA_ONLY = 2 };
// power iteration steps (k_power_vec / k_power_fold)
enum : int { PW_SUM_B0 = 0, PW_CENTER = 1, PW_SCALE = 2, PW_THETA = 3, PW_NEXT = 4 };

void launch_setup(const LaunchCtx& c, int n, int npairs, hipStream_t st);
void launch_setup_fields(const LaunchCtx& c, int n, int npairs, hipStream_t st);
int residual_tile_x(int n, int v);
int residual_blocks(int n, int v);
void launch_residual(const LaunchCtx& c, int n, int npairs, int step_mode, hipStream_t st,
                     const TimedLaunch& ev = TimedLaunch());
void launch_residual_only(const LaunchCtx& c, int n, int npairs, hipStream_t st,
                          const TimedLaunch& ev = TimedLaunch());
void launch_residual_shift(const LaunchCtx& c, int n, float* out, hipStream_t st);
void launch_step_update(const LaunchCtx& c, int n, int npairs, hipStream_t st);
void launch_outputs(const LaunchCtx& c, int n, int npairs, hipStream_t st);
void launch_summary(const PairState* s, const int* ids, int npairs, int* out, int seq, hipStream_t st,
                    int* phases = nullptr);
// compacted launch lists per size class (live: not done; solving: in a Newton direction)
void launch_compact(const PairState* state, const int* ids, const int2* cls, int ncls, int* live, int* solving,
                    int* cnt, hipStream_t st);
// the pairs of a launch list still inside their GMRES cycle (order kept) and their number
void launch_compact_running(const PairState* state, const int* in, const int* in_n, int count, int* out,
                            int* out_n, hipStream_t st);
// continuous batching: outputs and final states of finished slots (ids in the context),
// refill records scattered into their slots, validation of every pair's inputs
void launch_retire(const LaunchCtx& c, int n, int count, PairState* final_state, hipStream_t st);
void launch_refill(PairDesc* desc, PairState* state, const RefillRecord* rec, int count, hipStream_t st);
void launch_validate(const double* const* f, const double* const* g, const double* const* psi0, const int* n,
                     int npairs, int nmax, int* bad, hipStream_t st);
void launch_tune_fill(const LaunchCtx& c, int n, int npairs, hipStream_t st);

// FFT passes and GMRES kernels; `tw` is the length-n twiddle table
bool fft_size_supported(int n);
// launch-geometry variants 0..MA_NVARIANTS-1 of each pass (0 = default); the geometry
// functions return the variant's canonical index (a duplicate returns 0) or -1
constexpr int MA_NVARIANTS = 12;
// Variants 8..11 of the transform passes change the radix plan of their FFTs (fft.h):
// plan 1 (8, 10) or plan 2 (9, 11), at the default geometry (8, 9) or at the pass's
// second geometry (10, 11: geometry 2 for passes A and B, 3 for pass C).  A plan that
// equals plan 0 for the size leaves the kernel of that geometry.
constexpr bool is_plan_variant(int v) { return v >= 8 && v < 12; }
constexpr int plan_of_variant(int v) { return (v - 8) % 2 + 1; }
constexpr int plan_geometry(int v, int second) { return v < 10 ? 0 : second; }
int passA_geometry(int n, int v, int* row_pairs, int* threads);
int passB_geometry(int n, int v, int* columns, int* threads);
int passC_geometry(int n, int v, int* row_pairs, int* threads);
int residual_geometry(int n, int v, int* tile_x, int* threads);
int passA_blocks(int n, int v);
int passB_blocks(int n, int v);
int passC_blocks(int n, int v);
void launch_passA(const LaunchCtx& c, int n, int npairs, int mode, int jn, const float2* tw, hipStream_t st,
                  const TimedLaunch& ev = TimedLaunch());
void launch_passA_only(const LaunchCtx& c, int n, int npairs, int mode, int jn, const float2* tw, hipStream_t st,
                  const TimedLaunch& ev = TimedLaunch());
void launch_passB(const LaunchCtx& c, int n, int npairs, int mode, int j, const float2* tw, hipStream_t st,
                  const TimedLaunch& ev = TimedLaunch());
void launch_passC(const LaunchCtx& c, int n, int npairs, int mode, int j, const float2* tw, hipStream_t st,
                  const TimedLaunch& ev = TimedLaunch());
void launch_passC_only(const LaunchCtx& c, int n, int npairs, int mode, int j, const float2* tw, hipStream_t st,
                  const TimedLaunch& ev = TimedLaunch());
void launch_restart(const LaunchCtx& c, int n, int npairs, hipStream_t st);
// one power-iteration step on pair 0 of the context and its fold; `out` receives
// (rho_k, GMRES iterations so far) at index 2k, 2k+1 for mode PW_THETA
int power_blocks(int n);

// the finite-difference BiCG step (Section 4.1), one step of its launch sequence
enum : int { BI_INIT = 0, BI_MATVEC = 1, BI_UPDATE = 2, BI_FINISH = 3 };
int bicg_tx(int n);
int bicg_blocks(int n);
void launch_bicg(const LaunchCtx& c, int n, int npairs, int step, int j, hipStream_t st,
                 const TimedLaunch& ev = TimedLaunch());
void launch_power_vec(const LaunchCtx& c, int n, int mode, const float* b0, double* out, int k, hipStream_t st);
