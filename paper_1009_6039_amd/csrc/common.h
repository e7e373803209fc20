// Device data structures shared by the kernels and the host driver.
//
// Every pair (f, g) being solved owns one PairDesc (pointers into the plan's
// arena) and one PairState (its Newton / GMRES / step-halving state machine).
// Kernels launched for a class of equal-size pairs take blockIdx.y as the index
// into that class's list of pair ids.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define MA_MMAX 30        // largest GMRES restart length compiled in
#define MA_RES_TX_MAX 64  // residual-kernel tile width (columns)
#define MA_RES_TY 16      // residual-kernel tile height (rows)
#define MA_NPART_RES 16   // partial sums per residual block
#define MA_RES_STREAM_BLOCK 128  // streaming residual kernel: threads per block (2 waves)
#define MA_RES_STREAM_ROWS 32    // streaming residual kernel: rows per wave
#define MA_BLOCK 256
#define MA_SUMMARY_INTS 16  // host-loop counters written by the summary kernel
#define MA_SUMMARY_TAG 15   // slot of the sequence number the summary kernel writes last

// per-pair phase of the Newton loop
enum : int {
  PH_INIT = 0,       // nothing evaluated yet
  PH_SOLVE = 1,      // a Newton direction is being computed this tick
  PH_BACKTRACK = 2,  // the last trial was rejected: halve the step, evaluate again
  PH_REVERT = 3,     // halving exhausted: undo the trial step, evaluate, stop
  PH_DONE = 5,
};

// g, and the fourth-order grid gradient of g, interleaved for one 16-byte gather
struct __align__(16) GS {
  double g;
  float g1, g2;
};

struct PairDesc {
  int n;
  int cls;   // index of the size class this pair belongs to
  int pair;  // the caller's index of the pair in this slot (continuous batching)
  int pad0;
  // caller buffers
  const double* f_in;
  const double* g_in;
  const double* psi0_in;
  double* psi_out;
  double* map_out;
  // workspace
  double* u;       // n*n   current iterate
  double* f;       // n*n   f scaled to mean one
  GS* gs;          // n*n   g scaled to mean one, with its gradient
  float* coef;     // 5*n*n a11, a12, a22, b1, b2
  float* r;        // n*n   f - f_n (the translation constant is added by its readers)
  double* theta;   // n*n   last Newton correction (the initial potential before the first step)
  float* x;        // n*n   GMRES solution accumulated over restarts
  float* V;        // (m+1)*n*n Krylov basis, stored unnormalised (see vscale)
  float2* H;       // n*(n/2) half spectrum after the row pass
  float2* T;       // 3*n*(n/2) column-pass outputs
  double* part;    // per-block partial sums
  double* bv;      // 9*n*n BiCG vectors x, r, r~, q, q~, and p, p~ twice (finite-difference step only)
};

struct PairState {
  // --- Newton control -----------------------------------------------------
  int phase, status;
  int newton_iters, gmres_iters, backtracks, bt_step;
  int valid;            // set by the set-up kernel: 1 = densities positive and finite
  int warm;             // an initial potential was given: it is tried as the first step
  int warm_trial;       // the current trial is that step
  int warm_fallback;    // the trial was abandoned: continue from u = 0
  int warm_steps;       // 1 if the initial potential (possibly halved) was accepted
  int pad1, pad2;
  double tau0, tau;     // caller's damping, damping in force
  double tol;
  double step;          // multiplier of theta applied to the current trial
  double axpy;          // coefficient the next update kernel applies to theta
  double res_rms, res_max, res0, res_prev, mass_c, min_det, min_tr, w2, mean_u;
  double abar[5];
  double mean_f, mean_g, mean_psi0;
  double aux[2];        // power iteration: mean of b_0, then the current scale factor
  // --- GMRES ----------------------------------------------------------------
  int gm_running;       // an Arnoldi cycle is in progress
  int gm_restart;       // the cycle ended short of the tolerance: restart
  int gm_cycle;         // restarts done in this solve
  int gm_k;             // basis size at the end of the cycle
  double bnorm, gm_target;
  double eta;  // adaptive forcing: GMRES tolerance of the next direction (0 = gmres_tol)
  double vscale[MA_MMAX + 1];       // v_l = vscale[l] * V[l]
  double Hm[(MA_MMAX + 1) * MA_MMAX];  // Hessenberg, column-major: Hm[j*(MMAX+1)+i]
  double cs[MA_MMAX], sn[MA_MMAX], gv[MA_MMAX + 1], y[MA_MMAX + 1], q[MA_MMAX + 1];
  // --- BiCG (finite-difference step; gm_running, gm_k, bnorm, gm_target are shared) --
  // rho = r~ . r and the sums of p, p~ (the row of ones of tilde A), by parity of the
  // iteration: iteration j reads slot (j - 1) & 1 and writes slot j & 1
  double bi_rho[2], bi_sum_p[2], bi_sum_pt[2];
  int bi_break;  // a zero denominator: the iteration stops
  int bi_pad;
};

// one slot refilled with a new pair (continuous batching): written by the host into a
// staging buffer, scattered into the slot's descriptor and state by k_refill
struct RefillRecord {
  PairDesc desc;
  PairState state;
  int slot;
  int pad[3];
};

// parameters common to one launch (passed by value)
struct LaunchCtx {
  const PairDesc* desc;
  PairState* st;
  const int* pair_ids;  // pairs of this size class
  int m;                // GMRES restart length
  int max_newton, max_restarts, max_backtrack, damping_policy, interp, op_mode;
  double gmres_tol;
  const float2* mt;  // per-wavenumber multipliers (Im d/dx, d^2/dx^2) of the selected symbol
  unsigned long long* prof_bytes;  // algorithmic-byte counter of the timed class, or null
  int var[4];  // launch-geometry variants (pass A, pass B, pass C, residual), 0 = default
  int precond;  // MA_PRECOND_*: left scaling of the GMRES system by the relative trace
  double boundary_frac;  // step halving: smallest allowed ratio of min det to its current value
  int forcing;           // MA_FORCING_*: fixed or adaptive GMRES tolerance per Newton direction
  // compacted launches: when set, pair_ids is a device list of the pairs that take part
  // and *active_n its length; blocks with blockIdx.y >= *active_n exit at once (the grid
  // is sized by an upper bound the host knows)
  const int* active_n;
  int bicg_max;  // BiCG iterations per Newton step (finite-difference step)
  // pass A's Arnoldi step in a solve: pass C blocks per pair whose inner-product
  // partials pass A folds itself (their region of the partials comes first, pass A's own
  // after it); 0: the coefficients come from the pair's state (the autotuner's launches)
  int dots_nblk;
};

// Global-address-space view of a device buffer.  Accesses through it compile to
// global_* instructions, which count only against the vector-memory counter; the
// flat_* ones that generic pointers get count against the LDS counter as well, so
// every LDS or cross-lane wait would also wait for loads still in flight.  (The
// host pass, which only parses device code, keeps the plain pointer.)
#if defined(__HIP_DEVICE_COMPILE__)
#define MA_GLOBAL_AS __attribute__((address_space(1)))
#else
#define MA_GLOBAL_AS
#endif
template <class T>
__device__ __forceinline__ MA_GLOBAL_AS T* gmem(T* p) {
  return (MA_GLOBAL_AS T*)p;
}

// Stops the instruction scheduler from moving any instruction across this point.
__device__ __forceinline__ void sched_fence() {
#if defined(__HIP_DEVICE_COMPILE__)
  __builtin_amdgcn_sched_barrier(0);
#endif
}

// Runs use(l, x) for l = 0, 1, ..., n - 1 in that order, x holding the thread's K
// elements of vector l as load(l, x) reads them.  Two register sets take the vectors
// in turn, so the loads of vector l + 1 are in flight while vector l is used and no
// register copy waits on a load.  The look-ahead loads are unconditional (a branch
// around a load makes the wait before the next use drain every load in flight): when
// n is even the last one re-reads vector n - 1, which the thread has just read.  A
// scheduling fence after each group of loads keeps the other set's use below it.
template <int K, class LOAD, class USE>
__device__ __forceinline__ void stream_vectors(int n, LOAD load, USE use) {
  if (n <= 0) return;
  float x0[K], x1[K];
  load(0, x0);
  sched_fence();
  int l = 0;
  for (; l + 2 <= n; l += 2) {
    load(l + 1, x1);
    sched_fence();
    use(l, x0);
    load(l + 2 < n ? l + 2 : n - 1, x0);
    sched_fence();
    use(l + 1, x1);
  }
  if (l < n) use(l, x0);
}

// GMRES tolerance of the pair's next Newton direction (eta 0: not adapted yet)
__host__ __device__ inline double pair_eta(const PairState& s, const LaunchCtx& c) {
  return s.eta > 0.0 ? s.eta : c.gmres_tol;
}

// adds one pair's algorithmic bytes for this launch (timed class only)
__device__ inline void count_bytes(const LaunchCtx& c, double bytes_per_point, int n) {
  if (c.prof_bytes && blockIdx.x == 0 && threadIdx.x == 0)
    atomicAdd(c.prof_bytes, (unsigned long long)(bytes_per_point * (double)n * (double)n));
}

// the pair of this block, or -1 for a block beyond a compacted list (it exits)
__device__ inline int pair_of_block(const LaunchCtx& c) {
  if (c.active_n && (int)blockIdx.y >= *c.active_n) return -1;
  return c.pair_ids[blockIdx.y];
}

// ---------------------------------------------------------------------------
// Block reductions (FP64), deterministic order.
// ---------------------------------------------------------------------------
// Cross-lane moves of a double by DPP (VALU moves, no LDS traffic); lanes without a
// source read 0.  CTRL: 0x110 + n, row shift right (lane i of a row of 16 reads lane
// i - n of the row); 0x138, wave shift right (lane i reads lane i - 1); 0x130, wave
// shift left (lane i reads lane i + 1).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
template <int SHIFT>
__device__ __forceinline__ double row_shr(double v) {
  static_assert(SHIFT >= 1 && SHIFT <= 15, "row shift");
  return dpp_move<0x110 + SHIFT>(v);
}
// the same row shift, lanes without a source reading `fill`
template <int SHIFT>
__device__ __forceinline__ double row_shr_or(double v, double fill) {
  static_assert(SHIFT >= 1 && SHIFT <= 15, "row shift");
  const long long b = __double_as_longlong(v), f = __double_as_longlong(fill);
  const int lo = __builtin_amdgcn_update_dpp((int)f, (int)b, 0x110 + SHIFT, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(f >> 32), (int)(b >> 32), 0x110 + SHIFT, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ double read_lane(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
// Sum over the 64 lanes (every lane active), the same in every lane, in a fixed order:
// inclusive prefix sums within each row of 16 lanes by DPP row shifts of 1, 2, 4 and 8,
// then the four row totals (lanes 15, 31, 47, 63) added pairwise.
__device__ inline double wave_sum(double v) {
  v += row_shr<1>(v);
  v += row_shr<2>(v);
  v += row_shr<4>(v);
  v += row_shr<8>(v);
  return (read_lane(v, 15) + read_lane(v, 31)) + (read_lane(v, 47) + read_lane(v, 63));
}
// minimum and maximum over the 64 lanes in the same pattern (shifted-in lanes read the
// operation's identity)
__device__ inline double wave_min(double v) {
  v = fmin(v, row_shr_or<1>(v, INFINITY));
  v = fmin(v, row_shr_or<2>(v, INFINITY));
  v = fmin(v, row_shr_or<4>(v, INFINITY));
  v = fmin(v, row_shr_or<8>(v, INFINITY));
  return fmin(fmin(read_lane(v, 15), read_lane(v, 31)), fmin(read_lane(v, 47), read_lane(v, 63)));
}
__device__ inline double wave_max(double v) {
  v = fmax(v, row_shr_or<1>(v, -INFINITY));
  v = fmax(v, row_shr_or<2>(v, -INFINITY));
  v = fmax(v, row_shr_or<4>(v, -INFINITY));
  v = fmax(v, row_shr_or<8>(v, -INFINITY));
  return fmax(fmax(read_lane(v, 15), read_lane(v, 31)), fmax(read_lane(v, 47), read_lane(v, 63)));
}

// Reduces K values per thread across the block; result valid in thread 0 only.
// kinds[k]: 0 = sum, 1 = min, 2 = max.  scratch: >= (blockDim/64) * K doubles of LDS.
template <int K>
__device__ inline void block_reduce(double (&v)[K], const int (&kinds)[K], double* scratch) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double t = v[k];
    t = kinds[k] == 0 ? wave_sum(t) : (kinds[k] == 1 ? wave_min(t) : wave_max(t));
    if (lane == 0) scratch[wid * K + k] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double t = scratch[k];
      for (int w = 1; w < nw; ++w) {
        double s = scratch[w * K + k];
        t = kinds[k] == 0 ? t + s : (kinds[k] == 1 ? fmin(t, s) : fmax(t, s));
      }
      v[k] = t;
    }
  }
  __syncthreads();
}

// Fixed-order fold of per-block partials (K values per block) inside a
// one-block-per-pair finalize kernel: thread t takes blocks t, t + blockDim, ... in
// that order (for K < 4 the loads of four blocks issued before the first is combined;
// K >= 4 values of one block are already that many loads), then a block reduction.
// Result valid in thread 0.
template <int K>
__device__ inline void fold_partials(const double* part, int nblk, const int (&kinds)[K], double (&t)[K],
                                     double* scratch) {
  constexpr int U = K < 4 ? 4 : 1;
  const auto P = gmem<const double>(part);
#pragma unroll
  for (int k = 0; k < K; ++k) t[k] = kinds[k] == 1 ? 1e300 : (kinds[k] == 2 ? -1e300 : 0.0);
  const int bd = blockDim.x;
  for (int b = threadIdx.x; b < nblk; b += U * bd) {
    double v[U][K];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < K; ++k) v[u][k] = b + u * bd < nblk ? P[(long)(b + u * bd) * K + k] : 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (b + u * bd >= nblk) break;
#pragma unroll
      for (int k = 0; k < K; ++k)
        t[k] = kinds[k] == 0 ? t[k] + v[u][k] : (kinds[k] == 1 ? fmin(t[k], v[u][k]) : fmax(t[k], v[u][k]));
    }
  }
  block_reduce<K>(t, kinds, scratch);
}

// A structure staged in LDS for one thread's serial bookkeeping: the block loads it
// 8 bytes per lane (every load issued before the first use), stores it into LDS, and
// after the bookkeeping writes back the words that changed.  Launch with BLOCK threads.
template <class T, int BLOCK>
struct StagedWords {
  static_assert(sizeof(T) % 8 == 0, "whole 8-byte words");
  static constexpr int WORDS = sizeof(T) / 8, PER = (WORDS + BLOCK - 1) / BLOCK;
  unsigned long long v[PER];
  __device__ void load(const T* src) {
    const auto w = gmem<const unsigned long long>(reinterpret_cast<const unsigned long long*>(src));
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = threadIdx.x + q * BLOCK;
      v[q] = e < WORDS ? w[e] : 0ull;
    }
  }
  __device__ void to_lds(T* lds) const {
    unsigned long long* w = reinterpret_cast<unsigned long long*>(lds);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = threadIdx.x + q * BLOCK;
      if (e < WORDS) w[e] = v[q];
    }
  }
  __device__ void write_back(const T* lds, T* dst) const {
    const unsigned long long* w = reinterpret_cast<const unsigned long long*>(lds);
    const auto d = gmem<unsigned long long>(reinterpret_cast<unsigned long long*>(dst));
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = threadIdx.x + q * BLOCK;
      if (e < WORDS && w[e] != v[q]) d[e] = w[e];
    }
  }
};

// Sum of part[b * stride + l] over b = first, first + step, ... < nblk in a fixed
// order: U accumulators (block first + (r U + u) step goes to accumulator u), the U
// loads of a round issued before its adds, then a pairwise sum of the accumulators.
template <int U>
__device__ inline double strided_sum(const double* part, long stride, int l, int first, int step, int nblk) {
  static_assert((U & (U - 1)) == 0, "U: a power of two");
  const auto P = gmem<const double>(part);
  double a[U];
#pragma unroll
  for (int u = 0; u < U; ++u) a[u] = 0.0;
  for (int b = first; b < nblk; b += U * step) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = b + u * step < nblk ? P[(long)(b + u * step) * stride + l] : 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) a[u] += v[u];
  }
#pragma unroll
  for (int w = U / 2; w > 0; w >>= 1)
#pragma unroll
    for (int u = 0; u < w; ++u) a[u] += a[u + w];
  return a[0];
}
