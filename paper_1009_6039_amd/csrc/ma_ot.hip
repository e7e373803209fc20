// C ABI and host driver of the solver: plans, workspace arena, the per-tick
// launch sequence of the damped Newton loop (eq. linma) with its GMRES(m) linear
// solves (Section 4.2), and the single-step entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <vector>

#include "common.h"
#include "kernels.h"
#include "ma_ot.h"
#include "plan_internal.h"

namespace {

#define HIP_TRY(x)                          \
  do {                                      \
    if ((x) != hipSuccess) return MA_EHIP;  \
  } while (0)

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct Tune {
  int v[4] = {0, 0, 0, 0};  // pass A, pass B, pass C, residual
};

struct Class {
  int n;
  int count = 0;         // pairs of this size (of a compacted list: an upper bound)
  int* d_ids = nullptr;  // slice of the plan's id buffer (or of a compacted list)
  const int* active_n = nullptr;  // device length of a compacted list, else null
  const float2* tw = nullptr;
  const float2* mt = nullptr;
};

// the size classes of one solve, iterable with a range-for
struct ClassList {
  const Class* p;
  int n;
  const Class* begin() const { return p; }
  const Class* end() const { return p + n; }
};

}  // namespace

struct ma_plan {
  ma_options opt;
  int n_max = 0, cap = 0;
  char* arena = nullptr;
  size_t arena_bytes = 0;
  PairDesc* d_desc = nullptr;
  PairState* d_state = nullptr;
  int* d_ids = nullptr;
  // compacted lists: live ids, solving ids (pairs_cap each), then per class (offset,
  // count) and the two counts, then the GMRES cycle's running ids and their counts
  // (not in the no-allocation mode, whose lists hold the first six only)
  int* d_lists = nullptr;
  int pairs_cap = 0;
  // host-loop counters: 4 slots of MA_SUMMARY_INTS (the synchronous read, then a ring
  // of 3) in coherent pinned host memory that the summary kernel writes directly,
  // each ending with the sequence number of the launch that wrote it
  int* h_summary = nullptr;
  int* d_summary = nullptr;  // the device's address of h_summary
  int sum_seq = 0;           // sequence number of the last summary launched
  int ring_seq[3] = {0, 0, 0};
  std::map<int, float2*> tw;
  std::map<std::pair<int, int>, float2*> mt;  // (n, symbol) -> derivative multipliers
  std::map<int, Tune> tune;                   // n -> launch-geometry variants (absent: defaults)
  std::vector<PairDesc> h_desc;
  std::vector<PairState> h_state;
  std::vector<int2> h_ctab;  // class table staged for upload (lives as long as the plan)
  // timing hook
  int prof_kind = MA_PROF_NONE;
  unsigned long long* d_prof = nullptr;
  std::vector<hipEvent_t> ev;  // start/end pairs
  int ev_used = 0;
  double prof_ms = 0.0;
  long long prof_launches = 0;
  int prof_every = 1;       // time every prof_every-th launch of the class
  long long prof_seq = 0;   // launches of the class seen since ma_plan_profile
  // continuous batching: final states by pair, per-slot phases in mapped host memory,
  // a pinned host staging buffer and its device copy (validation tables, refill records)
  PairState* d_final = nullptr;
  int final_cap = 0;
  int* h_phase = nullptr;
  int* d_phase = nullptr;
  int phase_cap = 0;
  char* h_stage = nullptr;
  char* d_stage = nullptr;
  size_t stage_cap = 0;
  // no-allocation mode (ma_solve_noalloc): every device buffer is carved from the
  // library's static scratch array, the summary lives in device memory and is copied
  // back after each launch that the host waits on
  bool no_alloc = false;
  int h_summary_buf[MA_SUMMARY_INTS] = {};
};

namespace {

// partial-sum slots per pair: the largest need over all launch-geometry variants
size_t part_doubles(int n) {
  size_t need = 256 * 4, c_max = 0, a_max = 0;
  need = std::max(need, (size_t)bicg_blocks(n) * 5);
  for (int v = 0; v < MA_NVARIANTS; ++v) {
    need = std::max(need, (size_t)residual_blocks(n, v) * MA_NPART_RES);
    c_max = std::max(c_max, (size_t)passC_blocks(n, v) * (MA_MMAX + 1));
    a_max = std::max(a_max, (size_t)passA_blocks(n, v));
  }
  // pass C's inner-product partials, then pass A's norm partials of the Arnoldi step
  return std::max(need, c_max + a_max + 16);
}

size_t pair_bytes(int n, int m, bool bicg) {
  const size_t nn = (size_t)n * n;
  size_t b = 0;
  b += align256(8 * nn) * 2;              // u, f
  b += align256(16 * nn);                 // gs
  b += align256(20 * nn);                 // coef
  b += align256(4 * nn) * 2;              // r, x
  b += align256(8 * nn);                  // theta
  b += align256(4 * nn * (size_t)(m + 1));  // V
  b += align256(4 * nn);                  // H
  b += align256(12 * nn);                 // T
  b += align256(8 * part_doubles(n));     // partials
  if (bicg) b += align256(72 * nn);       // BiCG vectors
  return b;
}

void carve(PairDesc& d, char*& p, int n, int m, bool bicg) {
  const size_t nn = (size_t)n * n;
  auto take = [&](size_t bytes) {
    char* q = p;
    p += align256(bytes);
    return q;
  };
  d.n = n;
  d.u = (double*)take(8 * nn);
  d.f = (double*)take(8 * nn);
  d.gs = (GS*)take(16 * nn);
  d.coef = (float*)take(20 * nn);
  d.r = (float*)take(4 * nn);
  d.theta = (double*)take(8 * nn);
  d.x = (float*)take(4 * nn);
  d.V = (float*)take(4 * nn * (size_t)(m + 1));
  d.H = (float2*)take(4 * nn);
  d.T = (float2*)take(12 * nn);
  d.part = (double*)take(8 * part_doubles(n));
  d.bv = bicg ? (double*)take(72 * nn) : nullptr;
}

bool uses_bicg(const ma_options& o) { return o.linear_solver == MA_LINEAR_FD_BICG; }

bool n_ok(int n) { return n >= 16 && n <= 2048 && n % 16 == 0 && fft_size_supported(n); }

int validate_options(const ma_options& o) {
  if (o.max_newton < 0 || o.gmres_m < 1 || o.gmres_m > MA_MMAX || o.gmres_max_restarts < 0 ||
      !(o.gmres_tol > 0.0) || (o.interp != MA_INTERP_BILINEAR && o.interp != MA_INTERP_NEAREST) ||
      (o.op_mode != MA_OP_FULL && o.op_mode != MA_OP_NO_DRIFT) ||
      (o.damping_policy != MA_DAMP_FIXED && o.damping_policy != MA_DAMP_BACKTRACK) || o.max_backtrack < 0 ||
      (o.symbol != MA_SYMBOL_SPECTRAL && o.symbol != MA_SYMBOL_FD4) ||
      (o.precond != MA_PRECOND_NONE && o.precond != MA_PRECOND_DIAG) ||
      !(o.boundary_frac >= 0.0 && o.boundary_frac < 1.0) ||
      (o.forcing != MA_FORCING_FIXED && o.forcing != MA_FORCING_ADAPTIVE) || !(o.wait_limit_s > 0.0) ||
      o.max_active < 0 || (o.linear_solver != MA_LINEAR_STRAIN_GMRES && o.linear_solver != MA_LINEAR_FD_BICG) ||
      o.bicg_max_iters < 1 || (o.linear_solver == MA_LINEAR_FD_BICG && o.precond != MA_PRECOND_NONE))
    return MA_EINVAL;
  return MA_OK;
}

// tw[m] = exp(-2 pi i m / n), computed in FP64 and stored in FP32
void fill_twiddles(float2* h, int n) {
  for (int m = 0; m < n; ++m) {
    const double a = -2.0 * M_PI * (double)m / (double)n;
    h[m] = make_float2((float)std::cos(a), (float)std::sin(a));
  }
}

int ensure_twiddles(ma_plan* P, int n) {
  if (P->tw.count(n)) return MA_OK;
  std::vector<float2> h(n);
  fill_twiddles(h.data(), n);
  float2* d = nullptr;
  if (hipMalloc(&d, sizeof(float2) * n) != hipSuccess) return MA_ENOMEM;
  if (hipMemcpy(d, h.data(), sizeof(float2) * n, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(d);
    return MA_EHIP;
  }
  P->tw[n] = d;
  return MA_OK;
}

// (Im of the first-derivative multiplier, second-derivative multiplier) per FFT index q,
// computed in FP64: 2 pi i k, -(2 pi k)^2 (Section 4.2), or the fourth-order
// difference symbols i (8 sin t - sin 2t)/(6h), (-64 sin^2(t/2) + 4 sin^2 t)/(12 h^2),
// t = 2 pi k h; the first-derivative multiplier is zero at k = -N/2 in both.
void fill_multipliers(float2* h, int n, int symbol) {
  for (int q = 0; q < n; ++q) {
    const double ks = q < n / 2 ? q : q - n;
    double d1, d2;
    if (symbol == MA_SYMBOL_FD4) {
      const double t = 2.0 * M_PI * ks / n;
      d1 = (8.0 * std::sin(t) - std::sin(2.0 * t)) * n / 6.0;
      const double s1 = std::sin(0.5 * t), s2 = std::sin(t);
      d2 = (-64.0 * s1 * s1 + 4.0 * s2 * s2) * (double)n * n / 12.0;
    } else {
      d1 = 2.0 * M_PI * ks;
      d2 = -(2.0 * M_PI * ks) * (2.0 * M_PI * ks);
    }
    if (q == n / 2) d1 = 0.0;
    h[q] = make_float2((float)d1, (float)d2);
  }
}

int ensure_multipliers(ma_plan* P, int n, int symbol) {
  const auto key = std::make_pair(n, symbol);
  if (P->mt.count(key)) return MA_OK;
  std::vector<float2> h(n);
  fill_multipliers(h.data(), n, symbol);
  float2* d = nullptr;
  if (hipMalloc(&d, sizeof(float2) * n) != hipSuccess) return MA_ENOMEM;
  if (hipMemcpy(d, h.data(), sizeof(float2) * n, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(d);
    return MA_EHIP;
  }
  P->mt[key] = d;
  return MA_OK;
}

// workspace for `ns` pairs; descriptors carved in order
int ensure_workspace(ma_plan* P, const std::vector<int>& ns) {
  const int m = P->opt.gmres_m;
  size_t need = 0;
  for (int n : ns) need += pair_bytes(n, m, uses_bicg(P->opt));
  if (need > P->arena_bytes) {
    if (P->arena) (void)hipFree(P->arena);
    P->arena = nullptr;
    P->arena_bytes = 0;
    if (hipMalloc(&P->arena, need) != hipSuccess) return MA_ENOMEM;
    P->arena_bytes = need;
  }
  const int np = (int)ns.size();
  if (np > P->pairs_cap) {
    if (P->d_desc) (void)hipFree(P->d_desc);
    if (P->d_state) (void)hipFree(P->d_state);
    if (P->d_ids) (void)hipFree(P->d_ids);
    if (P->d_lists) (void)hipFree(P->d_lists);
    P->d_desc = nullptr;
    P->d_state = nullptr;
    P->d_ids = nullptr;
    P->d_lists = nullptr;
    P->pairs_cap = 0;
    if (hipMalloc(&P->d_desc, sizeof(PairDesc) * np) != hipSuccess) return MA_ENOMEM;
    if (hipMalloc(&P->d_state, sizeof(PairState) * np) != hipSuccess) return MA_ENOMEM;
    if (hipMalloc(&P->d_ids, sizeof(int) * np) != hipSuccess) return MA_ENOMEM;
    // live, solving, class table (2), counts (2), running, running counts
    if (hipMalloc(&P->d_lists, sizeof(int) * 8 * (size_t)np) != hipSuccess) return MA_ENOMEM;
    P->pairs_cap = np;
  }
  P->h_desc.assign(np, PairDesc{});
  char* p = P->arena;
  for (int q = 0; q < np; ++q) carve(P->h_desc[q], p, ns[q], P->opt.gmres_m, uses_bicg(P->opt));
  for (int n : ns) {
    int e = ensure_twiddles(P, n);
    if (!e) e = ensure_multipliers(P, n, P->opt.symbol);
    if (e) return e;
  }
  return MA_OK;
}

LaunchCtx make_ctx(const ma_plan* P, const Class& cl, int kind = MA_PROF_NONE, bool timed = false) {
  LaunchCtx c;
  // counter 0: the class's untimed launches, counter 1: its timed ones
  c.prof_bytes = (kind != MA_PROF_NONE && kind == P->prof_kind) ? P->d_prof + (timed ? 1 : 0) : nullptr;
  c.desc = P->d_desc;
  c.st = P->d_state;
  c.pair_ids = cl.d_ids;
  c.active_n = cl.active_n;
  c.mt = cl.mt;
  c.m = P->opt.gmres_m;
  c.max_newton = P->opt.max_newton;
  c.max_restarts = P->opt.gmres_max_restarts;
  c.max_backtrack = P->opt.max_backtrack;
  c.damping_policy = P->opt.damping_policy;
  c.interp = P->opt.interp;
  c.op_mode = P->opt.op_mode;
  c.gmres_tol = P->opt.gmres_tol;
  c.precond = P->opt.precond;
  c.boundary_frac = P->opt.boundary_frac;
  c.forcing = P->opt.forcing;
  c.bicg_max = P->opt.bicg_max_iters;
  c.dots_nblk = 0;  // set by the Arnoldi step's launcher
  auto t = P->tune.find(cl.n);
  for (int k = 0; k < 4; ++k) c.var[k] = t == P->tune.end() ? 0 : t->second.v[k];
  return c;
}

PairState fresh_state(double tau, double tol) {
  PairState s;
  std::memset(&s, 0, sizeof(s));
  s.phase = PH_INIT;
  s.status = MA_ENOCONV;
  s.tau0 = tau;
  s.tau = tau;
  s.tol = tol;
  s.step = 1.0;
  s.mean_f = s.mean_g = 1.0;
  return s;
}

// groups pairs by size; uploads id lists
int build_classes(ma_plan* P, const std::vector<int>& ns, std::vector<Class>& cls, hipStream_t st) {
  std::map<int, std::vector<int>> by;
  for (int q = 0; q < (int)ns.size(); ++q) by[ns[q]].push_back(q);
  std::vector<int> flat;
  for (auto& kv : by) {
    Class c;
    c.n = kv.first;
    c.count = (int)kv.second.size();
    c.tw = P->tw[c.n];
    c.mt = P->mt[std::make_pair(c.n, P->opt.symbol)];
    c.d_ids = P->d_ids + flat.size();
    flat.insert(flat.end(), kv.second.begin(), kv.second.end());
    cls.push_back(c);
  }
  HIP_TRY(hipMemcpyAsync(P->d_ids, flat.data(), sizeof(int) * flat.size(), hipMemcpyHostToDevice, st));
  return MA_OK;
}

// events stamped at the start and end of each launch of the timed class
TimedLaunch prof_events(ma_plan* P, int kind) {
  TimedLaunch ev;
  if (kind == MA_PROF_NONE || kind != P->prof_kind) return ev;
  while ((int)P->ev.size() < 2 * (P->ev_used + 1)) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return TimedLaunch();
    P->ev.push_back(e);
  }
  ev.start = P->ev[2 * P->ev_used];
  ev.stop = P->ev[2 * P->ev_used + 1];
  P->ev_used++;
  return ev;
}
// after a stream synchronisation: fold the recorded launches into the totals
void prof_flush(ma_plan* P) {
  for (int i = 0; i < P->ev_used; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, P->ev[2 * i], P->ev[2 * i + 1]) == hipSuccess) P->prof_ms += ms;
    P->prof_launches++;
  }
  P->ev_used = 0;
}

// whether this launch of class `kind` is timed (it is the timed class and its turn in
// the sampling stride): decided once, so that the timed byte counter and the events
// cover the same launches
bool prof_pick(ma_plan* P, int kind) {
  if (kind != P->prof_kind || kind == MA_PROF_NONE) return false;
  return (P->prof_seq++ % P->prof_every) == 0;
}

void L_res(ma_plan* P, const Class& c, int step_mode, hipStream_t st) {
  const bool t = prof_pick(P, MA_PROF_RESIDUAL);
  launch_residual(make_ctx(P, c, MA_PROF_RESIDUAL, t), c.n, c.count, step_mode, st,
                  prof_events(P, t ? MA_PROF_RESIDUAL : MA_PROF_NONE));
}
void L_A(ma_plan* P, const Class& c, int mode, int jn, hipStream_t st) {
  const bool t = prof_pick(P, MA_PROF_ROW_A);
  launch_passA(make_ctx(P, c, MA_PROF_ROW_A, t), c.n, c.count, mode, jn, c.tw, st,
               prof_events(P, t ? MA_PROF_ROW_A : MA_PROF_NONE));
}
void L_B(ma_plan* P, const Class& c, int mode, int j, hipStream_t st) {
  const bool t = prof_pick(P, MA_PROF_COLUMN);
  launch_passB(make_ctx(P, c, MA_PROF_COLUMN, t), c.n, c.count, mode, j, c.tw, st,
               prof_events(P, t ? MA_PROF_COLUMN : MA_PROF_NONE));
}
void L_C(ma_plan* P, const Class& c, int mode, int j, hipStream_t st) {
  const bool t = prof_pick(P, MA_PROF_ROW_C);
  launch_passC(make_ctx(P, c, MA_PROF_ROW_C, t), c.n, c.count, mode, j, c.tw, st,
               prof_events(P, t ? MA_PROF_ROW_C : MA_PROF_NONE));
}
void L_bicg(ma_plan* P, const Class& c, int step, int j, hipStream_t st) {
  const bool t = step == BI_MATVEC && prof_pick(P, MA_PROF_BICG_MATVEC);
  launch_bicg(make_ctx(P, c, step == BI_MATVEC ? MA_PROF_BICG_MATVEC : MA_PROF_NONE, t), c.n, c.count, step, j, st,
              prof_events(P, t ? MA_PROF_BICG_MATVEC : MA_PROF_NONE));
}

// Waits until slot `slot` of the summary holds the counts of the launch numbered
// `seq` by polling its tag in host memory (no stream synchronisation: the host
// resumes as soon as the kernel's fenced write lands).  Every 64 polls the wall
// clock is read and every 256 the stream is queried, so that a failed or drained
// stream, or a wait longer than the plan's wait_limit_s, ends the wait with MA_EHIP
// (the queued work is not cancelled: it runs on to its end).
int wait_summary(ma_plan* P, int slot, int seq, hipStream_t st) {
  int* tag = P->h_summary + MA_SUMMARY_INTS * slot + MA_SUMMARY_TAG;
  const auto t0 = std::chrono::steady_clock::now();
  for (unsigned spin = 1;; ++spin) {
    if (__atomic_load_n(tag, __ATOMIC_ACQUIRE) == seq) return MA_OK;
    if ((spin & 63) == 0 &&
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() > P->opt.wait_limit_s)
      return MA_EHIP;
    if ((spin & 255) == 0) {
      const hipError_t q = hipStreamQuery(st);
      if (q == hipSuccess) return __atomic_load_n(tag, __ATOMIC_ACQUIRE) == seq ? MA_OK : MA_EHIP;
      if (q != hipErrorNotReady) return MA_EHIP;
    }
    __builtin_ia32_pause();
  }
}

// the next summary sequence number (1 .. INT_MAX, then 1 again: a slot always holds a
// recent number, so a restarted count cannot meet a stale tag)
int next_seq(ma_plan* P) {
  P->sum_seq = P->sum_seq == 2147483647 ? 1 : P->sum_seq + 1;
  return P->sum_seq;
}

int read_summary(ma_plan* P, int npairs, hipStream_t st, int* phases = nullptr) {
  const int seq = next_seq(P);
  launch_summary(P->d_state, P->d_ids, npairs, P->d_summary, seq, st, phases);
  if (!P->no_alloc) return wait_summary(P, 0, seq, st);
  // device-memory summary: copy it back and wait for the stream, within wait_limit_s
  HIP_TRY(hipMemcpyAsync(P->h_summary, P->d_summary, sizeof(int) * MA_SUMMARY_INTS, hipMemcpyDeviceToHost, st));
  const auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    const hipError_t q = hipStreamQuery(st);
    if (q == hipSuccess) break;
    if (q != hipErrorNotReady ||
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() > P->opt.wait_limit_s)
      return MA_EHIP;
    __builtin_ia32_pause();
  }
  return P->h_summary[MA_SUMMARY_TAG] == seq ? MA_OK : MA_EHIP;
}

// The class table of the compaction kernel: (offset of each class's id slice, count).
int upload_class_table(ma_plan* P, ClassList cls, int npairs, hipStream_t st) {
  std::vector<int2>& t = P->h_ctab;
  if (t.size() < (size_t)cls.n) t.resize(cls.n);  // never in the no-allocation mode (one class)
  for (int k = 0; k < cls.n; ++k) t[k] = make_int2((int)(cls.p[k].d_ids - P->d_ids), cls.p[k].count);
  HIP_TRY(hipMemcpyAsync(P->d_lists + 2 * (size_t)P->pairs_cap, t.data(), sizeof(int2) * cls.n,
                         hipMemcpyHostToDevice, st));
  return MA_OK;
}

// After a summary: the live and solving lists of every class, and the views of the
// classes that the next launches use (grids bounded by the totals the summary gave)
void compact_views(ma_plan* P, ClassList cls, int n_live, int n_solve, std::vector<Class>& live,
                   std::vector<Class>& solving, hipStream_t st) {
  const size_t cap = P->pairs_cap;
  int* lists = P->d_lists;
  int* cnt = P->d_lists + 2 * cap + 2 * cap;  // after the (offset, count) table
  launch_compact(P->d_state, P->d_ids, (const int2*)(P->d_lists + 2 * cap), cls.n, lists, lists + cap, cnt, st);
  live.assign(cls.begin(), cls.end());
  solving.assign(cls.begin(), cls.end());
  for (int k = 0; k < cls.n; ++k) {
    const size_t off = (size_t)(cls.p[k].d_ids - P->d_ids);
    live[k].d_ids = lists + off;
    live[k].active_n = cnt + 2 * k;
    live[k].count = std::min(cls.p[k].count, n_live);
    solving[k].d_ids = lists + cap + off;
    solving[k].active_n = cnt + 2 * k + 1;
    solving[k].count = std::min(cls.p[k].count, n_solve);
  }
}

// The iterations of one GMRES cycle.  From the third on, a summary of the state is
// queued after each iteration, and the host reads the one queued two iterations
// earlier (so the device queue never drains while the host waits): once no pair is
// inside the cycle, the remaining iterations, which would all exit at once, are not
// launched.  At most two such iterations are queued.  Pairs leave the cycle at
// different iterations; once that summary shows fewer than three quarters of a
// launch's pairs still inside, the launch lists are compacted on the device to those
// pairs and the grids sized by the summary's count (an upper bound for every later
// iteration of the cycle), so that the blocks of pairs that left are not launched.
int launch_cycle_body(ma_plan* P, ClassList cls, int npairs, hipStream_t st) {
  const int m = P->opt.gmres_m;
  constexpr int LAG = 2, FIRST = 2;
  std::vector<Class> run(cls.begin(), cls.end());  // the launch views of the iterations
  const size_t cap = P->pairs_cap;
  for (int j = 0; j < m; ++j) {
    for (const Class& c : run) {
      L_B(P, c, PB_MATVEC, j, st);
      L_C(P, c, PC_MATVEC, j, st);
      L_A(P, c, PA_ARNOLDI, j + 1, st);
    }
    // (the no-allocation mode has no mapped summary: every iteration is launched, and
    // those after a pair's convergence exit at once)
    if (j + 1 >= m || j < FIRST || P->no_alloc) continue;
    const int slot = j % (LAG + 1);
    P->ring_seq[slot] = next_seq(P);
    launch_summary(P->d_state, P->d_ids, npairs, P->d_summary + MA_SUMMARY_INTS * (1 + slot), P->ring_seq[slot],
                   st);
    if (j >= FIRST + LAG) {
      const int old = (j - LAG) % (LAG + 1);
      const int e = wait_summary(P, 1 + old, P->ring_seq[old], st);
      if (e) return e;
      const int nrun = P->h_summary[MA_SUMMARY_INTS * (1 + old) + 8];
      if (nrun == 0) break;
      // running lists after this iteration, in the plan's lists past the counts: each
      // class's slice at the offset of its pairs among all launched (the views' counts
      // sum to at most the capacity)
      int* lists = P->d_lists + 6 * cap;
      int* counts = P->d_lists + 7 * cap;
      size_t off = 0;
      for (int k = 0; k < cls.n; ++k) {
        const Class& c = cls.p[k];
        if (4 * nrun < 3 * run[k].count) {
          launch_compact_running(P->d_state, c.d_ids, c.active_n, c.count, lists + off, counts + k, st);
          run[k].d_ids = lists + off;
          run[k].active_n = counts + k;
          run[k].count = nrun;
        }
        off += (size_t)c.count;
      }
    }
  }
  return MA_OK;
}

// BiCG iterations of the finite-difference step (Section 4.1).  As for GMRES, a summary
// is queued after every iteration and the host reads the one queued two iterations
// earlier; once no pair is still iterating, no further iteration is launched.  In the
// no-allocation mode (no mapped summary) the stream is drained every 16 iterations.
int launch_bicg_body(ma_plan* P, ClassList cls, int npairs, hipStream_t st) {
  constexpr int LAG = 2, NOALLOC_PERIOD = 16;
  for (int j = 0; j < P->opt.bicg_max_iters; ++j) {
    for (const Class& c : cls) {
      L_bicg(P, c, BI_MATVEC, j, st);
      L_bicg(P, c, BI_UPDATE, j, st);
    }
    if (P->no_alloc) {
      if ((j + 1) % NOALLOC_PERIOD) continue;
      const int e = read_summary(P, npairs, st);
      if (e) return e;
      if (P->h_summary[8] == 0) break;
      continue;
    }
    const int slot = j % (LAG + 1);
    P->ring_seq[slot] = next_seq(P);
    launch_summary(P->d_state, P->d_ids, npairs, P->d_summary + MA_SUMMARY_INTS * (1 + slot), P->ring_seq[slot],
                   st);
    if (j >= LAG) {
      const int old = (j - LAG) % (LAG + 1);
      const int e = wait_summary(P, 1 + old, P->ring_seq[old], st);
      if (e) return e;
      if (P->h_summary[MA_SUMMARY_INTS * (1 + old) + 8] == 0) break;
    }
  }
  return MA_OK;
}

// The linear step of one Newton iteration for the solving pairs: theta written, u += theta
int linear_step(ma_plan* P, const std::vector<Class>& vsolve, int npairs, hipStream_t st) {
  const ClassList sl{vsolve.data(), (int)vsolve.size()};
  if (uses_bicg(P->opt)) {
    for (const Class& c : vsolve) L_bicg(P, c, BI_INIT, 0, st);
    int e = launch_bicg_body(P, sl, npairs, st);
    if (e) return e;
    for (const Class& c : vsolve) L_bicg(P, c, BI_FINISH, 0, st);
    return MA_OK;
  }
  for (const Class& c : vsolve) L_A(P, c, PA_INIT, 0, st);
  int e = launch_cycle_body(P, sl, npairs, st);
  if (e) return e;
  for (int cyc = 0; cyc < P->opt.gmres_max_restarts; ++cyc) {
    e = read_summary(P, npairs, st);
    if (e) return e;
    if (P->h_summary[6] == 0) break;
    for (const Class& c : vsolve) {
      launch_restart(make_ctx(P, c), c.n, c.count, st);
      L_A(P, c, PA_PLAIN, 0, st);
    }
    e = launch_cycle_body(P, sl, npairs, st);
    if (e) return e;
  }
  for (const Class& c : vsolve) {
    L_A(P, c, PA_RECOVER, 0, st);
    L_B(P, c, PB_RECOVER, 0, st);
    L_C(P, c, PC_RECOVER, 0, st);
  }
  return MA_OK;
}

// the whole damped Newton loop for the pairs already described in P->h_desc
int run_solver(ma_plan* P, int npairs, double damping, double tol, hipStream_t st, ClassList cls) {
  HIP_TRY(hipMemcpyAsync(P->d_desc, P->h_desc.data(), sizeof(PairDesc) * npairs, hipMemcpyHostToDevice, st));
  P->h_state.assign(npairs, fresh_state(damping, tol));
  for (int q = 0; q < npairs; ++q) P->h_state[q].warm = P->h_desc[q].psi0_in != nullptr;
  HIP_TRY(hipMemcpyAsync(P->d_state, P->h_state.data(), sizeof(PairState) * npairs, hipMemcpyHostToDevice, st));
  for (const Class& c : cls) launch_setup(make_ctx(P, c), c.n, c.count, st);
  int e = read_summary(P, npairs, st);
  if (e) return e;
  if (P->h_summary[7] > 0) return MA_EINVAL;
  e = upload_class_table(P, cls, npairs, st);
  if (e) return e;

  // launches of each tick over the pairs that take part: the residual and the step
  // updates over the live pairs, the GMRES kernels over the solving ones (compacted
  // lists after every residual's summary; the first residual takes every pair)
  std::vector<Class> vlive(cls.begin(), cls.end()), vsolve;
  const long max_ticks = (long)(P->opt.max_newton + 1) * (P->opt.max_backtrack + 3) + 8;
  for (long tick = 0; tick < max_ticks; ++tick) {
    for (const Class& c : vlive) L_res(P, c, 0, st);
    e = read_summary(P, npairs, st);
    if (e) return e;
    const int n_solve = P->h_summary[PH_SOLVE];
    const int n_update = P->h_summary[PH_BACKTRACK] + P->h_summary[PH_REVERT];
    if (n_solve == 0 && n_update == 0) break;  // every pair is done
    compact_views(P, cls, npairs - P->h_summary[PH_DONE], n_solve, vlive, vsolve, st);
    if (n_solve > 0) {
      e = linear_step(P, vsolve, npairs, st);
      if (e) return e;
    }
    if (n_update > 0)
      for (const Class& c : vlive) launch_step_update(make_ctx(P, c), c.n, c.count, st);
  }
  for (const Class& c : cls) launch_outputs(make_ctx(P, c), c.n, c.count, st);
  HIP_TRY(hipMemcpyAsync(P->h_state.data(), P->d_state, sizeof(PairState) * npairs, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  prof_flush(P);
  return MA_OK;
}

// buffers of the continuous mode, grown on demand
int ensure_continuous(ma_plan* P, int npairs, int nslots, size_t stage_bytes) {
  if (npairs > P->final_cap) {
    if (P->d_final) (void)hipFree(P->d_final);
    P->d_final = nullptr;
    P->final_cap = 0;
    if (hipMalloc(&P->d_final, sizeof(PairState) * npairs) != hipSuccess) return MA_ENOMEM;
    P->final_cap = npairs;
  }
  if (nslots > P->phase_cap) {
    if (P->h_phase) (void)hipHostFree(P->h_phase);
    P->h_phase = P->d_phase = nullptr;
    P->phase_cap = 0;
    if (hipHostMalloc(&P->h_phase, sizeof(int) * nslots, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
        hipHostGetDevicePointer((void**)&P->d_phase, P->h_phase, 0) != hipSuccess)
      return MA_ENOMEM;
    P->phase_cap = nslots;
  }
  if (stage_bytes > P->stage_cap) {
    if (P->h_stage) (void)hipHostFree(P->h_stage);
    if (P->d_stage) (void)hipFree(P->d_stage);
    P->h_stage = P->d_stage = nullptr;
    P->stage_cap = 0;
    if (hipHostMalloc(&P->h_stage, stage_bytes, hipHostMallocDefault) != hipSuccess ||
        hipMalloc(&P->d_stage, stage_bytes) != hipSuccess)
      return MA_ENOMEM;
    P->stage_cap = stage_bytes;
  }
  return MA_OK;
}

// The caller's pair q in slot s: its buffers, a fresh state (the initial potential, if
// any, as a checked start)
void fill_slot(ma_plan* P, int s, int q, const double* const* f, const double* const* g, const double* const* psi0,
               double* const* psi, double* const* map, double damping, double tol, PairDesc& d, PairState& st) {
  d = P->h_desc[s];  // the slot's workspace
  d.pair = q;
  d.f_in = f[q];
  d.g_in = g[q];
  d.psi0_in = psi0 ? psi0[q] : nullptr;
  d.psi_out = psi[q];
  d.map_out = map ? map[q] : nullptr;
  st = fresh_state(damping, tol);
  st.warm = d.psi0_in != nullptr;
}

// Continuous batching (option max_active): at most max_active pairs are in flight, in
// slots shared among the size classes in proportion to their pair counts; when the
// summary after a residual shows a slot's pair finished, its outputs and final state
// are written (k_retire) and the slot takes the next pending pair of its size
// (k_refill, then the set-up kernels for those slots), which enters the next tick's
// residual.  Each pair's arithmetic is that of run_solver.  All inputs are validated
// first, so that an invalid density is a hard error before anything is written.
int run_continuous(ma_plan* P, int npairs, const std::vector<int>& ns, const double* const* f,
                   const double* const* g, const double* const* psi0, double* const* psi, double* const* map,
                   double damping, double tol, hipStream_t st, std::vector<PairState>& final_states) {
  struct Queue {
    int n, first_slot, nslots;
    std::vector<int> pairs;
    size_t next = 0;
  };
  std::map<int, std::vector<int>> by;
  for (int q = 0; q < npairs; ++q) by[ns[q]].push_back(q);
  std::vector<int> slot_n;
  std::vector<Queue> qs;
  for (auto& kv : by) {
    Queue q;
    q.n = kv.first;
    q.pairs = kv.second;
    const long share = std::lround((double)P->opt.max_active * (double)kv.second.size() / (double)npairs);
    q.nslots = (int)std::max(1L, std::min((long)kv.second.size(), share));
    q.first_slot = (int)slot_n.size();
    for (int k = 0; k < q.nslots; ++k) slot_n.push_back(q.n);
    qs.push_back(q);
  }
  const int S = (int)slot_n.size();
  int e = ensure_workspace(P, slot_n);
  if (e) return e;
  const size_t val_bytes = align256((size_t)npairs * (3 * sizeof(void*) + sizeof(int))) + 256;
  const size_t tick_bytes = align256((size_t)S * 2 * sizeof(int)) + (size_t)S * sizeof(RefillRecord);
  e = ensure_continuous(P, npairs, S, std::max(val_bytes, tick_bytes));
  if (e) return e;
  // 1. every pair's inputs
  {
    char* h = P->h_stage;
    const void** hf = (const void**)h;
    const void** hg = hf + npairs;
    const void** hp = hg + npairs;
    int* hn = (int*)(hp + npairs);
    int* hbad = (int*)(h + val_bytes - 256);
    for (int q = 0; q < npairs; ++q) {
      hf[q] = f[q];
      hg[q] = g[q];
      hp[q] = psi0 ? psi0[q] : nullptr;
      hn[q] = ns[q];
    }
    *hbad = 0;
    HIP_TRY(hipMemcpyAsync(P->d_stage, h, val_bytes, hipMemcpyHostToDevice, st));
    const double* const* df = (const double* const*)P->d_stage;
    int nmax = 0;
    for (int n : ns) nmax = std::max(nmax, n);
    launch_validate(df, df + npairs, psi0 ? df + 2 * npairs : nullptr, (const int*)(df + 3 * npairs), npairs, nmax,
                    (int*)(P->d_stage + val_bytes - 256), st);
    int bad = 0;
    HIP_TRY(hipMemcpyAsync(&bad, P->d_stage + val_bytes - 256, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (bad) return MA_EINVAL;
  }
  // 2. slots 0..S-1 in class order, filled with the first pairs of each class
  std::vector<int> ids(S);
  for (int s = 0; s < S; ++s) ids[s] = s;
  HIP_TRY(hipMemcpyAsync(P->d_ids, ids.data(), sizeof(int) * S, hipMemcpyHostToDevice, st));
  std::vector<Class> cls;
  for (const Queue& q : qs) {
    Class c;
    c.n = q.n;
    c.count = q.nslots;
    c.d_ids = P->d_ids + q.first_slot;
    c.tw = P->tw[q.n];
    c.mt = P->mt[std::make_pair(q.n, P->opt.symbol)];
    cls.push_back(c);
  }
  std::vector<int> slot_pair(S, -1);
  std::vector<PairDesc> hd(S);
  P->h_state.assign(S, PairState{});
  for (Queue& q : qs)
    for (int k = 0; k < q.nslots; ++k) {
      const int s = q.first_slot + k, pr = q.pairs[q.next++];
      fill_slot(P, s, pr, f, g, psi0, psi, map, damping, tol, hd[s], P->h_state[s]);
      slot_pair[s] = pr;
    }
  HIP_TRY(hipMemcpyAsync(P->d_desc, hd.data(), sizeof(PairDesc) * S, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(P->d_state, P->h_state.data(), sizeof(PairState) * S, hipMemcpyHostToDevice, st));
  for (const Class& c : cls) launch_setup(make_ctx(P, c), c.n, c.count, st);
  e = upload_class_table(P, ClassList{cls.data(), (int)cls.size()}, S, st);
  if (e) return e;
  std::vector<Class> vlive(cls.begin(), cls.end()), vsolve;
  // 3. ticks; a refilled slot enters the next tick's residual
  const long per_pair = (long)(P->opt.max_newton + 1) * (P->opt.max_backtrack + 3) + 8;
  const long max_ticks = per_pair * (long)((npairs + S - 1) / S + 1);
  int retired = 0;
  const ClassList cl{cls.data(), (int)cls.size()};
  for (long tick = 0; tick < max_ticks && retired < npairs; ++tick) {
    for (const Class& c : vlive) L_res(P, c, 0, st);
    e = read_summary(P, S, st, P->d_phase);
    if (e) return e;
    const int n_solve = P->h_summary[PH_SOLVE];
    const int n_update = P->h_summary[PH_BACKTRACK] + P->h_summary[PH_REVERT];
    // finished slots: retire their pairs and refill from the class's queue
    int* rid = (int*)P->h_stage;
    int* fid = rid + S;
    RefillRecord* rec = (RefillRecord*)(P->h_stage + align256((size_t)S * 2 * sizeof(int)));
    std::vector<int> nret(qs.size(), 0), nref(qs.size(), 0), ret_at(qs.size()), ref_at(qs.size());
    int nr = 0, nf = 0;
    for (size_t k = 0; k < qs.size(); ++k) {
      Queue& q = qs[k];
      ret_at[k] = nr;
      for (int s = q.first_slot; s < q.first_slot + q.nslots; ++s)
        if (slot_pair[s] >= 0 && P->h_phase[s] == PH_DONE) rid[nr++] = s;
      nret[k] = nr - ret_at[k];
      ref_at[k] = nf;
      for (int r = ret_at[k]; r < nr; ++r) {
        const int s = rid[r];
        slot_pair[s] = -1;
        ++retired;
        if (q.next < q.pairs.size()) {
          const int pr = q.pairs[q.next++];
          rec[nf].slot = s;
          fill_slot(P, s, pr, f, g, psi0, psi, map, damping, tol, rec[nf].desc, rec[nf].state);
          fid[nf++] = s;
          slot_pair[s] = pr;
        }
      }
      nref[k] = nf - ref_at[k];
    }
    if (nr > 0) {
      const size_t bytes = align256((size_t)S * 2 * sizeof(int)) + (size_t)nf * sizeof(RefillRecord);
      HIP_TRY(hipMemcpyAsync(P->d_stage, P->h_stage, bytes, hipMemcpyHostToDevice, st));
      const int* d_rid = (const int*)P->d_stage;
      const int* d_fid = d_rid + S;
      for (size_t k = 0; k < qs.size(); ++k)
        if (nret[k]) {
          LaunchCtx x = make_ctx(P, cls[k]);
          x.pair_ids = d_rid + ret_at[k];
          launch_retire(x, qs[k].n, nret[k], P->d_final, st);
        }
      if (nf) {
        launch_refill(P->d_desc, P->d_state,
                      (const RefillRecord*)(P->d_stage + align256((size_t)S * 2 * sizeof(int))), nf, st);
        for (size_t k = 0; k < qs.size(); ++k)
          if (nref[k]) {
            LaunchCtx x = make_ctx(P, cls[k]);
            x.pair_ids = d_fid + ref_at[k];
            launch_setup(x, qs[k].n, nref[k], st);
          }
      }
    }
    // after the refills: the live slots (a pair in them) and the solving ones
    int n_live = 0;
    for (int s = 0; s < S; ++s) n_live += slot_pair[s] >= 0;
    compact_views(P, cl, n_live, n_solve, vlive, vsolve, st);
    if (n_solve > 0) {
      e = linear_step(P, vsolve, S, st);
      if (e) return e;
    }
    if (n_update > 0)
      for (const Class& c : vlive) launch_step_update(make_ctx(P, c), c.n, c.count, st);
  }
  if (retired < npairs) {  // the tick limit: write what the unfinished slots hold
    HIP_TRY(hipStreamSynchronize(st));  // the staging buffer's last copy has been read
    int nr = 0;
    int* rid = (int*)P->h_stage;
    for (int s = 0; s < S; ++s)
      if (slot_pair[s] >= 0) rid[nr++] = s;
    HIP_TRY(hipMemcpyAsync(P->d_stage, P->h_stage, sizeof(int) * S, hipMemcpyHostToDevice, st));
    for (size_t k = 0; k < qs.size(); ++k) {
      int cnt = 0, at = -1;
      for (int r = 0; r < nr; ++r)
        if (slot_n[rid[r]] == qs[k].n) {
          if (at < 0) at = r;
          ++cnt;
        }
      if (cnt) {
        LaunchCtx x = make_ctx(P, cls[k]);
        x.pair_ids = (const int*)P->d_stage + at;
        launch_retire(x, qs[k].n, cnt, P->d_final, st);
      }
    }
  }
  final_states.assign(npairs, PairState{});
  HIP_TRY(hipMemcpyAsync(final_states.data(), P->d_final, sizeof(PairState) * npairs, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  prof_flush(P);
  return MA_OK;
}

void fill_report(const PairState& s, ma_report* r, double ms) {
  r->status = s.phase == PH_DONE ? s.status : MA_ENOCONV;
  r->newton_iters = s.newton_iters;
  r->gmres_iters = s.gmres_iters;
  r->backtracks = s.backtracks;
  r->res_rms = s.res_rms;
  r->res_max = s.res_max;
  r->res0_rms = s.res0;
  r->mass_defect = s.mass_c;
  r->min_det = s.min_det;
  r->w2sq = s.w2;
  r->tau_final = s.tau;
  r->time_ms = ms;
  r->warm_steps = s.warm_steps;
}

// one-pair workspace for the step entry points; state copied from `s`
int step_prepare(ma_plan* P, int n, const PairState& s, hipStream_t st, Class& c) {
  if (!n_ok(n)) return MA_EINVAL;
  std::vector<int> ns(1, n);
  int e = ensure_workspace(P, ns);
  if (e) return e;
  std::vector<Class> cls;
  e = build_classes(P, ns, cls, st);
  if (e) return e;
  c = cls[0];
  HIP_TRY(hipMemcpyAsync(P->d_desc, P->h_desc.data(), sizeof(PairDesc), hipMemcpyHostToDevice, st));
  P->h_state.assign(1, s);
  HIP_TRY(hipMemcpyAsync(P->d_state, P->h_state.data(), sizeof(PairState), hipMemcpyHostToDevice, st));
  return MA_OK;
}

PairState step_state(const double* abar) {
  PairState s = fresh_state(1.0, 1.0);
  s.phase = PH_SOLVE;
  s.gm_running = 1;
  s.vscale[0] = 1.0;
  if (abar)
    for (int k = 0; k < 5; ++k) s.abar[k] = abar[k];
  return s;
}

}  // namespace

int plan_lbar_inverse_many(ma_plan* P, int n, int count, const float* const* sigma, const double* abar,
                           float* const* theta, hipStream_t st) {
  if (!P || count < 1 || !sigma || !abar || !theta || !n_ok(n)) return MA_EINVAL;
  std::vector<int> ns(count, n);
  int e = ensure_workspace(P, ns);
  if (e) return e;
  std::vector<Class> cls;
  e = build_classes(P, ns, cls, st);
  if (e) return e;
  for (int q = 0; q < count; ++q) {  // the step modes read only V[0] and write only x
    P->h_desc[q].V = const_cast<float*>(sigma[q]);
    P->h_desc[q].x = theta[q];
  }
  HIP_TRY(hipMemcpyAsync(P->d_desc, P->h_desc.data(), sizeof(PairDesc) * count, hipMemcpyHostToDevice, st));
  P->h_state.assign(count, step_state(abar));
  HIP_TRY(hipMemcpyAsync(P->d_state, P->h_state.data(), sizeof(PairState) * count, hipMemcpyHostToDevice, st));
  LaunchCtx x = make_ctx(P, cls[0]);
  launch_passA(x, n, count, PA_STEP, 0, cls[0].tw, st);
  launch_passB(x, n, count, PB_RECOVER, 0, cls[0].tw, st);
  launch_passC(x, n, count, PC_THETA_ONLY, 0, cls[0].tw, st);
  return hipGetLastError() == hipSuccess ? MA_OK : MA_EHIP;
}

// ---------------------------------------------------------------------------
// No-allocation solves (ma_solve_noalloc): one pair, all device memory carved from
// `scratch`, a file-scope device array of MA_NOALLOC_BYTES that each GPU holds from
// the library's load to the end of the process.  In host code `scratch` names a
// host-side stand-in; its device address comes from hipGetSymbolAddress, once per
// device, with that device current, and only that address is used.
// ---------------------------------------------------------------------------
constexpr size_t MA_NOALLOC_BYTES = (size_t)48 << 20;
constexpr int MA_NOALLOC_DEVICES = 64;
constexpr int MA_NOALLOC_NMAX = 512;

static __device__ __align__(256) char scratch[MA_NOALLOC_BYTES];

namespace {

struct NoAllocSlot {
  char* base = nullptr;  // device address of this GPU's `scratch`
  float2* d_tw = nullptr;
  float2* d_mt = nullptr;
  float2 h_tw[MA_NOALLOC_NMAX], h_mt[MA_NOALLOC_NMAX];  // host sources of the last upload
  int h_zero = 0;
};
NoAllocSlot g_noalloc[MA_NOALLOC_DEVICES];
ma_plan g_noalloc_plan[MA_NOALLOC_DEVICES];

// first call on device `dev`: the address of its scratch array and the carving of the
// fixed regions (pair descriptor, state, id, summary, tables, then the pair's arena)
int noalloc_setup(int dev) {
  NoAllocSlot& S = g_noalloc[dev];
  if (S.base) return MA_OK;
  char* ptr = nullptr;
  if (hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return MA_EHIP;
  ma_plan* P = &g_noalloc_plan[dev];
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* q = ptr + off;
    off += align256(bytes);
    return q;
  };
  P->d_desc = (PairDesc*)take(sizeof(PairDesc));
  P->d_state = (PairState*)take(sizeof(PairState));
  P->d_ids = (int*)take(sizeof(int));
  P->d_summary = (int*)take(sizeof(int) * MA_SUMMARY_INTS);
  P->d_lists = (int*)take(sizeof(int) * 6);  // the compaction lists of one pair
  S.d_tw = (float2*)take(sizeof(float2) * MA_NOALLOC_NMAX);
  S.d_mt = (float2*)take(sizeof(float2) * MA_NOALLOC_NMAX);
  P->arena = ptr + off;
  P->arena_bytes = MA_NOALLOC_BYTES - off;
  P->h_summary = P->h_summary_buf;
  P->pairs_cap = 1;
  P->no_alloc = true;
  P->h_desc.assign(1, PairDesc{});  // host vectors of one entry, sized once here
  P->h_state.assign(1, PairState{});
  P->h_ctab.assign(1, int2{});
  S.base = ptr;
  return MA_OK;
}

}  // namespace

extern "C" {

int ma_abi_version(void) { return MA_OT_ABI_VERSION; }

void ma_options_default(ma_options* o) {
  if (!o) return;
  o->max_newton = 100;
  o->gmres_m = 10;
  o->gmres_max_restarts = 20;
  o->gmres_tol = 1e-4;
  o->interp = MA_INTERP_BILINEAR;
  o->op_mode = MA_OP_FULL;
  o->damping_policy = MA_DAMP_FIXED;
  o->max_backtrack = 12;
  o->symbol = MA_SYMBOL_SPECTRAL;
  o->precond = MA_PRECOND_NONE;
  o->boundary_frac = 0.1;
  o->forcing = MA_FORCING_FIXED;
  o->wait_limit_s = 600.0;
  o->max_active = 0;
  o->linear_solver = MA_LINEAR_STRAIN_GMRES;
  o->bicg_max_iters = 1000;
}

const char* ma_strerror(int code) {
  switch (code) {
    case MA_OK: return "converged";
    case MA_ENOCONV: return "no convergence within the iteration limits";
    case MA_ENONCONVEX: return "iterate lost convexity (det or trace of I + D^2 u not positive)";
    case MA_ENAN: return "non-finite residual";
    case MA_EINVAL: return "invalid argument";
    case MA_ENOMEM: return "device allocation failed";
    case MA_EHIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

int ma_plan_create(int n_max, int batch_capacity, const ma_options* opt, ma_plan** out) {
  if (!out) return MA_EINVAL;
  *out = nullptr;
  if (!n_ok(n_max) || batch_capacity < 1) return MA_EINVAL;
  ma_plan* P = new ma_plan();
  if (opt) P->opt = *opt;
  else ma_options_default(&P->opt);
  if (validate_options(P->opt)) {
    delete P;
    return MA_EINVAL;
  }
  P->n_max = n_max;
  P->cap = batch_capacity;
  if (hipMalloc(&P->d_prof, 2 * sizeof(unsigned long long)) != hipSuccess ||
      hipMemset(P->d_prof, 0, 2 * sizeof(unsigned long long)) != hipSuccess ||
      hipHostMalloc(&P->h_summary, sizeof(int) * 4 * MA_SUMMARY_INTS,
                    hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
      hipHostGetDevicePointer((void**)&P->d_summary, P->h_summary, 0) != hipSuccess) {
    ma_plan_destroy(P);
    return MA_ENOMEM;
  }
  std::memset(P->h_summary, 0, sizeof(int) * 4 * MA_SUMMARY_INTS);  // no tag matches a launch (they start at 1)
  std::vector<int> ns(batch_capacity, n_max);
  int e = ensure_workspace(P, ns);
  if (e) {
    ma_plan_destroy(P);
    return e;
  }
  *out = P;
  return MA_OK;
}

void ma_plan_destroy(ma_plan* P) {
  if (!P) return;
  if (P->arena) (void)hipFree(P->arena);
  if (P->d_desc) (void)hipFree(P->d_desc);
  if (P->d_state) (void)hipFree(P->d_state);
  if (P->d_ids) (void)hipFree(P->d_ids);
  if (P->d_lists) (void)hipFree(P->d_lists);
  if (P->h_summary) (void)hipHostFree(P->h_summary);
  if (P->d_final) (void)hipFree(P->d_final);
  if (P->h_phase) (void)hipHostFree(P->h_phase);
  if (P->h_stage) (void)hipHostFree(P->h_stage);
  if (P->d_stage) (void)hipFree(P->d_stage);
  for (auto& kv : P->tw) (void)hipFree(kv.second);
  for (auto& kv : P->mt) (void)hipFree(kv.second);
  for (hipEvent_t e : P->ev) (void)hipEventDestroy(e);
  if (P->d_prof) (void)hipFree(P->d_prof);
  delete P;
}

int ma_plan_set_options(ma_plan* P, const ma_options* opt) {
  if (!P || !opt || validate_options(*opt)) return MA_EINVAL;
  P->opt = *opt;
  return MA_OK;
}

int ma_plan_autotune(ma_plan* P, int n, int npairs, const char* cache_path, ma_tuning* out, void* stream) {
  if (!P || !out || npairs < 1 || !n_ok(n)) return MA_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  ma_tuning t;
  std::memset(&t, 0, sizeof(t));
  t.n = n;
  t.npairs = npairs;
  if (tune_cache_lookup(cache_path, n, npairs, P->opt.gmres_m, &t)) {
    int u = 0, th = 0;
    bool ok = true;
    for (int k = 0; k < 4; ++k) {
      if (t.variant[k] < 0 || t.variant[k] >= MA_TUNE_VARIANTS) ok = false;
      if (ok && ma_tune_geometry(k, n, t.variant[k], &u, &th) != t.variant[k]) ok = false;
    }
    if (ok) {
      t.from_cache = 1;
      Tune tu;
      for (int k = 0; k < 4; ++k) tu.v[k] = t.variant[k];
      P->tune[n] = tu;
      *out = t;
      return MA_OK;
    }
    std::memset(t.variant, 0, sizeof(t.variant));
  }
  std::vector<int> ns(npairs, n);
  int e = ensure_workspace(P, ns);
  if (e) return e;
  std::vector<Class> cls;
  e = build_classes(P, ns, cls, st);
  if (e) return e;
  HIP_TRY(hipMemcpyAsync(P->d_desc, P->h_desc.data(), sizeof(PairDesc) * npairs, hipMemcpyHostToDevice, st));
  const double lap[5] = {1.0, 0.0, 1.0, 0.0, 0.0};
  PairState s = step_state(lap);
  for (int l = 0; l <= MA_MMAX; ++l) s.vscale[l] = 1.0;
  P->h_state.assign(npairs, s);
  HIP_TRY(hipMemcpyAsync(P->d_state, P->h_state.data(), sizeof(PairState) * npairs, hipMemcpyHostToDevice, st));
  TunerView tv;
  tv.ctx = make_ctx(P, cls[0]);
  for (int k = 0; k < 4; ++k) tv.ctx.var[k] = 0;
  tv.n = n;
  tv.npairs = npairs;
  tv.tw = cls[0].tw;
  tv.desc0 = P->h_desc[0];
  launch_tune_fill(tv.ctx, n, npairs, st);
  e = tune_passes(tv, &t, st);
  if (e) return e;
  Tune tu;
  for (int k = 0; k < 4; ++k) tu.v[k] = t.variant[k];
  P->tune[n] = tu;
  tune_cache_store(cache_path, n, npairs, P->opt.gmres_m, t);
  *out = t;
  return MA_OK;
}

int ma_plan_set_tuning(ma_plan* P, const ma_tuning* t) {
  if (!P || !t || !n_ok(t->n)) return MA_EINVAL;
  Tune tu;
  for (int k = 0; k < 4; ++k) {
    int u = 0, th = 0;
    if (t->variant[k] < 0 || t->variant[k] >= MA_TUNE_VARIANTS || ma_tune_geometry(k, t->n, t->variant[k], &u, &th) < 0)
      return MA_EINVAL;
    tu.v[k] = t->variant[k];
  }
  P->tune[t->n] = tu;
  return MA_OK;
}

int ma_plan_get_tuning(const ma_plan* P, int n, ma_tuning* out) {
  if (!P || !out) return MA_EINVAL;
  std::memset(out, 0, sizeof(*out));
  out->n = n;
  auto it = P->tune.find(n);
  if (it != P->tune.end())
    for (int k = 0; k < 4; ++k) out->variant[k] = it->second.v[k];
  return MA_OK;
}

int ma_plan_profile(ma_plan* P, int kind, int every) {
  if (!P || kind < MA_PROF_NONE || kind > MA_PROF_BICG_MATVEC || every < 1) return MA_EINVAL;
  HIP_TRY(hipDeviceSynchronize());
  P->prof_kind = kind;
  P->prof_every = every;
  P->prof_seq = 0;
  P->prof_ms = 0.0;
  P->prof_launches = 0;
  P->ev_used = 0;
  HIP_TRY(hipMemset(P->d_prof, 0, 2 * sizeof(unsigned long long)));
  return MA_OK;
}

int ma_plan_profile_read(ma_plan* P, double* ms, long long* launches, double* bytes, long long* all_launches,
                         double* all_bytes) {
  if (!P) return MA_EINVAL;
  unsigned long long b[2] = {0, 0};
  HIP_TRY(hipMemcpy(b, P->d_prof, sizeof(b), hipMemcpyDeviceToHost));
  if (ms) *ms = P->prof_ms;
  if (launches) *launches = P->prof_launches;
  if (bytes) *bytes = (double)b[1];
  if (all_launches) *all_launches = P->prof_seq;
  if (all_bytes) *all_bytes = (double)b[0] + (double)b[1];
  return MA_OK;
}

int ma_solve_batched(ma_plan* P, int npairs, const int* n, const double* const* f, const double* const* g,
                     const double* const* psi0, double damping, double tol, double* const* psi,
                     double* const* map, ma_report* reps, void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!P || npairs < 1 || !n || !f || !g || !psi || !(damping >= 1.0) || !(tol > 0.0)) return MA_EINVAL;
  std::vector<int> ns(n, n + npairs);
  for (int q = 0; q < npairs; ++q)
    if (!n_ok(ns[q]) || !f[q] || !g[q] || !psi[q]) return MA_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  if (P->opt.max_active > 0 && P->opt.max_active < npairs) {  // continuous batching
    std::vector<PairState> fin;
    int e = run_continuous(P, npairs, ns, f, g, psi0, psi, map, damping, tol, st, fin);
    if (e) return e;
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    int worst = MA_OK;
    for (int q = 0; q < npairs; ++q) {
      ma_report r;
      fill_report(fin[q], &r, ms);
      if (reps) reps[q] = r;
      worst = std::max(worst, r.status);
    }
    return worst;
  }
  int e = ensure_workspace(P, ns);
  if (e) return e;
  for (int q = 0; q < npairs; ++q) {
    PairDesc& d = P->h_desc[q];
    d.f_in = f[q];
    d.g_in = g[q];
    d.psi0_in = psi0 ? psi0[q] : nullptr;
    d.psi_out = psi[q];
    d.map_out = map ? map[q] : nullptr;
  }
  std::vector<Class> cls;
  e = build_classes(P, ns, cls, st);
  if (e) return e;
  e = run_solver(P, npairs, damping, tol, st, ClassList{cls.data(), (int)cls.size()});
  if (e) return e;
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  int worst = MA_OK;
  for (int q = 0; q < npairs; ++q) {
    ma_report r;
    fill_report(P->h_state[q], &r, ms);
    if (reps) reps[q] = r;
    worst = std::max(worst, r.status);
  }
  return worst;
}

int ma_solve(ma_plan* P, const double* f, const double* g, int n, double damping, double tol,
             const double* psi0, double* psi, double* map, ma_report* rep, void* stream) {
  const double* fa[1] = {f};
  const double* ga[1] = {g};
  const double* pa[1] = {psi0};
  double* oa[1] = {psi};
  double* ma[1] = {map};
  return ma_solve_batched(P, 1, &n, fa, ga, pa, damping, tol, oa, ma, rep, stream);
}

int ma_step_residual(ma_plan* P, int n, const double* u, const double* f, const double* g, float* r,
                     float* coef, double* scalars, void* stream) {
  if (!P || !u || !f || !g) return MA_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  Class c;
  int e = step_prepare(P, n, fresh_state(1.0, 1.0), st, c);
  if (e) return e;
  PairDesc& d = P->h_desc[0];
  d.f_in = f;
  d.g_in = g;
  d.psi0_in = u;  // u0 = u - 0: the state's means are 1 and 0, so f and g are used as given
  HIP_TRY(hipMemcpyAsync(P->d_desc, P->h_desc.data(), sizeof(PairDesc), hipMemcpyHostToDevice, st));
  LaunchCtx x = make_ctx(P, c);
  x.precond = MA_PRECOND_NONE;  // the step entry points apply the operator of Section 4.2
  launch_setup_fields(x, n, 1, st);
  launch_residual(x, n, 1, 1, st);
  if (r) launch_residual_shift(x, n, r, st);
  if (coef) HIP_TRY(hipMemcpyAsync(coef, d.coef, 20 * (size_t)n * n, hipMemcpyDeviceToDevice, st));
  if (scalars) {
    HIP_TRY(hipMemcpyAsync(P->h_state.data(), P->d_state, sizeof(PairState), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const PairState& q = P->h_state[0];
    const double v[12] = {q.res_rms, q.res_max, q.mass_c, q.min_det, q.min_tr, q.abar[0],
                          q.abar[1], q.abar[2], q.abar[3], q.abar[4], q.w2, q.mean_u};
    std::memcpy(scalars, v, sizeof(v));
  }
  return MA_OK;
}

int ma_step_fft2(ma_plan* P, int n, const float* v, float* spec, void* stream) {
  if (!P || !v || !spec) return MA_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  Class c;
  int e = step_prepare(P, n, step_state(nullptr), st, c);
  if (e) return e;
  const PairDesc& d = P->h_desc[0];
  HIP_TRY(hipMemcpyAsync(d.V, v, 4 * (size_t)n * n, hipMemcpyDeviceToDevice, st));
  LaunchCtx x = make_ctx(P, c);
  x.precond = MA_PRECOND_NONE;  // the step entry points apply the operator of Section 4.2
  launch_passA(x, n, 1, PA_STEP, 0, c.tw, st);
  launch_passB(x, n, 1, PB_FORWARD, 0, c.tw, st);
  HIP_TRY(hipMemcpyAsync(spec, d.T, 4 * (size_t)n * n, hipMemcpyDeviceToDevice, st));
  return MA_OK;
}

int ma_step_strain_apply(ma_plan* P, int n, const float* v, const float* coef, const double* abar, float* w,
                         void* stream) {
  if (!P || !v || !coef || !abar || !w) return MA_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  Class c;
  int e = step_prepare(P, n, step_state(abar), st, c);
  if (e) return e;
  const PairDesc& d = P->h_desc[0];
  const size_t nn = (size_t)n * n;
  HIP_TRY(hipMemcpyAsync(d.V, v, 4 * nn, hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipMemcpyAsync(d.coef, coef, 20 * nn, hipMemcpyDeviceToDevice, st));
  LaunchCtx x = make_ctx(P, c);
  x.precond = MA_PRECOND_NONE;  // the step entry points apply the operator of Section 4.2
  launch_passA(x, n, 1, PA_STEP, 0, c.tw, st);
  launch_passB(x, n, 1, PB_MATVEC, 0, c.tw, st);
  launch_passC(x, n, 1, PC_MATVEC, 0, c.tw, st);
  HIP_TRY(hipMemcpyAsync(w, d.V + nn, 4 * nn, hipMemcpyDeviceToDevice, st));
  return MA_OK;
}

int ma_step_lbar_inverse(ma_plan* P, int n, const float* sigma, const double* abar, float* theta,
                         void* stream) {
  if (!P || !sigma || !abar || !theta) return MA_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  Class c;
  int e = step_prepare(P, n, step_state(abar), st, c);
  if (e) return e;
  const PairDesc& d = P->h_desc[0];
  const size_t nn = (size_t)n * n;
  HIP_TRY(hipMemcpyAsync(d.V, sigma, 4 * nn, hipMemcpyDeviceToDevice, st));
  LaunchCtx x = make_ctx(P, c);
  x.precond = MA_PRECOND_NONE;  // the step entry points apply the operator of Section 4.2
  launch_passA(x, n, 1, PA_STEP, 0, c.tw, st);
  launch_passB(x, n, 1, PB_RECOVER, 0, c.tw, st);
  launch_passC(x, n, 1, PC_THETA_ONLY, 0, c.tw, st);
  HIP_TRY(hipMemcpyAsync(theta, d.x, 4 * nn, hipMemcpyDeviceToDevice, st));
  return MA_OK;
}

int ma_step_gmres(ma_plan* P, int n, const float* h, const float* coef, const double* abar, int m, double tol,
                  int max_restarts, float* theta, int* iters, void* stream) {
  if (!P || !h || !coef || !abar || !theta || m < 1 || m > MA_MMAX || !(tol > 0.0) || max_restarts < 0)
    return MA_EINVAL;
  if (!n_ok(n)) return MA_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const size_t nn = (size_t)n * n;
  std::vector<float> hh(nn);
  HIP_TRY(hipMemcpyAsync(hh.data(), h, 4 * nn, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  double b2 = 0.0;
  for (float v : hh) b2 += (double)v * v;
  const double bn = std::sqrt(b2);
  ma_options saved = P->opt;
  P->opt.gmres_m = m;
  P->opt.gmres_max_restarts = max_restarts;
  P->opt.gmres_tol = tol;
  P->opt.precond = MA_PRECOND_NONE;  // the operator of Section 4.2
  PairState s = step_state(abar);
  s.bnorm = bn;
  s.gm_target = tol * bn;
  s.gm_running = bn > 0.0;
  s.vscale[0] = bn > 0.0 ? 1.0 / bn : 0.0;
  s.gv[0] = bn;
  s.mass_c = 0.0;
  Class c;
  int e = step_prepare(P, n, s, st, c);
  if (e) {
    P->opt = saved;
    return e;
  }
  const PairDesc& d = P->h_desc[0];
  std::vector<Class> cls(1, c);
  int rc = MA_OK;
  do {
    if (hipMemcpyAsync(d.r, h, 4 * nn, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(d.coef, coef, 20 * nn, hipMemcpyDeviceToDevice, st) != hipSuccess) {
      rc = MA_EHIP;
      break;
    }
    LaunchCtx x = make_ctx(P, c);
    x.precond = MA_PRECOND_NONE;  // the step entry points apply the operator of Section 4.2
    launch_passA(x, n, 1, PA_INIT, 0, c.tw, st);
    if ((rc = launch_cycle_body(P, ClassList{cls.data(), 1}, 1, st))) break;
    for (int cyc = 0; cyc < max_restarts; ++cyc) {
      if ((rc = read_summary(P, 1, st))) break;
      if (P->h_summary[6] == 0) break;
      launch_restart(x, n, 1, st);
      launch_passA(x, n, 1, PA_PLAIN, 0, c.tw, st);
      if ((rc = launch_cycle_body(P, ClassList{cls.data(), 1}, 1, st))) break;
    }
    if (rc) break;
    launch_passA(x, n, 1, PA_RECOVER, 0, c.tw, st);
    launch_passB(x, n, 1, PB_RECOVER, 0, c.tw, st);
    launch_passC(x, n, 1, PC_THETA_ONLY, 0, c.tw, st);
    if (hipMemcpyAsync(theta, d.x, 4 * nn, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(P->h_state.data(), P->d_state, sizeof(PairState), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      rc = MA_EHIP;
      break;
    }
    if (iters) *iters = P->h_state[0].gmres_iters;
  } while (0);
  P->opt = saved;
  return rc;
}

int ma_step_fd_apply(ma_plan* P, int n, const double* p, const double* pt, const float* coef, double* q,
                     double* qt, void* stream) {
  if (!P || !p || !pt || !coef || !q || !qt || !n_ok(n)) return MA_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const size_t nn = (size_t)n * n;
  std::vector<double> hp(nn), hpt(nn);
  HIP_TRY(hipMemcpyAsync(hp.data(), p, 8 * nn, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(hpt.data(), pt, 8 * nn, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  double sp = 0.0, spt = 0.0;
  for (size_t k = 0; k < nn; ++k) {
    sp += hp[k];
    spt += hpt[k];
  }
  const ma_options saved = P->opt;
  P->opt.linear_solver = MA_LINEAR_FD_BICG;
  P->opt.precond = MA_PRECOND_NONE;
  PairState s = step_state(nullptr);
  s.bi_sum_p[0] = sp;
  s.bi_sum_pt[0] = spt;
  Class c;
  int rc = step_prepare(P, n, s, st, c);
  if (!rc) {
    const PairDesc& d = P->h_desc[0];
    // planes of PairDesc::bv: p_0, p~_0 in 5, 6; q, q~ in 3, 4
    if (hipMemcpyAsync(d.bv + 5 * nn, p, 8 * nn, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(d.bv + 6 * nn, pt, 8 * nn, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(d.coef, coef, 20 * nn, hipMemcpyDeviceToDevice, st) != hipSuccess) {
      rc = MA_EHIP;
    } else {
      launch_bicg(make_ctx(P, c), n, 1, BI_MATVEC, 0, st);
      if (hipGetLastError() != hipSuccess ||
          hipMemcpyAsync(q, d.bv + 3 * nn, 8 * nn, hipMemcpyDeviceToDevice, st) != hipSuccess ||
          hipMemcpyAsync(qt, d.bv + 4 * nn, 8 * nn, hipMemcpyDeviceToDevice, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        rc = MA_EHIP;
    }
  }
  P->opt = saved;
  return rc;
}

int ma_step_bicg(ma_plan* P, int n, const float* h, const float* coef, double tol, int max_iters, double* x,
                 int* iters, void* stream) {
  if (!P || !h || !coef || !x || !(tol > 0.0) || max_iters < 1 || !n_ok(n)) return MA_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const size_t nn = (size_t)n * n;
  const ma_options saved = P->opt;
  P->opt.linear_solver = MA_LINEAR_FD_BICG;
  P->opt.precond = MA_PRECOND_NONE;
  P->opt.gmres_tol = tol;
  P->opt.bicg_max_iters = max_iters;
  PairState s = step_state(nullptr);  // tau = 1, no translation: b = h
  s.mass_c = 0.0;
  Class c;
  int rc = step_prepare(P, n, s, st, c);
  do {
    if (rc) break;
    const PairDesc& d = P->h_desc[0];
    if (hipMemcpyAsync(d.r, h, 4 * nn, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(d.coef, coef, 20 * nn, hipMemcpyDeviceToDevice, st) != hipSuccess) {
      rc = MA_EHIP;
      break;
    }
    launch_bicg(make_ctx(P, c), n, 1, BI_INIT, 0, st);
    if ((rc = launch_bicg_body(P, ClassList{&c, 1}, 1, st))) break;
    if (hipMemcpyAsync(x, d.bv, 8 * nn, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(P->h_state.data(), P->d_state, sizeof(PairState), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      rc = MA_EHIP;
      break;
    }
    if (iters) *iters = P->h_state[0].gm_k;
  } while (0);
  P->opt = saved;
  return rc;
}

int ma_power_inverse(ma_plan* P, int n, const float* coef, const double* abar, const float* b0, int iters,
                     double gmres_tol, int gmres_m, int max_restarts, double* rho, int* gmres_iters, void* stream) {
  if (!P || !coef || !abar || !b0 || !rho || iters < 1 || iters > 100000 || gmres_m < 1 || gmres_m > MA_MMAX ||
      !(gmres_tol > 0.0) || max_restarts < 0 || !n_ok(n))
    return MA_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  double* d_out = nullptr;
  if (hipMalloc(&d_out, sizeof(double) * 2 * (size_t)iters) != hipSuccess) return MA_ENOMEM;
  const ma_options saved = P->opt;
  P->opt.gmres_m = gmres_m;
  P->opt.gmres_max_restarts = max_restarts;
  P->opt.gmres_tol = gmres_tol;
  P->opt.precond = MA_PRECOND_NONE;  // the operator of Section 4.2
  Class c;
  int rc = step_prepare(P, n, step_state(abar), st, c);
  std::vector<double> out(2 * (size_t)iters, 0.0);
  while (rc == MA_OK) {
    const PairDesc& d = P->h_desc[0];
    if (hipMemcpyAsync(d.coef, coef, 20 * (size_t)n * n, hipMemcpyDeviceToDevice, st) != hipSuccess) {
      rc = MA_EHIP;
      break;
    }
    LaunchCtx x = make_ctx(P, c);
    x.precond = MA_PRECOND_NONE;
    std::vector<Class> cls(1, c);
    // b_0 - mean(b_0), normalised; the first GMRES solve starts from it
    launch_power_vec(x, n, PW_SUM_B0, b0, d_out, 0, st);
    launch_power_vec(x, n, PW_CENTER, b0, d_out, 0, st);
    launch_power_vec(x, n, PW_SCALE, b0, d_out, 0, st);
    for (int k = 0; k < iters && rc == MA_OK; ++k) {
      // theta = A^{-1} b_k: GMRES on L Lbar^{-1} sigma = b_k, theta = Lbar^{-1} sigma (Section 4.2)
      launch_passA(x, n, 1, PA_INIT, 0, c.tw, st);
      if ((rc = launch_cycle_body(P, ClassList{cls.data(), 1}, 1, st))) break;
      for (int cyc = 0; cyc < max_restarts; ++cyc) {
        if ((rc = read_summary(P, 1, st))) break;
        if (P->h_summary[6] == 0) break;
        launch_restart(x, n, 1, st);
        launch_passA(x, n, 1, PA_PLAIN, 0, c.tw, st);
        if ((rc = launch_cycle_body(P, ClassList{cls.data(), 1}, 1, st))) break;
      }
      if (rc) break;
      launch_passA(x, n, 1, PA_RECOVER, 0, c.tw, st);
      launch_passB(x, n, 1, PB_RECOVER, 0, c.tw, st);
      launch_passC(x, n, 1, PC_THETA_ONLY, 0, c.tw, st);
      // rho_k = ||theta||, b_{k+1} = theta / rho_k
      launch_power_vec(x, n, PW_THETA, b0, d_out, k, st);
      if (k + 1 < iters) launch_power_vec(x, n, PW_NEXT, b0, d_out, k, st);
    }
    if (rc) break;
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(out.data(), d_out, sizeof(double) * out.size(), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      rc = MA_EHIP;
      break;
    }
    for (int k = 0; k < iters; ++k) {
      rho[k] = out[2 * k];
      if (gmres_iters) gmres_iters[k] = (int)(out[2 * k + 1] - (k > 0 ? out[2 * k - 1] : 0.0));
    }
    break;
  }
  P->opt = saved;
  if (hipStreamSynchronize(st) != hipSuccess) rc = rc ? rc : MA_EHIP;
  (void)hipFree(d_out);
  return rc;
}

int ma_solve_noalloc(const ma_options* opt, const double* f, const double* g, int n, double damping, double tol,
                     const double* psi0, double* psi, double* map, ma_report* rep, void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!opt || !f || !g || !psi || !(damping >= 1.0) || !(tol > 0.0) || validate_options(*opt)) return MA_EINVAL;
  if (!n_ok(n) || n > MA_NOALLOC_NMAX) return MA_EINVAL;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MA_NOALLOC_DEVICES) return MA_EHIP;
  int e = noalloc_setup(dev);
  if (e) return e;
  NoAllocSlot& S = g_noalloc[dev];
  ma_plan* P = &g_noalloc_plan[dev];
  if (pair_bytes(n, opt->gmres_m, uses_bicg(*opt)) > P->arena_bytes) return MA_EINVAL;  // beyond the scratch array
  P->opt = *opt;
  hipStream_t st = (hipStream_t)stream;
  PairDesc& d = P->h_desc[0];
  d = PairDesc{};
  char* p = P->arena;
  carve(d, p, n, P->opt.gmres_m, uses_bicg(P->opt));
  d.cls = 0;
  d.f_in = f;
  d.g_in = g;
  d.psi0_in = psi0;
  d.psi_out = psi;
  d.map_out = map;
  fill_twiddles(S.h_tw, n);
  fill_multipliers(S.h_mt, n, P->opt.symbol);
  HIP_TRY(hipMemcpyAsync(S.d_tw, S.h_tw, sizeof(float2) * n, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(S.d_mt, S.h_mt, sizeof(float2) * n, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(P->d_ids, &S.h_zero, sizeof(int), hipMemcpyHostToDevice, st));
  Class c;
  c.n = n;
  c.count = 1;
  c.d_ids = P->d_ids;
  c.tw = S.d_tw;
  c.mt = S.d_mt;
  e = run_solver(P, 1, damping, tol, st, ClassList{&c, 1});
  if (e) return e;
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  ma_report r;
  fill_report(P->h_state[0], &r, ms);
  if (rep) *rep = r;
  return r.status;
}

}  // extern "C"
