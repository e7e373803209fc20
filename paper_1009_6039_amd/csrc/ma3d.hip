// C ABI and host driver of the three-dimensional solver: its plan and workspace, the
// damped Newton loop (eq. linma) with fixed or halved steps, the GMRES(m) cycles around
// Strain's operator (Section 4.2 in three dimensions), and its single-step entry points.
// The host reads one small device summary per Newton evaluation and per GMRES cycle;
// every field operation runs in the kernels of k3d.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "k3d.h"
#include "ma_ot.h"

namespace {

#define HIP_TRY3(x)                         \
  do {                                      \
    if ((x) != hipSuccess) return MA_EHIP;  \
  } while (0)

size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t part3_doubles(int n) {
  size_t need = (size_t)k3_blocks(n) * MA3_NPART;
  need = std::max(need, (size_t)k3_dot_blocks(n) * (MA3_MMAX + 1));
  return need;
}

size_t pair3_bytes(int n, int m) {
  const size_t nn = (size_t)n * n * n;
  size_t b = al256(8 * nn) * 4;            // u, f, g, theta
  b += al256(16 * nn);                     // gg
  b += al256(36 * nn);                     // coef
  b += al256(4 * nn) * 2;                  // r, x
  b += al256(4 * nn * (size_t)(m + 1));    // V
  b += al256(8 * nn) + al256(24 * nn) + al256(48 * nn);  // S, T, U
  b += al256(8 * part3_doubles(n));        // partials
  b += al256(16 * (size_t)n);              // twiddles and multipliers
  return b;
}

}  // namespace

struct ma3_plan {
  ma_options opt;
  int n_max = 0;
  char* arena = nullptr;
  size_t arena_bytes = 0;
  State3* d_state = nullptr;
  State3* h_state = nullptr;  // pinned host copy
  Desc3 d{};
};

namespace {

void carve3(ma3_plan* P, int n) {
  const size_t nn = (size_t)n * n * n;
  char* p = P->arena;
  auto take = [&](size_t bytes) {
    char* q = p;
    p += al256(bytes);
    return q;
  };
  Desc3& d = P->d;
  d = Desc3{};
  d.n = n;
  d.u = (double*)take(8 * nn);
  d.f = (double*)take(8 * nn);
  d.g = (double*)take(8 * nn);
  d.theta = (double*)take(8 * nn);
  d.gg = (float4*)take(16 * nn);
  d.coef = (float*)take(36 * nn);
  d.r = (float*)take(4 * nn);
  d.x = (float*)take(4 * nn);
  d.V = (float*)take(4 * nn * (size_t)(P->opt.gmres_m + 1));
  d.S = (float2*)take(8 * nn);
  d.T = (float2*)take(24 * nn);
  d.U = (float2*)take(48 * nn);
  d.part = (double*)take(8 * part3_doubles(n));
  float2* tables = (float2*)take(16 * (size_t)n);
  d.tw = tables;
  d.mt = tables + n;
}

// twiddles exp(-2 pi i m / n) and the per-wavenumber multipliers (reading P8; fd4 symbols
// as an option), computed in FP64 and stored in FP32
int upload_tables3(ma3_plan* P, int n, hipStream_t st) {
  std::vector<float2> h(2 * (size_t)n);
  for (int m = 0; m < n; ++m) {
    const double a = -2.0 * M_PI * (double)m / (double)n;
    h[m] = make_float2((float)std::cos(a), (float)std::sin(a));
    const double ks = m < n / 2 ? m : m - n;
    double d1, d2;
    if (P->opt.symbol == MA_SYMBOL_FD4) {
      const double t = 2.0 * M_PI * ks / n;
      d1 = (8.0 * std::sin(t) - std::sin(2.0 * t)) * n / 6.0;
      const double s1 = std::sin(0.5 * t), s2 = std::sin(t);
      d2 = (-64.0 * s1 * s1 + 4.0 * s2 * s2) * (double)n * n / 12.0;
    } else {
      d1 = 2.0 * M_PI * ks;
      d2 = -(2.0 * M_PI * ks) * (2.0 * M_PI * ks);
    }
    if (m == n / 2) d1 = 0.0;
    h[n + m] = make_float2((float)d1, (float)d2);
  }
  HIP_TRY3(hipMemcpyAsync(const_cast<float2*>(P->d.tw), h.data(), sizeof(float2) * 2 * n, hipMemcpyHostToDevice, st));
  return hipStreamSynchronize(st) == hipSuccess ? MA_OK : MA_EHIP;  // h is released on return
}

int prepare3(ma3_plan* P, int n, hipStream_t st) {
  if (!n3_supported(n) || n > P->n_max) return MA_EINVAL;
  const size_t need = pair3_bytes(n, P->opt.gmres_m);
  if (need > P->arena_bytes) {
    if (P->arena) (void)hipFree(P->arena);
    P->arena = nullptr;
    P->arena_bytes = 0;
    if (hipMalloc(&P->arena, need) != hipSuccess) return MA_ENOMEM;
    P->arena_bytes = need;
  }
  carve3(P, n);
  return upload_tables3(P, n, st);
}

int push_state(ma3_plan* P, hipStream_t st) {
  HIP_TRY3(hipMemcpyAsync(P->d_state, P->h_state, sizeof(State3), hipMemcpyHostToDevice, st));
  return MA_OK;
}

int pull_state(ma3_plan* P, hipStream_t st) {
  HIP_TRY3(hipMemcpyAsync(P->h_state, P->d_state, sizeof(State3), hipMemcpyDeviceToHost, st));
  HIP_TRY3(hipStreamSynchronize(st));
  return MA_OK;
}

void fresh_state3(ma3_plan* P) {
  std::memset(P->h_state, 0, sizeof(State3));
  P->h_state->m = P->opt.gmres_m;
  P->h_state->max_restarts = P->opt.gmres_max_restarts;
  P->h_state->gmres_tol = P->opt.gmres_tol;
  P->h_state->tau = 1.0;
}

// what one residual evaluation tells the Newton loop (the oracle's quantities)
struct Eval3 {
  double res, res_max, cst, min_det, w2, mean_u;
  bool finite, convex;
};

Eval3 read_eval(const State3& s, int n) {
  const double* t = s.sums;
  const double NN = (double)n * n * n;
  Eval3 e;
  e.cst = t[0] / NN - 1.0;
  const double ss = t[2] + 2.0 * e.cst * t[1] + NN * e.cst * e.cst;
  e.res = std::sqrt(std::max(ss, 0.0) / NN);
  e.res_max = std::max(std::fabs(t[17] + e.cst), std::fabs(t[18] + e.cst));
  e.min_det = t[14];
  e.w2 = t[12] / NN;
  e.mean_u = t[13] / NN;
  e.finite = t[19] == 0.0 && std::isfinite(e.res);
  e.convex = e.finite && t[15] > 0.0 && t[16] > 0.0 && t[14] > 0.0;
  return e;
}

int evaluate3(ma3_plan* P, hipStream_t st, Eval3& e) {
  k3_residual(P->d, P->d_state, P->opt.op_mode, st);
  const int rc = pull_state(P, st);
  if (rc) return rc;
  e = read_eval(*P->h_state, P->d.n);
  return MA_OK;
}

// theta solving the linearised equation for the right-hand side (r + translation) / tau
// by GMRES(m) on L Lbar^{-1} sigma = h, then u += theta = Lbar^{-1} sigma
int newton_step3(ma3_plan* P, double tau, hipStream_t st) {
  const Desc3& d = P->d;
  P->h_state->tau = tau;
  // (the device copy holds the fold's mass constant and averages: update tau only)
  HIP_TRY3(hipMemcpyAsync(&P->d_state->tau, &P->h_state->tau, sizeof(double), hipMemcpyHostToDevice, st));
  k3_vector(d, P->d_state, V3_INIT, 0, st);
  const int m = P->opt.gmres_m;
  for (int cyc = 0; cyc <= P->opt.gmres_max_restarts; ++cyc) {
    for (int j = 0; j < m; ++j) {
      k3_first_pass(d, P->d_state, P3_MATVEC, j, st);
      k3_forward_rest(d, P->d_state, P3_MATVEC, st);
      k3_inverse(d, P->d_state, P3_MATVEC, j, st);
      k3_vector(d, P->d_state, V3_ARNOLDI, j + 1, st);
    }
    const int rc = pull_state(P, st);
    if (rc) return rc;
    if (!P->h_state->gm_restart) break;
    k3_restart(d, P->d_state, st);
  }
  k3_vector(d, P->d_state, V3_RECOVER, 0, st);
  k3_first_pass(d, P->d_state, P3_THETA, 0, st);
  k3_forward_rest(d, P->d_state, P3_THETA, st);
  k3_inverse(d, P->d_state, P3_THETA, 0, st);
  return hipGetLastError() == hipSuccess ? MA_OK : MA_EHIP;
}

int validate3(const ma_options& o) {
  if (o.max_newton < 0 || o.gmres_m < 1 || o.gmres_m > MA3_MMAX || o.gmres_max_restarts < 0 ||
      !(o.gmres_tol > 0.0) || o.interp != MA_INTERP_BILINEAR || (o.op_mode != MA_OP_FULL && o.op_mode != MA_OP_NO_DRIFT) ||
      (o.damping_policy != MA_DAMP_FIXED && o.damping_policy != MA_DAMP_BACKTRACK) || o.max_backtrack < 0 ||
      (o.symbol != MA_SYMBOL_SPECTRAL && o.symbol != MA_SYMBOL_FD4) || o.precond != MA_PRECOND_NONE ||
      !(o.boundary_frac >= 0.0 && o.boundary_frac < 1.0) || o.forcing != MA_FORCING_FIXED ||
      o.linear_solver != MA_LINEAR_STRAIN_GMRES)
    return MA_EINVAL;
  return MA_OK;
}

}  // namespace

extern "C" {

int ma3_plan_create(int n_max, const ma_options* opt, ma3_plan** out) {
  if (!out) return MA_EINVAL;
  *out = nullptr;
  if (!n3_supported(n_max)) return MA_EINVAL;
  ma3_plan* P = new ma3_plan();
  if (opt) P->opt = *opt;
  else ma_options_default(&P->opt);
  if (validate3(P->opt)) {
    delete P;
    return MA_EINVAL;
  }
  P->n_max = n_max;
  if (hipMalloc(&P->d_state, sizeof(State3)) != hipSuccess ||
      hipHostMalloc(&P->h_state, sizeof(State3), hipHostMallocDefault) != hipSuccess) {
    ma3_plan_destroy(P);
    return MA_ENOMEM;
  }
  *out = P;
  return MA_OK;
}

void ma3_plan_destroy(ma3_plan* P) {
  if (!P) return;
  if (P->arena) (void)hipFree(P->arena);
  if (P->d_state) (void)hipFree(P->d_state);
  if (P->h_state) (void)hipHostFree(P->h_state);
  delete P;
}

int ma3_solve(ma3_plan* P, const double* f, const double* g, int n, double damping, double tol, double* psi,
              double* map, ma_report* rep, void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!P || !f || !g || !psi || !(damping >= 1.0) || !(tol > 0.0)) return MA_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  int rc = prepare3(P, n, st);
  if (rc) return rc;
  Desc3& d = P->d;
  d.f_in = f;
  d.g_in = g;
  fresh_state3(P);
  if ((rc = push_state(P, st))) return rc;
  k3_setup(d, P->d_state, true, st);
  if ((rc = pull_state(P, st))) return rc;
  if (!(P->h_state->sums[0] > 0.0) || P->h_state->sums[1] != 0.0) return MA_EINVAL;  // densities > 0, finite

  Eval3 ev;
  if ((rc = evaluate3(P, st, ev))) return rc;
  const double res0 = ev.res;
  int newton = 0, backtracks = 0, status = MA_ENOCONV;
  double tau = damping;
  while (true) {
    if (!ev.finite) { status = MA_ENAN; break; }
    if (!ev.convex) { status = MA_ENONCONVEX; break; }
    if (ev.res <= tol) { status = MA_OK; break; }
    if (newton >= P->opt.max_newton) { status = MA_ENOCONV; break; }
    if ((rc = newton_step3(P, tau, st))) return rc;  // u += theta
    ++newton;
    Eval3 tr;
    if ((rc = evaluate3(P, st, tr))) return rc;
    if (P->opt.damping_policy == MA_DAMP_FIXED) {
      ev = tr;
      continue;
    }
    // step halving with the boundary rule, as the 2-D solver's
    double step = 1.0;
    bool accepted = false;
    for (int h = 0; h <= P->opt.max_backtrack; ++h) {
      if (tr.convex && tr.res < ev.res && tr.min_det >= P->opt.boundary_frac * ev.min_det) {
        accepted = true;
        break;
      }
      tau *= 2.0;
      ++backtracks;
      if (h == P->opt.max_backtrack) break;
      k3_update(d, -0.5 * step, st);
      step *= 0.5;
      if ((rc = evaluate3(P, st, tr))) return rc;
    }
    if (!accepted) {  // give up: restore the last accepted iterate
      k3_update(d, -step, st);
      if ((rc = evaluate3(P, st, ev))) return rc;
      status = MA_ENOCONV;
      break;
    }
    ev = tr;
    tau = std::max(damping, 0.5 * tau);
  }
  k3_outputs(d, P->d_state, psi, map, st);
  HIP_TRY3(hipStreamSynchronize(st));
  if (rep) {
    std::memset(rep, 0, sizeof(*rep));
    rep->status = status;
    rep->newton_iters = newton;
    rep->gmres_iters = P->h_state->gmres_iters;
    rep->backtracks = backtracks;
    rep->res_rms = ev.res;
    rep->res_max = ev.res_max;
    rep->res0_rms = res0;
    rep->mass_defect = ev.cst;
    rep->min_det = ev.min_det;
    rep->w2sq = ev.w2;
    rep->tau_final = tau;
    rep->time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return status;
}

int ma3_step_residual(ma3_plan* P, int n, const double* u, const double* f, const double* g, float* r, float* coef,
                      double* scalars, void* stream) {
  if (!P || !u || !f || !g || !r || !coef || !scalars) return MA_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  int rc = prepare3(P, n, st);
  if (rc) return rc;
  Desc3& d = P->d;
  d.f_in = f;
  d.g_in = g;
  fresh_state3(P);
  P->h_state->mean_f = P->h_state->mean_g = 1.0;  // f and g used as given
  if ((rc = push_state(P, st))) return rc;
  k3_setup(d, P->d_state, false, st);
  const size_t nn = (size_t)n * n * n;
  HIP_TRY3(hipMemcpyAsync(d.u, u, 8 * nn, hipMemcpyDeviceToDevice, st));
  Eval3 e;
  if ((rc = evaluate3(P, st, e))) return rc;
  HIP_TRY3(hipMemcpyAsync(r, d.r, 4 * nn, hipMemcpyDeviceToDevice, st));
  HIP_TRY3(hipMemcpyAsync(coef, d.coef, 36 * nn, hipMemcpyDeviceToDevice, st));
  HIP_TRY3(hipStreamSynchronize(st));
  const double* t = P->h_state->sums;
  const double out[17] = {e.res, e.res_max, e.cst, t[14], t[15], t[16], t[3], t[4], t[5], t[6], t[7], t[8],
                          t[9], t[10], t[11], e.w2, e.mean_u};
  std::memcpy(scalars, out, sizeof(out));
  return MA_OK;
}

// single operator product w = L Lbar^{-1} v (coefficients and averages given)
int ma3_step_strain_apply(ma3_plan* P, int n, const float* v, const float* coef, const double* abar, float* w,
                          void* stream) {
  if (!P || !v || !coef || !abar || !w) return MA_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  int rc = prepare3(P, n, st);
  if (rc) return rc;
  Desc3& d = P->d;
  const size_t nn = (size_t)n * n * n;
  fresh_state3(P);
  for (int q = 0; q < 9; ++q) P->h_state->abar[q] = abar[q];
  P->h_state->vscale[0] = 1.0;
  P->h_state->gm_running = 1;
  if ((rc = push_state(P, st))) return rc;
  HIP_TRY3(hipMemcpyAsync(d.V, v, 4 * nn, hipMemcpyDeviceToDevice, st));
  HIP_TRY3(hipMemcpyAsync(d.coef, coef, 36 * nn, hipMemcpyDeviceToDevice, st));
  k3_first_pass(d, P->d_state, P3_MATVEC, 0, st);
  k3_forward_rest(d, P->d_state, P3_MATVEC, st);
  k3_inverse(d, P->d_state, P3_MATVEC, 0, st);
  HIP_TRY3(hipGetLastError());
  HIP_TRY3(hipMemcpyAsync(w, d.V + nn, 4 * nn, hipMemcpyDeviceToDevice, st));
  HIP_TRY3(hipStreamSynchronize(st));
  return MA_OK;
}

// theta = Lbar^{-1} sigma (averages given)
int ma3_step_lbar_inverse(ma3_plan* P, int n, const float* sigma, const double* abar, float* theta, void* stream) {
  if (!P || !sigma || !abar || !theta) return MA_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  int rc = prepare3(P, n, st);
  if (rc) return rc;
  Desc3& d = P->d;
  const size_t nn = (size_t)n * n * n;
  fresh_state3(P);
  for (int q = 0; q < 9; ++q) P->h_state->abar[q] = abar[q];
  if ((rc = push_state(P, st))) return rc;
  HIP_TRY3(hipMemcpyAsync(d.x, sigma, 4 * nn, hipMemcpyDeviceToDevice, st));
  k3_first_pass(d, P->d_state, P3_STEP, 0, st);
  k3_forward_rest(d, P->d_state, P3_STEP, st);
  k3_inverse(d, P->d_state, P3_STEP, 0, st);
  HIP_TRY3(hipGetLastError());
  HIP_TRY3(hipMemcpyAsync(theta, d.x, 4 * nn, hipMemcpyDeviceToDevice, st));
  HIP_TRY3(hipStreamSynchronize(st));
  return MA_OK;
}

}  // extern "C"
