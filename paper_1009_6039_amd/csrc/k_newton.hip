// FP64 kernels of the Newton loop: set-up, the fused residual / coefficient
// kernel and its per-pair decision logic, the step-halving update and the outputs.
//
// Section 3.1 (eq. ma2, linearmaeq, linma) and Section 4 (fourth-order differences,
// interpolation of g, eq. translation) of Saumier, Agueh, Khouider.
#include "common.h"
#include "ma_ot.h"
#include "kernels.h"

// ---------------------------------------------------------------------------
// Set-up: means of f, g, psi0 and the validity of the densities.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(MA_BLOCK) void k_setup_sums(LaunchCtx c, int nblk) {
  const int p = pair_of_block(c);
  if (p < 0) return;
  const PairDesc d = c.desc[p];
  const long nn = (long)d.n * d.n;
  double sf = 0, sg = 0, sp = 0, bad = 0;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (long)nblk * blockDim.x) {
    double fv = d.f_in[e], gv = d.g_in[e];
    sf += fv;
    sg += gv;
    if (!(fv > 0.0) || !(gv > 0.0) || !isfinite(fv) || !isfinite(gv)) bad += 1.0;
    if (d.psi0_in) {
      double pv = d.psi0_in[e];
      sp += pv;
      if (!isfinite(pv)) bad += 1.0;
    }
  }
  __shared__ double scratch[(MA_BLOCK / 64) * 4];
  double v[4] = {sf, sg, sp, bad};
  const int kinds[4] = {0, 0, 0, 0};
  block_reduce<4>(v, kinds, scratch);
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) d.part[blockIdx.x * 4 + k] = v[k];
}

__global__ __launch_bounds__(MA_BLOCK) void k_setup_finalize(LaunchCtx c, int nblk) {
  const int p = pair_of_block(c);
  if (p < 0) return;
  const PairDesc d = c.desc[p];
  PairState& s = c.st[p];
  __shared__ double scratch[(MA_BLOCK / 64) * 4];
  const int kinds[4] = {0, 0, 0, 0};
  double t[4];
  fold_partials<4>(d.part, nblk, kinds, t, scratch);
  if (threadIdx.x == 0) {
    const double nn = (double)d.n * d.n;
    s.mean_f = t[0] / nn;
    s.mean_g = t[1] / nn;
    s.mean_psi0 = t[2] / nn;
    s.valid = (t[3] == 0.0) && isfinite(t[0]) && isfinite(t[1]) && isfinite(t[2]);
  }
}

// f and g scaled to mean one (reading P1), the fourth-order grid gradient of g
// (reading P5) and the initial iterate u0 = psi0 - mean(psi0) or 0.
__global__ __launch_bounds__(MA_BLOCK) void k_setup_fields(LaunchCtx c) {
  const int p = pair_of_block(c);
  if (p < 0) return;
  const PairDesc d = c.desc[p];
  const PairState& s = c.st[p];
  const int n = d.n;
  const long nn = (long)n * n;
  const double inv_f = 1.0 / s.mean_f, inv_g = 1.0 / s.mean_g;
  const double inv12h = (double)n / 12.0;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    const int im1 = (i + n - 1) % n, im2 = (i + n - 2) % n, ip1 = (i + 1) % n, ip2 = (i + 2) % n;
    const int jm1 = (j + n - 1) % n, jm2 = (j + n - 2) % n, jp1 = (j + 1) % n, jp2 = (j + 2) % n;
    const double* g = d.g_in;
    double g1 = (g[(long)im2 * n + j] - 8.0 * g[(long)im1 * n + j] + 8.0 * g[(long)ip1 * n + j] -
                 g[(long)ip2 * n + j]) * inv12h * inv_g;
    double g2 = (g[(long)i * n + jm2] - 8.0 * g[(long)i * n + jm1] + 8.0 * g[(long)i * n + jp1] -
                 g[(long)i * n + jp2]) * inv12h * inv_g;
    GS v;
    v.g = g[e] * inv_g;
    v.g1 = (float)g1;
    v.g2 = (float)g2;
    d.gs[e] = v;
    d.f[e] = d.f_in[e] * inv_f;
    if (s.warm) {  // checked start: u0 = 0, the initial potential waits in theta
      d.u[e] = 0.0;
      d.theta[e] = d.psi0_in[e] - s.mean_psi0;
    } else {
      d.u[e] = d.psi0_in ? d.psi0_in[e] - s.mean_psi0 : 0.0;
    }
  }
}

// ---------------------------------------------------------------------------
// Per-pair Newton decisions, run by one thread after a residual evaluation.
// ---------------------------------------------------------------------------
// tot: sum fn, sum r, sum r^2, Simpson sums of a11 a12 a22 b1 b2, sum |grad u|^2 f,
//      sum u, min det, min trace, max r, min r, count of non-finite values
__device__ static void newton_decide(PairState& s, const LaunchCtx& c, int n, const double* tot) {
  const double NN = (double)n * n;
  const double cst = tot[0] / NN - 1.0;  // mean(f_n) - 1: the translation of eq. (translation)
  const double ss = tot[2] + 2.0 * cst * tot[1] + NN * cst * cst;  // sum (r_raw + cst)^2
  const double res = sqrt(fmax(ss, 0.0) / NN);
  const bool finite = tot[14] == 0.0 && isfinite(res);
  const bool convex = finite && tot[10] > 0.0 && tot[11] > 0.0;
  const int ph = s.phase;

  if (ph == PH_REVERT && s.warm_fallback) {
    s.warm_fallback = 0;  // the initial potential never helped: continue Newton from u = 0
  } else if (ph == PH_REVERT) {  // the restored iterate: record it and stop (status already set)
    s.res_rms = res;
    s.res_max = fmax(fabs(tot[12] + cst), fabs(tot[13] + cst));
    s.mass_c = cst;
    s.min_det = tot[10];
    s.w2 = tot[8] / NN;
    s.mean_u = tot[9] / NN;
    s.phase = PH_DONE;
    return;
  }
  const bool trial = (ph == PH_SOLVE || ph == PH_BACKTRACK);
  if (trial && (c.damping_policy == MA_DAMP_BACKTRACK || s.warm_trial)) {
    // a Newton step must also keep min det(I + D^2 u) above a fraction of its value at
    // the current iterate (fraction to the boundary of convexity); the checked start
    // is measured against u = 0 and only needs convexity and a lower residual
    const bool accept = convex && res < s.res_prev && (s.warm_trial || tot[10] >= c.boundary_frac * s.min_det);
    if (!accept) {
      s.bt_step++;
      if (!s.warm_trial) {
        s.backtracks++;
        s.tau *= 2.0;
      }
      if (s.bt_step > c.max_backtrack) {  // give up: restore the last accepted iterate
        s.phase = PH_REVERT;
        s.axpy = -s.step;
        if (s.warm_trial) {
          s.warm_trial = 0;
          s.warm_fallback = 1;
        } else {
          s.status = MA_ENOCONV;
        }
      } else {
        s.phase = PH_BACKTRACK;
        s.axpy = -0.5 * s.step;
        s.step *= 0.5;
      }
      return;
    }
    if (s.warm_trial) {
      s.warm_trial = 0;
      s.warm_steps = 1;
    } else if (c.damping_policy == MA_DAMP_BACKTRACK) {
      s.tau = fmax(s.tau0, 0.5 * s.tau);
      if (c.forcing == MA_FORCING_ADAPTIVE) {
        // a direction (after the first) that needed two or more halvings was solved too
        // loosely for the distance to the solution: the next one 4x tighter; a full step
        // relaxes it 4x again
        const double eta = pair_eta(s, c), eta_min = fmin(c.gmres_tol, 1e-3);
        if (s.bt_step >= 2 && s.newton_iters > 1) s.eta = fmax(0.25 * eta, eta_min);
        else if (s.bt_step == 0) s.eta = fmin(c.gmres_tol, 4.0 * eta);
      }
    }
  }
  // the evaluation is accepted: record it
  s.res_rms = res;
  s.res_max = fmax(fabs(tot[12] + cst), fabs(tot[13] + cst));
  s.mass_c = cst;
  s.min_det = tot[10];
  s.min_tr = tot[11];
  s.w2 = tot[8] / NN;
  s.mean_u = tot[9] / NN;
  for (int k = 0; k < 5; ++k) s.abar[k] = tot[3 + k];
  if (ph == PH_INIT) s.res0 = res;
  if (ph == PH_INIT && s.warm && finite && res > s.tol) {
    // checked start: try the initial potential (stored in theta) as the first step
    s.phase = PH_BACKTRACK;
    s.warm_trial = 1;
    s.axpy = 1.0;
    s.step = 1.0;
    s.bt_step = 0;
    s.res_prev = res;
    return;
  }
  if (!finite) {
    s.status = MA_ENAN;
    s.phase = PH_DONE;
  } else if (!convex) {
    s.status = MA_ENONCONVEX;
    s.phase = PH_DONE;
  } else if (res <= s.tol) {
    s.status = MA_OK;
    s.phase = PH_DONE;
  } else if (s.newton_iters >= c.max_newton) {
    s.status = MA_ENOCONV;
    s.phase = PH_DONE;
  } else {
    // next Newton direction: GMRES on L Lbar^{-1} sigma = r / tau (Section 4.2)
    s.phase = PH_SOLVE;
    s.newton_iters++;
    s.res_prev = res;
    s.bt_step = 0;
    s.step = 1.0;
    s.bnorm = sqrt(fmax(ss, 0.0)) / s.tau;
    s.gm_target = pair_eta(s, c) * s.bnorm;
    s.gm_running = s.bnorm > 0.0;
    s.gm_restart = 0;
    s.gm_cycle = 0;
    s.gm_k = 0;
    s.vscale[0] = s.bnorm > 0.0 ? 1.0 / s.bnorm : 0.0;
    s.gv[0] = s.bnorm;
  }
}

// f mod n for an integer-valued f with |f| < 2^50, in [0, n).  The quotient
// floor(f * (1/N)) differs from floor(f / N) by at most one (1/N is rounded, f * (1/N)
// too), so the FP64 remainder f - N q (exact: integers below 2^53) lies in [-n, 2n)
// and one fold finishes it.  Replaces a division and a 64-bit integer remainder.
__device__ inline int wrap_index(double f, int n, double N, double invN) {
  int a = (int)(f - N * floor(f * invN));
  a += a < 0 ? n : (a >= n ? -n : 0);
  return a;
}

// ---------------------------------------------------------------------------
// Fused residual + coefficient kernel (one Newton evaluation).
// ---------------------------------------------------------------------------
// The part after the derivatives, for one grid point (i, j): g and grad g at
// y = x + grad u (Section 4, periodic), det(I + D^2 u), f_n, r = f - f_n, the
// coefficients of eq. (linearmaeq) (stored FP32), and this point's share of the
// block's partial sums (acc, layout as k_residual_finalize reads it).
struct ResidualViews {
  MA_GLOBAL_AS const GS* gs;
  MA_GLOBAL_AS const double* F;
  MA_GLOBAL_AS float* R;
  MA_GLOBAL_AS float* coef;
};

__device__ __forceinline__ void residual_acc_init(double (&acc)[MA_NPART_RES]) {
  for (int k = 0; k < 10; ++k) acc[k] = 0.0;
  acc[10] = 1e300;   // min det
  acc[11] = 1e300;   // min trace
  acc[12] = -1e300;  // max r
  acc[13] = 1e300;   // min r
  acc[14] = 0.0;     // non-finite count
  acc[15] = 0.0;
}

template <int INTERP>
__device__ __forceinline__ void residual_point(const LaunchCtx& c, const ResidualViews& v, int n, int i, int j,
                                               double uc, double u1, double u2, double u11, double u22,
                                               double u12, double fv, double (&acc)[MA_NPART_RES]) {
  const double N = (double)n, invN = 1.0 / N;
  const int nn = n * n;  // n * n < 2^31
  // a diverging iterate must not produce a wild gather index (it is flagged below)
  double t1 = (double)i + N * u1, t2 = (double)j + N * u2;
  if (!(fabs(t1) < 1e15)) t1 = 0.0;
  if (!(fabs(t2) < 1e15)) t2 = 0.0;
  double gy, gy1, gy2;
  if constexpr (INTERP == MA_INTERP_NEAREST) {
    const int a = wrap_index(floor(t1 + 0.5), n, N, invN), b = wrap_index(floor(t2 + 0.5), n, N, invN);
    GS w = v.gs[a * n + b];
    gy = w.g; gy1 = w.g1; gy2 = w.g2;
  } else {
    const double f1 = floor(t1), f2 = floor(t2);
    const double wa = t1 - f1, wb = t2 - f2;
    const int a = wrap_index(f1, n, N, invN), b = wrap_index(f2, n, N, invN);
    const int a1 = (a + 1 == n) ? 0 : a + 1, b1 = (b + 1 == n) ? 0 : b + 1;
    const GS v00 = v.gs[a * n + b], v10 = v.gs[a1 * n + b], v01 = v.gs[a * n + b1], v11 = v.gs[a1 * n + b1];
    const double w00 = (1 - wa) * (1 - wb), w10 = wa * (1 - wb), w01 = (1 - wa) * wb, w11 = wa * wb;
    gy = w00 * v00.g + w10 * v10.g + w01 * v01.g + w11 * v11.g;
    gy1 = w00 * v00.g1 + w10 * v10.g1 + w01 * v01.g1 + w11 * v11.g1;
    gy2 = w00 * v00.g2 + w10 * v10.g2 + w01 * v01.g2 + w11 * v11.g2;
  }
  const double det = (1.0 + u11) * (1.0 + u22) - u12 * u12;
  const double fn = gy * det;
  const int e = i * n + j;
  const double rr = fv - fn;
  const double a11 = gy * (1.0 + u22), a22 = gy * (1.0 + u11), a12 = -gy * u12;
  const double b1 = c.op_mode == MA_OP_NO_DRIFT ? 0.0 : det * gy1;
  const double b2 = c.op_mode == MA_OP_NO_DRIFT ? 0.0 : det * gy2;
  v.R[e] = (float)rr;
  v.coef[e] = (float)a11;
  v.coef[nn + e] = (float)a12;
  v.coef[2 * nn + e] = (float)a22;
  v.coef[3 * nn + e] = (float)b1;
  v.coef[4 * nn + e] = (float)b2;
  // periodic Simpson weights (reading P7): 2h/3 at even nodes, 4h/3 at odd ones
  const double w = (double)((i & 1) ? 4 : 2) * (double)((j & 1) ? 4 : 2) * (1.0 / (9.0 * N * N));
  acc[0] += fn;
  acc[1] += rr;
  acc[2] += rr * rr;
  acc[3] += w * a11;
  acc[4] += w * a12;
  acc[5] += w * a22;
  acc[6] += w * b1;
  acc[7] += w * b2;
  acc[8] += (u1 * u1 + u2 * u2) * fv;
  acc[9] += uc;
  acc[10] = fmin(acc[10], det);
  acc[11] = fmin(acc[11], 2.0 + u11 + u22);
  acc[12] = fmax(acc[12], rr);
  acc[13] = fmin(acc[13], rr);
  if (!isfinite(rr) || !isfinite(det)) acc[14] += 1.0;
}

constexpr int RES_KINDS[MA_NPART_RES] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 2, 1, 0, 0};

// Tile: TX columns x MA_RES_TY rows per block, halo 2 staged in LDS (FP64).
template <int TX, int INTERP>
__global__ __launch_bounds__(MA_BLOCK) void k_residual(LaunchCtx c) {
  const int p = pair_of_block(c);
  if (p < 0) return;
  const PairDesc d = c.desc[p];
  PairState& s = c.st[p];
  if (s.phase == PH_DONE) return;
  count_bytes(c, 56.0, d.n);  // u 8, f 8, g with gradient 16 (once), r 4, coefficients 20
  constexpr int TY = MA_RES_TY;
  constexpr int LW = TX + 4;
  __shared__ double tile[(TY + 4) * LW];
  __shared__ double scratch[(MA_BLOCK / 64) * MA_NPART_RES];
  const int n = d.n;
  const int nbx = n / TX;
  const int i0 = (blockIdx.x / nbx) * TY, j0 = (blockIdx.x % nbx) * TX;
  const auto u = gmem<const double>(d.u);
  for (int e = threadIdx.x; e < (TY + 4) * LW; e += MA_BLOCK) {
    const int li = e / LW, lj = e % LW;
    int gi = i0 + li - 2, gj = j0 + lj - 2;  // within [-2, n + 2): one periodic fold
    gi += gi < 0 ? n : (gi >= n ? -n : 0);
    gj += gj < 0 ? n : (gj >= n ? -n : 0);
    tile[e] = u[(long)gi * n + gj];
  }
  __syncthreads();

  const double N = (double)n;
  const double i12h = N / 12.0, i12h2 = N * N / 12.0, i144h2 = N * N / 144.0;
  double acc[MA_NPART_RES];
  residual_acc_init(acc);
  const ResidualViews views{gmem<const GS>(d.gs), gmem<const double>(d.f), gmem<float>(d.r), gmem<float>(d.coef)};
  constexpr int TROWS = MA_BLOCK / TX;
  const int tx = threadIdx.x % TX, ty0 = threadIdx.x / TX;
  for (int ty = ty0; ty < TY; ty += TROWS) {
    const int li = ty + 2, lj = tx + 2;
#define U(a, b) tile[(li + (a)) * LW + lj + (b)]
    const double u1 = (U(-2, 0) - 8.0 * U(-1, 0) + 8.0 * U(1, 0) - U(2, 0)) * i12h;
    const double u2 = (U(0, -2) - 8.0 * U(0, -1) + 8.0 * U(0, 1) - U(0, 2)) * i12h;
    const double u11 = (-U(-2, 0) + 16.0 * U(-1, 0) - 30.0 * U(0, 0) + 16.0 * U(1, 0) - U(2, 0)) * i12h2;
    const double u22 = (-U(0, -2) + 16.0 * U(0, -1) - 30.0 * U(0, 0) + 16.0 * U(0, 1) - U(0, 2)) * i12h2;
    double q[5];
#pragma unroll
    for (int a = -2; a <= 2; ++a)
      q[a + 2] = (a == 0) ? 0.0 : (U(a, -2) - 8.0 * U(a, -1) + 8.0 * U(a, 1) - U(a, 2));
    const double u12 = (q[0] - 8.0 * q[1] + 8.0 * q[3] - q[4]) * i144h2;
    residual_point<INTERP>(c, views, n, i0 + ty, j0 + tx, U(0, 0), u1, u2, u11, u22, u12,
                           views.F[(i0 + ty) * n + j0 + tx], acc);
#undef U
  }
  block_reduce<MA_NPART_RES>(acc, RES_KINDS, scratch);
  if (threadIdx.x == 0)
    for (int k = 0; k < MA_NPART_RES; ++k) d.part[(long)blockIdx.x * MA_NPART_RES + k] = acc[k];
}


// Streaming variant: a wave takes 64 consecutive columns j0 .. j0+63 and walks down
// RPW rows.  The five rows of u around the current row sit in registers (a sliding
// window, the x1 stencils), the x2 stencils take the neighbouring columns from the
// neighbouring lanes (cross-lane reads; the wave's edge lanes take columns j0-2,
// j0-1, j0+64, j0+65, which lanes 0..3 load besides their own), and the next row of
// u is loaded before the current one is evaluated.  No LDS tile, no barrier before
// the block's final reduction; the arithmetic of each point is that of k_residual.
// Needs n % 64 == 0; a block of MA_RES_STREAM_BLOCK threads covers 64 columns and
// (MA_RES_STREAM_BLOCK / 64) * RPW rows.
template <int RPW, int INTERP>
__global__ __launch_bounds__(MA_RES_STREAM_BLOCK) void k_residual_stream(LaunchCtx c) {
  const int p = pair_of_block(c);
  if (p < 0) return;
  const PairDesc d = c.desc[p];
  PairState& s = c.st[p];
  if (s.phase == PH_DONE) return;
  count_bytes(c, 56.0, d.n);
  constexpr int WPB = MA_RES_STREAM_BLOCK / 64;
  __shared__ double scratch[WPB * MA_NPART_RES];
  const int n = d.n;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nbx = n / 64;
  const int j0 = (blockIdx.x % nbx) * 64;
  const int i0 = (blockIdx.x / nbx) * (WPB * RPW) + wv * RPW;
  const int j = j0 + lane;
  int jh = lane < 2 ? j0 - 2 + lane : j0 + 62 + lane;  // lanes 0..3: j0-2, j0-1, j0+64, j0+65
  jh += jh < 0 ? n : (jh >= n ? -n : 0);
  if (lane >= 4) jh = j;  // read but unused
  const auto u = gmem<const double>(d.u);
  auto row = [&](int i) {  // offset of row i (within [-2, n + 3)), periodic
    i += i < 0 ? n : (i >= n ? -n : 0);
    return i * n;  // n * n < 2^31
  };
  const double N = (double)n;
  const double i12h = N / 12.0, i12h2 = N * N / 12.0, i144h2 = N * N / 144.0;
  // x2 stencils of one row: q = the first-difference combination (unscaled), d2 the
  // second derivative
  auto across = [&](double v, double hv, double& q, double& d2) {
    const double h0 = read_lane(hv, 0), h1 = read_lane(hv, 1), h2 = read_lane(hv, 2), h3 = read_lane(hv, 3);
    // neighbours by DPP wave shifts (lanes 0, 1, 62, 63 take the halo values below)
    double vm1 = dpp_move<0x138>(v), vp1 = dpp_move<0x130>(v);
    double vm2 = dpp_move<0x138>(vm1), vp2 = dpp_move<0x130>(vp1);
    vm1 = lane >= 1 ? vm1 : h1;
    vm2 = lane >= 2 ? vm2 : (lane == 1 ? h1 : h0);
    vp1 = lane <= 62 ? vp1 : h2;
    vp2 = lane <= 61 ? vp2 : (lane == 62 ? h2 : h3);
    q = vm2 - 8.0 * vm1 + 8.0 * vp1 - vp2;
    d2 = (-vm2 + 16.0 * vm1 - 30.0 * v + 16.0 * vp1 - vp2) * i12h2;
  };
  // window: rows i-2 .. i+2 of u and q; d2 of rows i .. i+2
  double wu[5], wq[5], wd[3];
  {
    double v[5], hv[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const int o = row(i0 - 2 + k);
      v[k] = u[o + j];
      hv[k] = u[o + jh];
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      double dd;
      wu[k] = v[k];
      across(v[k], hv[k], wq[k], dd);
      if (k >= 2) wd[k - 2] = dd;
    }
  }
  double acc[MA_NPART_RES];
  residual_acc_init(acc);
  const ResidualViews views{gmem<const GS>(d.gs), gmem<const double>(d.f), gmem<float>(d.r), gmem<float>(d.coef)};
#pragma unroll 1
  for (int k = 0; k < RPW; ++k) {
    const int i = i0 + k;
    const double fv = views.F[i * n + j];  // issued with the next row's u, before the gathers
    double nv = 0.0, nhv = 0.0;
    if (k + 1 < RPW) {  // row i + 3, for the next window
      const int o = row(i + 3);
      nv = u[o + j];
      nhv = u[o + jh];
    }
    const double u1 = (wu[0] - 8.0 * wu[1] + 8.0 * wu[3] - wu[4]) * i12h;
    const double u2 = wq[2] * i12h;
    const double u11 = (-wu[0] + 16.0 * wu[1] - 30.0 * wu[2] + 16.0 * wu[3] - wu[4]) * i12h2;
    const double u22 = wd[0];
    const double u12 = (wq[0] - 8.0 * wq[1] + 8.0 * wq[3] - wq[4]) * i144h2;
    residual_point<INTERP>(c, views, n, i, j, wu[2], u1, u2, u11, u22, u12, fv, acc);
    if (k + 1 < RPW) {
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        wu[m] = wu[m + 1];
        wq[m] = wq[m + 1];
      }
      wd[0] = wd[1];
      wd[1] = wd[2];
      wu[4] = nv;
      across(nv, nhv, wq[4], wd[2]);
    }
  }
  block_reduce<MA_NPART_RES>(acc, RES_KINDS, scratch);
  if (threadIdx.x == 0)
    for (int k = 0; k < MA_NPART_RES; ++k) d.part[(long)blockIdx.x * MA_NPART_RES + k] = acc[k];
}

// folds the residual partials of one pair and runs its Newton decisions
__global__ __launch_bounds__(MA_BLOCK) void k_residual_finalize(LaunchCtx c, int nblk, int step_mode) {
  const int p = pair_of_block(c);
  if (p < 0) return;
  const PairDesc d = c.desc[p];
  PairState& s = c.st[p];
  if (s.phase == PH_DONE) return;
  __shared__ double scratch[(MA_BLOCK / 64) * MA_NPART_RES];
  double t[MA_NPART_RES];
  fold_partials<MA_NPART_RES>(d.part, nblk, RES_KINDS, t, scratch);
  if (threadIdx.x != 0) return;
  const int n = d.n;
  if (step_mode) {  // single-step use: record the evaluation only
    const double NN = (double)n * n;
    const double cst = t[0] / NN - 1.0;
    const double ss = t[2] + 2.0 * cst * t[1] + NN * cst * cst;
    s.res_rms = sqrt(fmax(ss, 0.0) / NN);
    s.res_max = fmax(fabs(t[12] + cst), fabs(t[13] + cst));
    s.mass_c = cst;
    s.min_det = t[10];
    s.min_tr = t[11];
    s.w2 = t[8] / NN;
    s.mean_u = t[9] / NN;
    for (int k = 0; k < 5; ++k) s.abar[k] = t[3 + k];
  } else {
    newton_decide(s, c, n, t);
  }
}

// r + translation constant, as FP32, for the single-step entry point
__global__ __launch_bounds__(MA_BLOCK) void k_residual_shift(LaunchCtx c, float* out) {
  const int p = pair_of_block(c);
  if (p < 0) return;
  const PairDesc d = c.desc[p];
  const float cst = (float)c.st[p].mass_c;
  const long nn = (long)d.n * d.n;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (long)gridDim.x * blockDim.x)
    out[e] = d.r[e] + cst;
}

// u += axpy * theta for pairs halving a rejected step or restoring the last iterate
__global__ __launch_bounds__(MA_BLOCK) void k_step_update(LaunchCtx c) {
  const int p = pair_of_block(c);
  if (p < 0) return;
  const PairDesc d = c.desc[p];
  const PairState& s = c.st[p];
  if (s.phase != PH_BACKTRACK && s.phase != PH_REVERT) return;
  const double a = s.axpy;
  const long nn = (long)d.n * d.n;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (long)gridDim.x * blockDim.x)
    d.u[e] += a * d.theta[e];
}

// psi = u - mean(u); map = x + D_h u (fourth-order differences), unwrapped
__global__ __launch_bounds__(MA_BLOCK) void k_outputs(LaunchCtx c) {
  const int p = pair_of_block(c);
  if (p < 0) return;
  const PairDesc d = c.desc[p];
  const PairState& s = c.st[p];
  const int n = d.n;
  const long nn = (long)n * n;
  const double mu = s.mean_u, i12h = (double)n / 12.0, h = 1.0 / (double)n;
  const double* u = d.u;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    d.psi_out[e] = u[e] - mu;
    if (d.map_out) {
      const int im1 = (i + n - 1) % n, im2 = (i + n - 2) % n, ip1 = (i + 1) % n, ip2 = (i + 2) % n;
      const int jm1 = (j + n - 1) % n, jm2 = (j + n - 2) % n, jp1 = (j + 1) % n, jp2 = (j + 2) % n;
      const double u1 = (u[(long)im2 * n + j] - 8.0 * u[(long)im1 * n + j] + 8.0 * u[(long)ip1 * n + j] -
                         u[(long)ip2 * n + j]) * i12h;
      const double u2 = (u[(long)i * n + jm2] - 8.0 * u[(long)i * n + jm1] + 8.0 * u[(long)i * n + jp1] -
                         u[(long)i * n + jp2]) * i12h;
      d.map_out[e] = (double)i * h + u1;
      d.map_out[nn + e] = (double)j * h + u2;
    }
  }
}

// Counts of the pairs per phase and flag, written to host-visible memory: [0..5] pairs
// per phase, [6] pairs to restart GMRES, [7] invalid inputs, [8] pairs inside a GMRES
// cycle; with `phases`, each slot's phase as well.  The sequence number goes last,
// after a system-scope fence, so that a host that sees it also sees the rest.
__global__ __launch_bounds__(256) void k_summary(const PairState* st, const int* ids, int npairs, int* out,
                                                 int seq, int* phases) {
  __shared__ int cnt[MA_SUMMARY_INTS];
  if (threadIdx.x < MA_SUMMARY_INTS) cnt[threadIdx.x] = 0;
  __syncthreads();
  for (int q = threadIdx.x; q < npairs; q += blockDim.x) {
    const PairState& s = st[ids[q]];
    atomicAdd(&cnt[s.phase], 1);  // phases are 0..5
    if (s.phase == PH_SOLVE && s.gm_restart) atomicAdd(&cnt[6], 1);
    if (!s.valid) atomicAdd(&cnt[7], 1);
    if (s.phase == PH_SOLVE && s.gm_running) atomicAdd(&cnt[8], 1);
    if (phases) phases[q] = s.phase;
  }
  if (phases) __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 0; k < MA_SUMMARY_TAG; ++k) out[k] = cnt[k];
    __threadfence_system();
    out[MA_SUMMARY_TAG] = seq;
  }
}

// Compaction of the launch lists (one block per size class): the class's pairs whose
// phase is not done (for the residual and the step updates) and those solving (for the
// GMRES launches), in the class's order, and their numbers.  cls[k] = (offset of the
// class's slice in ids, count); lists and counts are written at the same offsets, the
// counts at cnt[2k] (live) and cnt[2k + 1] (solving).
__global__ __launch_bounds__(256) void k_compact(const PairState* st, const int* ids, const int2* cls, int* live,
                                                 int* solving, int* cnt) {
  const int2 cl = cls[blockIdx.x];
  __shared__ int sl[256], ss[256];
  __shared__ int base_l, base_s;
  if (threadIdx.x == 0) base_l = base_s = 0;
  __syncthreads();
  for (int b = 0; b < cl.y; b += 256) {
    const int q = b + threadIdx.x;
    int id = 0, fl = 0, fs = 0;
    if (q < cl.y) {
      id = ids[cl.x + q];
      const int ph = st[id].phase;
      fl = ph != PH_DONE;
      fs = ph == PH_SOLVE;
    }
    sl[threadIdx.x] = fl;
    ss[threadIdx.x] = fs;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {  // inclusive scans
      const int al = threadIdx.x >= o ? sl[threadIdx.x - o] : 0;
      const int as = threadIdx.x >= o ? ss[threadIdx.x - o] : 0;
      __syncthreads();
      sl[threadIdx.x] += al;
      ss[threadIdx.x] += as;
      __syncthreads();
    }
    if (fl) live[cl.x + base_l + sl[threadIdx.x] - 1] = id;
    if (fs) solving[cl.x + base_s + ss[threadIdx.x] - 1] = id;
    __syncthreads();
    if (threadIdx.x == 255) {
      base_l += sl[255];
      base_s += ss[255];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    cnt[2 * blockIdx.x] = base_l;
    cnt[2 * blockIdx.x + 1] = base_s;
  }
}

// The pairs of one class's launch list (its first *in_n entries, or count where in_n is
// null) that are inside a GMRES cycle, in list order, and their number: the launch
// list of the cycle's later iterations once pairs have left it.
__global__ __launch_bounds__(256) void k_compact_running(const PairState* st, const int* in, const int* in_n,
                                                         int count, int* out, int* out_n) {
  const int n = in_n ? min(*in_n, count) : count;
  __shared__ int sr[256];
  __shared__ int base;
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  for (int b = 0; b < n; b += 256) {
    const int q = b + threadIdx.x;
    int id = 0, f = 0;
    if (q < n) {
      id = in[q];
      f = st[id].phase == PH_SOLVE && st[id].gm_running;
    }
    sr[threadIdx.x] = f;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {  // inclusive scan
      const int a = threadIdx.x >= o ? sr[threadIdx.x - o] : 0;
      __syncthreads();
      sr[threadIdx.x] += a;
      __syncthreads();
    }
    if (f) out[base + sr[threadIdx.x] - 1] = id;
    __syncthreads();
    if (threadIdx.x == 255) base += sr[255];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out_n = base;
}

// Continuous batching.  k_retire: for the slots in the launch's id list (pairs that
// finished), the outputs of k_outputs and the final state into final[pair].
__global__ __launch_bounds__(MA_BLOCK) void k_retire(LaunchCtx c, PairState* final_state) {
  const int p = pair_of_block(c);
  if (p < 0) return;
  const PairDesc d = c.desc[p];
  const PairState& s = c.st[p];
  const int n = d.n;
  const long nn = (long)n * n;
  const double mu = s.mean_u, i12h = (double)n / 12.0, h = 1.0 / (double)n;
  const double* u = d.u;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    d.psi_out[e] = u[e] - mu;
    if (d.map_out) {
      const int im1 = (i + n - 1) % n, im2 = (i + n - 2) % n, ip1 = (i + 1) % n, ip2 = (i + 2) % n;
      const int jm1 = (j + n - 1) % n, jm2 = (j + n - 2) % n, jp1 = (j + 1) % n, jp2 = (j + 2) % n;
      const double u1 = (u[(long)im2 * n + j] - 8.0 * u[(long)im1 * n + j] + 8.0 * u[(long)ip1 * n + j] -
                         u[(long)ip2 * n + j]) * i12h;
      const double u2 = (u[(long)i * n + jm2] - 8.0 * u[(long)i * n + jm1] + 8.0 * u[(long)i * n + jp1] -
                         u[(long)i * n + jp2]) * i12h;
      d.map_out[e] = (double)i * h + u1;
      d.map_out[nn + e] = (double)j * h + u2;
    }
  }
  if (blockIdx.x == 0) {  // the state, copied word by word by the block
    const int* src = reinterpret_cast<const int*>(&s);
    int* dst = reinterpret_cast<int*>(&final_state[d.pair]);
    for (int w = threadIdx.x; w < (int)(sizeof(PairState) / sizeof(int)); w += blockDim.x) dst[w] = src[w];
  }
}

// k_refill: record r's descriptor and fresh state into its slot
__global__ __launch_bounds__(256) void k_refill(PairDesc* desc, PairState* st, const RefillRecord* rec) {
  const RefillRecord& r = rec[blockIdx.x];
  {
    const int* src = reinterpret_cast<const int*>(&r.desc);
    int* dst = reinterpret_cast<int*>(&desc[r.slot]);
    for (int w = threadIdx.x; w < (int)(sizeof(PairDesc) / sizeof(int)); w += blockDim.x) dst[w] = src[w];
  }
  const int* src = reinterpret_cast<const int*>(&r.state);
  int* dst = reinterpret_cast<int*>(&st[r.slot]);
  for (int w = threadIdx.x; w < (int)(sizeof(PairState) / sizeof(int)); w += blockDim.x) dst[w] = src[w];
}

// k_validate: counts the pairs whose densities are not finite and positive (or whose
// initial potential is not finite) before any of them is solved; one block row per pair
__global__ __launch_bounds__(MA_BLOCK) void k_validate(const double* const* f, const double* const* g,
                                                       const double* const* psi0, const int* n, int* bad) {
  const int q = blockIdx.y;
  const long nn = (long)n[q] * n[q];
  const double* fq = f[q];
  const double* gq = g[q];
  const double* pq = psi0 ? psi0[q] : nullptr;
  int b = 0;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (long)gridDim.x * blockDim.x) {
    const double fv = fq[e], gv = gq[e];
    if (!(fv > 0.0) || !(gv > 0.0) || !isfinite(fv) || !isfinite(gv)) b = 1;
    if (pq && !isfinite(pq[e])) b = 1;
  }
  if (__syncthreads_or(b) && threadIdx.x == 0) atomicAdd(bad, 1);
}

// Synthetic fields for timing launch geometries: smooth positive densities, a small
// potential, coefficients near those of the Laplacian and pseudo-random Krylov
// vectors (a 32-bit integer hash of the pair, vector and point index).
__global__ __launch_bounds__(MA_BLOCK) void k_tune_fill(LaunchCtx c) {
  const int p = pair_of_block(c);
  if (p < 0) return;
  const PairDesc d = c.desc[p];
  const int n = d.n;
  const long nn = (long)n * n;
  const double tp = 6.283185307179586;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (long)gridDim.x * blockDim.x) {
    const double x1 = (double)(e / n) / n, x2 = (double)(e % n) / n;
    d.u[e] = 0.002 * sin(tp * x1) * sin(tp * x2);
    d.f[e] = 1.0 + 0.3 * cos(tp * (x1 + 2.0 * x2));
    const double ph = tp * (2.0 * x1 - x2);
    GS gs;
    gs.g = 1.0 + 0.2 * sin(ph);
    gs.g1 = (float)(0.4 * tp * cos(ph));
    gs.g2 = (float)(-0.2 * tp * cos(ph));
    d.gs[e] = gs;
    d.coef[e] = (float)(1.0 + 0.2 * sin(tp * x1));
    d.coef[nn + e] = (float)(0.1 * cos(tp * x2));
    d.coef[2 * nn + e] = (float)(1.0 + 0.2 * cos(tp * (x1 + x2)));
    d.coef[3 * nn + e] = (float)(0.05 * sin(tp * x2));
    d.coef[4 * nn + e] = (float)(0.05 * cos(tp * x1));
    d.r[e] = 0.f;
    d.x[e] = 0.f;
    for (int l = 0; l <= c.m; ++l) {
      unsigned h = (unsigned)e * 2654435761u ^ (unsigned)(l * 40503 + p * 977 + 17);
      h ^= h >> 15;
      h *= 2246822519u;
      h ^= h >> 13;
      d.V[(long)l * nn + e] = (float)((double)(h & 0xFFFFFF) / 8388608.0 - 1.0);
    }
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
void launch_tune_fill(const LaunchCtx& c, int n, int npairs, hipStream_t st) {
  long b = (long)n * n / (MA_BLOCK * 4);
  const int nb = b < 1 ? 1 : (int)(b > 4096 ? 4096 : b);
  hipLaunchKernelGGL(k_tune_fill, dim3(nb, npairs), dim3(MA_BLOCK), 0, st, c);
}
void launch_setup_fields(const LaunchCtx& c, int n, int npairs, hipStream_t st) {
  int nb2 = (int)((long)n * n / (MA_BLOCK * 4));
  nb2 = nb2 < 1 ? 1 : (nb2 > 4096 ? 4096 : nb2);
  hipLaunchKernelGGL(k_setup_fields, dim3(nb2, npairs), dim3(MA_BLOCK), 0, st, c);
}

void launch_setup(const LaunchCtx& c, int n, int npairs, hipStream_t st) {
  int nblk = (int)((long)n * n / 4096);
  nblk = nblk < 1 ? 1 : (nblk > 256 ? 256 : nblk);
  hipLaunchKernelGGL(k_setup_sums, dim3(nblk, npairs), dim3(MA_BLOCK), 0, st, c, nblk);
  hipLaunchKernelGGL(k_setup_finalize, dim3(1, npairs), dim3(MA_BLOCK), 0, st, c, nblk);
  launch_setup_fields(c, n, npairs, st);
}

// tile width of the residual stencil: variant 0 the widest that divides n (64, 32 or
// 16 columns), 1 half of it, 2 a quarter (never below 16), 3 the streaming kernel
// (64 columns per wave, MA_RES_STREAM_ROWS rows per wave) where n % 64 == 0, else the
// same as 0
int residual_tile_x(int n, int v) {
  if (v >= 4) v = 0;
  const int t0 = (n % 64 == 0) ? 64 : ((n % 32 == 0) ? 32 : 16);
  const int t = v == 1 ? t0 / 2 : (v == 2 ? t0 / 4 : t0);
  return t < 16 ? 16 : t;
}

bool residual_streams(int n, int v) { return v == 3 && n % 64 == 0; }

int residual_geometry(int n, int v, int* tile_x, int* threads) {
  if (v < 0 || v >= MA_NVARIANTS || n % 16) return -1;
  if (v >= 4) return residual_geometry(n, 0, tile_x, threads) < 0 ? -1 : 0;  // no wave-owned residual
  *tile_x = residual_tile_x(n, v);
  *threads = residual_streams(n, v) ? MA_RES_STREAM_BLOCK : MA_BLOCK;
  if (residual_streams(n, v)) return v;
  for (int u = 0; u < v; ++u)
    if (residual_tile_x(n, u) == *tile_x) return u;
  return v;
}

int residual_blocks(int n, int v) {
  if (residual_streams(n, v)) return (n / 64) * (n / (MA_RES_STREAM_BLOCK / 64 * MA_RES_STREAM_ROWS));
  return (n / residual_tile_x(n, v)) * (n / MA_RES_TY);
}

void launch_residual_only(const LaunchCtx& c, int n, int npairs, hipStream_t st, const TimedLaunch& ev) {
  dim3 grid(residual_blocks(n, c.var[3]), npairs);
  const bool nearest = c.interp == MA_INTERP_NEAREST;
  if (residual_streams(n, c.var[3])) {
    if (nearest)
      MA_LAUNCH(ev, (k_residual_stream<MA_RES_STREAM_ROWS, MA_INTERP_NEAREST>), grid, dim3(MA_RES_STREAM_BLOCK), st, c);
    else
      MA_LAUNCH(ev, (k_residual_stream<MA_RES_STREAM_ROWS, MA_INTERP_BILINEAR>), grid, dim3(MA_RES_STREAM_BLOCK), st,
                c);
    return;
  }
  const int tx = residual_tile_x(n, c.var[3]);
  if (nearest) {
    if (tx == 64) MA_LAUNCH(ev, (k_residual<64, MA_INTERP_NEAREST>), grid, dim3(MA_BLOCK), st, c);
    else if (tx == 32) MA_LAUNCH(ev, (k_residual<32, MA_INTERP_NEAREST>), grid, dim3(MA_BLOCK), st, c);
    else MA_LAUNCH(ev, (k_residual<16, MA_INTERP_NEAREST>), grid, dim3(MA_BLOCK), st, c);
  } else {
    if (tx == 64) MA_LAUNCH(ev, (k_residual<64, MA_INTERP_BILINEAR>), grid, dim3(MA_BLOCK), st, c);
    else if (tx == 32) MA_LAUNCH(ev, (k_residual<32, MA_INTERP_BILINEAR>), grid, dim3(MA_BLOCK), st, c);
    else MA_LAUNCH(ev, (k_residual<16, MA_INTERP_BILINEAR>), grid, dim3(MA_BLOCK), st, c);
  }
}

void launch_residual(const LaunchCtx& c, int n, int npairs, int step_mode, hipStream_t st, const TimedLaunch& ev) {
  launch_residual_only(c, n, npairs, st, ev);
  hipLaunchKernelGGL(k_residual_finalize, dim3(1, npairs), dim3(MA_BLOCK), 0, st, c, residual_blocks(n, c.var[3]),
                     step_mode);
}

static int elementwise_blocks(int n) {
  long b = (long)n * n / (MA_BLOCK * 4);
  return b < 1 ? 1 : (int)(b > 4096 ? 4096 : b);
}

void launch_residual_shift(const LaunchCtx& c, int n, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_residual_shift, dim3(elementwise_blocks(n), 1), dim3(MA_BLOCK), 0, st, c, out);
}

void launch_step_update(const LaunchCtx& c, int n, int npairs, hipStream_t st) {
  hipLaunchKernelGGL(k_step_update, dim3(elementwise_blocks(n), npairs), dim3(MA_BLOCK), 0, st, c);
}

void launch_outputs(const LaunchCtx& c, int n, int npairs, hipStream_t st) {
  hipLaunchKernelGGL(k_outputs, dim3(elementwise_blocks(n), npairs), dim3(MA_BLOCK), 0, st, c);
}

void launch_summary(const PairState* s, const int* ids, int npairs, int* out, int seq, hipStream_t st,
                    int* phases) {
  hipLaunchKernelGGL(k_summary, dim3(1), dim3(256), 0, st, s, ids, npairs, out, seq, phases);
}

void launch_compact(const PairState* st_, const int* ids, const int2* cls, int ncls, int* live, int* solving, int* cnt,
                    hipStream_t st) {
  hipLaunchKernelGGL(k_compact, dim3(ncls), dim3(256), 0, st, st_, ids, cls, live, solving, cnt);
}

void launch_compact_running(const PairState* st_, const int* in, const int* in_n, int count, int* out, int* out_n,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_compact_running, dim3(1), dim3(256), 0, st, st_, in, in_n, count, out, out_n);
}

void launch_retire(const LaunchCtx& c, int n, int count, PairState* final_state, hipStream_t st) {
  hipLaunchKernelGGL(k_retire, dim3(elementwise_blocks(n), count), dim3(MA_BLOCK), 0, st, c, final_state);
}

void launch_refill(PairDesc* desc, PairState* state, const RefillRecord* rec, int count, hipStream_t st) {
  hipLaunchKernelGGL(k_refill, dim3(count), dim3(256), 0, st, desc, state, rec);
}

void launch_validate(const double* const* f, const double* const* g, const double* const* psi0, const int* n,
                     int npairs, int nmax, int* bad, hipStream_t st) {
  hipLaunchKernelGGL(k_validate, dim3(elementwise_blocks(nmax), npairs), dim3(MA_BLOCK), 0, st, f, g, psi0, n, bad);
}
