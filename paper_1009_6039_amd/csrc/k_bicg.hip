// The finite-difference linear step of Section 4.1: tilde A theta = b by BiCG.
//
// tilde A = A + 1 1^T, A the nine-point second-order discretisation of
//   L theta = a11 theta_11 + 2 a12 theta_12 + a22 theta_22 + b1 theta_1 + b2 theta_2
// (coefficients of eq. linearmaeq, FP32 planes written by the residual kernel), and
//   A^T y = D11(a11 y) + 2 D12(a12 y) + D22(a22 y) - D1(b1 y) - D2(b2 y),
// since the centred second differences are symmetric and the first differences
// antisymmetric on the periodic grid.  The row of ones adds sum(p) to every entry of
// tilde A p; that sum is carried as a scalar (sum p_{k+1} = sum r_{k+1} + beta sum p_k).
//
// One BiCG iteration over a batch is five launches:
//   matvec     q = tilde A p, q~ = tilde A^T p~, partial sums of p~ . q      (HBM bound)
//   alpha      one block per pair: alpha = rho / (p~ . q), breakdown if zero
//   update     x += alpha p, r -= alpha q, r~ -= alpha q~; partials of r~.r, r.r,
//              sum r, sum r~                                                 (HBM bound)
//   beta       one block per pair: convergence test ||r|| <= tol ||b||, the
//              iteration cap, beta = rho_new / rho, the sums of the new p, p~
//   direction  p = r + beta p, p~ = r~ + beta p~                            (HBM bound)
// Vectors and reductions are FP64; the partial sums are folded in a fixed order, so
// the result does not depend on the batch or the launch order.
#include "common.h"
#include "kernels.h"

namespace {

constexpr int BI_TY = 16;  // tile rows; a block is BI_TY x TX points, 256 threads

// BiCG vector planes inside PairDesc::bv
enum : int { BV_X = 0, BV_R = 1, BV_RT = 2, BV_P = 3, BV_PT = 4, BV_Q = 5, BV_QT = 6 };

__device__ inline bool bicg_live(const PairState& s) {
  return s.phase == PH_SOLVE && s.gm_running && !s.bi_break;
}

// b = (r + translation) / tau; x = 0; r = r~ = p = p~ = b; partials of b.b and sum b
template <int TX>
__global__ __launch_bounds__(256) void k_bicg_init(LaunchCtx c) {
  const int p = pair_of_block(c);
  if (p < 0) return;
  const PairState& s = c.st[p];
  if (s.phase != PH_SOLVE) return;
  const PairDesc& d = c.desc[p];
  const long nn = (long)d.n * d.n;
  const double cst = s.mass_c, inv_tau = 1.0 / s.tau;
  double* bv = d.bv;
  double v[2] = {0.0, 0.0};
  const long base = (long)blockIdx.x * (BI_TY * TX);
  for (int e = threadIdx.x; e < BI_TY * TX; e += 256) {
    const long g = base + e;
    const double b = ((double)d.r[g] + cst) * inv_tau;
    bv[BV_X * nn + g] = 0.0;
    bv[BV_R * nn + g] = b;
    bv[BV_RT * nn + g] = b;
    bv[BV_P * nn + g] = b;
    bv[BV_PT * nn + g] = b;
    v[0] += b * b;
    v[1] += b;
  }
  __shared__ double scratch[4 * 2];
  const int kinds[2] = {0, 0};
  block_reduce<2>(v, kinds, scratch);
  if (threadIdx.x == 0) {
    d.part[(long)blockIdx.x * 2] = v[0];
    d.part[(long)blockIdx.x * 2 + 1] = v[1];
  }
}

// rho_0 = b.b, the sums of p_0 = p~_0 = b, the target tol ||b||
__global__ __launch_bounds__(256) void k_bicg_start(LaunchCtx c, int nblk) {
  const int p = pair_of_block(c);
  if (p < 0) return;
  PairState& s = c.st[p];
  if (s.phase != PH_SOLVE) return;
  const PairDesc& d = c.desc[p];
  __shared__ double scratch[4 * 2];
  const int kinds[2] = {0, 0};
  double t[2];
  fold_partials<2>(d.part, nblk, kinds, t, scratch);
  if (threadIdx.x == 0) {
    s.bi_rho = t[0];
    s.bi_sum_p = t[1];
    s.bi_sum_pt = t[1];
    s.bi_alpha = s.bi_beta = 0.0;
    s.bi_break = 0;
    s.bnorm = sqrt(t[0]);
    s.gm_target = pair_eta(s, c) * s.bnorm;
    s.gm_running = s.bnorm > 0.0;
    s.gm_k = 0;
  }
}

template <int TX>
__global__ __launch_bounds__(256) void k_bicg_matvec(LaunchCtx c) {
  const int p = pair_of_block(c);
  if (p < 0) return;
  const PairState& s = c.st[p];
  if (!bicg_live(s)) return;
  const PairDesc& d = c.desc[p];
  const int n = d.n;
  const long nn = (long)n * n;
  count_bytes(c, 52.0, n);  // p, p~ (FP64), five FP32 coefficients read; q, q~ written
  constexpr int W = TX + 2, H = BI_TY + 2;
  __shared__ double sp[H][W], spt[H][W];
  __shared__ float sc[5][H][W];
  __shared__ double scratch[4];
  const int tpr = n / TX;
  const int i0 = (int)(blockIdx.x / tpr) * BI_TY, j0 = (int)(blockIdx.x % tpr) * TX;
  const double* P_ = d.bv + BV_P * nn;
  const double* PT = d.bv + BV_PT * nn;
  for (int e = threadIdx.x; e < H * W; e += 256) {
    const int a = e / W, b = e % W;
    int gi = i0 + a - 1, gj = j0 + b - 1;
    gi += gi < 0 ? n : (gi >= n ? -n : 0);
    gj += gj < 0 ? n : (gj >= n ? -n : 0);
    const long g = (long)gi * n + gj;
    sp[a][b] = P_[g];
    spt[a][b] = PT[g];
#pragma unroll
    for (int k = 0; k < 5; ++k) sc[k][a][b] = d.coef[k * nn + g];
  }
  __syncthreads();
  const double ih = (double)n, ih2 = (double)n * (double)n, hih = 0.5 * ih, hih2 = 0.5 * ih2;
  const double S = s.bi_sum_p, ST = s.bi_sum_pt;
  double* Q = d.bv + BV_Q * nn;
  double* QT = d.bv + BV_QT * nn;
  double v[1] = {0.0};
  for (int e = threadIdx.x; e < BI_TY * TX; e += 256) {
    const int a = e / TX + 1, b = e % TX + 1;
    const double a11 = sc[0][a][b], a12 = sc[1][a][b], a22 = sc[2][a][b], b1 = sc[3][a][b], b2 = sc[4][a][b];
    const double pc = sp[a][b];
    const double ap = a11 * (sp[a + 1][b] - 2.0 * pc + sp[a - 1][b]) * ih2 +
                      a12 * (sp[a + 1][b + 1] - sp[a + 1][b - 1] - sp[a - 1][b + 1] + sp[a - 1][b - 1]) * hih2 +
                      a22 * (sp[a][b + 1] - 2.0 * pc + sp[a][b - 1]) * ih2 + b1 * (sp[a + 1][b] - sp[a - 1][b]) * hih +
                      b2 * (sp[a][b + 1] - sp[a][b - 1]) * hih + S;
    auto w = [&](int k, int aa, int bb) { return (double)sc[k][aa][bb] * spt[aa][bb]; };
    const double atp = (w(0, a + 1, b) - 2.0 * w(0, a, b) + w(0, a - 1, b)) * ih2 +
                       (w(1, a + 1, b + 1) - w(1, a + 1, b - 1) - w(1, a - 1, b + 1) + w(1, a - 1, b - 1)) * hih2 +
                       (w(2, a, b + 1) - 2.0 * w(2, a, b) + w(2, a, b - 1)) * ih2 -
                       (w(3, a + 1, b) - w(3, a - 1, b)) * hih - (w(4, a, b + 1) - w(4, a, b - 1)) * hih + ST;
    const long g = (long)(i0 + a - 1) * n + (j0 + b - 1);
    Q[g] = ap;
    QT[g] = atp;
    v[0] += spt[a][b] * ap;
  }
  const int kinds[1] = {0};
  block_reduce<1>(v, kinds, scratch);
  if (threadIdx.x == 0) d.part[blockIdx.x] = v[0];
}

__global__ __launch_bounds__(256) void k_bicg_alpha(LaunchCtx c, int nblk) {
  const int p = pair_of_block(c);
  if (p < 0) return;
  PairState& s = c.st[p];
  if (!bicg_live(s)) return;
  const PairDesc& d = c.desc[p];
  __shared__ double scratch[4];
  const int kinds[1] = {0};
  double t[1];
  fold_partials<1>(d.part, nblk, kinds, t, scratch);
  if (threadIdx.x == 0) {
    const double sigma = t[0];
    if (sigma == 0.0 || !isfinite(sigma)) s.bi_break = 1;  // breakdown: keep x as it is
    else s.bi_alpha = s.bi_rho / sigma;
  }
}

template <int TX>
__global__ __launch_bounds__(256) void k_bicg_update(LaunchCtx c) {
  const int p = pair_of_block(c);
  if (p < 0) return;
  const PairState& s = c.st[p];
  if (!bicg_live(s)) return;
  const PairDesc& d = c.desc[p];
  const long nn = (long)d.n * d.n;
  count_bytes(c, 72.0, d.n);  // x, p, r, q, r~, q~ read; x, r, r~ written (FP64)
  const double al = s.bi_alpha;
  double* bv = d.bv;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  const long base = (long)blockIdx.x * (BI_TY * TX);
  for (int e = threadIdx.x; e < BI_TY * TX; e += 256) {
    const long g = base + e;
    bv[BV_X * nn + g] += al * bv[BV_P * nn + g];
    const double r = bv[BV_R * nn + g] - al * bv[BV_Q * nn + g];
    const double rt = bv[BV_RT * nn + g] - al * bv[BV_QT * nn + g];
    bv[BV_R * nn + g] = r;
    bv[BV_RT * nn + g] = rt;
    v[0] += rt * r;
    v[1] += r * r;
    v[2] += r;
    v[3] += rt;
  }
  __shared__ double scratch[4 * 4];
  const int kinds[4] = {0, 0, 0, 0};
  block_reduce<4>(v, kinds, scratch);
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) d.part[(long)blockIdx.x * 4 + k] = v[k];
}

__global__ __launch_bounds__(256) void k_bicg_beta(LaunchCtx c, int nblk) {
  const int p = pair_of_block(c);
  if (p < 0) return;
  PairState& s = c.st[p];
  if (s.phase != PH_SOLVE || !s.gm_running) return;
  if (s.bi_break) {  // (every thread reads the flag before thread 0 clears gm_running)
    __syncthreads();
    if (threadIdx.x == 0) s.gm_running = 0;
    return;
  }
  const PairDesc& d = c.desc[p];
  __shared__ double scratch[4 * 4];
  const int kinds[4] = {0, 0, 0, 0};
  double t[4];
  fold_partials<4>(d.part, nblk, kinds, t, scratch);
  if (threadIdx.x == 0) {
    s.gm_k++;
    s.gmres_iters++;
    const double rho = t[0], rr = t[1];
    if (sqrt(rr) <= s.gm_target || s.gm_k >= c.bicg_max || rho == 0.0 || !isfinite(rho) || !isfinite(rr)) {
      s.gm_running = 0;
    } else {
      const double beta = rho / s.bi_rho;
      s.bi_beta = beta;
      s.bi_rho = rho;
      s.bi_sum_p = t[2] + beta * s.bi_sum_p;
      s.bi_sum_pt = t[3] + beta * s.bi_sum_pt;
    }
  }
}

template <int TX>
__global__ __launch_bounds__(256) void k_bicg_direction(LaunchCtx c) {
  const int p = pair_of_block(c);
  if (p < 0) return;
  const PairState& s = c.st[p];
  if (!bicg_live(s)) return;
  const PairDesc& d = c.desc[p];
  const long nn = (long)d.n * d.n;
  count_bytes(c, 48.0, d.n);  // r, p, r~, p~ read; p, p~ written (FP64)
  const double be = s.bi_beta;
  double* bv = d.bv;
  const long base = (long)blockIdx.x * (BI_TY * TX);
  for (int e = threadIdx.x; e < BI_TY * TX; e += 256) {
    const long g = base + e;
    bv[BV_P * nn + g] = bv[BV_R * nn + g] + be * bv[BV_P * nn + g];
    bv[BV_PT * nn + g] = bv[BV_RT * nn + g] + be * bv[BV_PT * nn + g];
  }
}

// theta = x (kept for step halving), u += x
template <int TX>
__global__ __launch_bounds__(256) void k_bicg_finish(LaunchCtx c) {
  const int p = pair_of_block(c);
  if (p < 0) return;
  const PairState& s = c.st[p];
  if (s.phase != PH_SOLVE) return;
  const PairDesc& d = c.desc[p];
  const long base = (long)blockIdx.x * (BI_TY * TX);
  for (int e = threadIdx.x; e < BI_TY * TX; e += 256) {
    const long g = base + e;
    const double x = d.bv[BV_X * (long)d.n * d.n + g];
    d.theta[g] = x;
    d.u[g] += x;
  }
}

}  // namespace

// tile width: the widest of 64, 32, 16 that divides n (n is a multiple of 16)
int bicg_tx(int n) { return n % 64 == 0 ? 64 : (n % 32 == 0 ? 32 : 16); }
int bicg_blocks(int n) { return n / BI_TY * (n / bicg_tx(n)); }

#define MA_BICG_DISPATCH(EV, KERNEL, ...)                                  \
  do {                                                                     \
    const dim3 grid(bicg_blocks(n), npairs);                               \
    switch (bicg_tx(n)) {                                                  \
      case 64: MA_LAUNCH(EV, KERNEL<64>, grid, dim3(256), st, __VA_ARGS__); break; \
      case 32: MA_LAUNCH(EV, KERNEL<32>, grid, dim3(256), st, __VA_ARGS__); break; \
      default: MA_LAUNCH(EV, KERNEL<16>, grid, dim3(256), st, __VA_ARGS__); break; \
    }                                                                      \
  } while (0)

// one step of the BiCG sequence for the pairs of a class; ev times the matvec only
void launch_bicg(const LaunchCtx& c, int n, int npairs, int step, hipStream_t st, const TimedLaunch& ev) {
  const dim3 one(1, npairs);
  const int nb = bicg_blocks(n);
  const TimedLaunch none;
  switch (step) {
    case BI_INIT:
      MA_BICG_DISPATCH(none, k_bicg_init, c);
      hipLaunchKernelGGL(k_bicg_start, one, dim3(256), 0, st, c, nb);
      break;
    case BI_MATVEC: MA_BICG_DISPATCH(ev, k_bicg_matvec, c); break;
    case BI_ALPHA: hipLaunchKernelGGL(k_bicg_alpha, one, dim3(256), 0, st, c, nb); break;
    case BI_UPDATE: MA_BICG_DISPATCH(none, k_bicg_update, c); break;
    case BI_BETA: hipLaunchKernelGGL(k_bicg_beta, one, dim3(256), 0, st, c, nb); break;
    case BI_DIRECTION: MA_BICG_DISPATCH(none, k_bicg_direction, c); break;
    case BI_FINISH: MA_BICG_DISPATCH(none, k_bicg_finish, c); break;
    default: break;
  }
}
