// The finite-difference linear step of Section 4.1: tilde A theta = b by BiCG.
//
// tilde A = A + 1 1^T, A the nine-point second-order discretisation of
//   L theta = a11 theta_11 + 2 a12 theta_12 + a22 theta_22 + b1 theta_1 + b2 theta_2
// (coefficients of eq. linearmaeq, FP32 planes written by the residual kernel), and
//   A^T y = D11(a11 y) + 2 D12(a12 y) + D22(a22 y) - D1(b1 y) - D2(b2 y),
// since the centred second differences are symmetric and the first differences
// antisymmetric on the periodic grid.  The row of ones adds sum(p) to every entry of
// tilde A p; that sum is carried as a scalar (sum p_j = sum r_j + beta_j sum p_{j-1}).
//
// BiCG iteration j over a batch is two launches:
//   direction+matvec  every block folds the previous update's partial sums (r~.r, r.r,
//                     sum r, sum r~), takes the convergence test ||r|| <= tol ||b|| and
//                     beta_j = rho_j / rho_{j-1}, forms p_j = r_j + beta_j p_{j-1} (and
//                     p~_j) over its tile and halo in LDS, writes them, and applies
//                     tilde A and tilde A^T; partial sums of p~_j . q_j   (HBM bound)
//   update            every block folds the p~.q partials: alpha_j = rho_j / (p~.q)
//                     (a zero denominator stops the iteration), x += alpha p,
//                     r -= alpha q, r~ -= alpha q~; partial sums for the next test
//                                                                         (HBM bound)
// p and p~ alternate between two planes by the parity of j, so that no block
// overwrites a value another block still reads; rho and sum p alternate in the pair
// state in the same way.  Decisions taken by every block from the same fixed-order fold
// agree; only block 0 writes them to the state.  Vectors and reductions are FP64.
#include "common.h"
#include "kernels.h"

namespace {

constexpr int BI_TY = 16;  // tile rows; a block is BI_TY x TX points, 256 threads
static_assert(BI_TY * 16 % 256 == 0, "whole points per thread in the elementwise kernels");

// BiCG vector planes inside PairDesc::bv (p, p~ in two planes each, by parity)
enum : int { BV_X = 0, BV_R = 1, BV_RT = 2, BV_Q = 3, BV_QT = 4, BV_P0 = 5, BV_PT0 = 6, BV_P1 = 7, BV_PT1 = 8 };
__device__ inline int bv_p(int j) { return (j & 1) ? BV_P1 : BV_P0; }
__device__ inline int bicg_blocks_dev(int n, int tx) { return n / BI_TY * (n / tx); }
__device__ inline int bv_pt(int j) { return (j & 1) ? BV_PT1 : BV_PT0; }

// Sums of K partials per block over nblk blocks, in a fixed order, in every thread
template <int K>
__device__ inline void fold_all(const double* part, int nblk, double (&t)[K]) {
  __shared__ double scratch[4 * K];
  __shared__ double out[K];
  const int kinds[K] = {};
  fold_partials<K>(part, nblk, kinds, t, scratch);
  if (threadIdx.x == 0)
    for (int k = 0; k < K; ++k) out[k] = t[k];
  __syncthreads();
  for (int k = 0; k < K; ++k) t[k] = out[k];
}

// b = (r + translation) / tau; x = 0; r = r~ = p_0 = p~_0 = b; partials of b.b and sum b
template <int TX>
__global__ __launch_bounds__(256) void k_bicg_init(LaunchCtx c) {
  const int p = pair_of_block(c);
  if (p < 0) return;
  const PairState& s = c.st[p];
  if (s.phase != PH_SOLVE) return;
  const PairDesc d = c.desc[p];
  const long nn = (long)d.n * d.n;
  const int nb = bicg_blocks_dev(d.n, TX);
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
    bv[BV_P0 * nn + g] = b;
    bv[BV_PT0 * nn + g] = b;
    v[0] += b * b;
    v[1] += b;
  }
  __shared__ double scratch[4 * 2];
  const int kinds[2] = {0, 0};
  block_reduce<2>(v, kinds, scratch);
  if (threadIdx.x == 0) {
    d.part[nb + (long)blockIdx.x * 2] = v[0];
    d.part[nb + (long)blockIdx.x * 2 + 1] = v[1];
  }
}

// rho_0 = b.b, the sums of p_0 = p~_0 = b, the target tol ||b|| (one block per pair)
__global__ __launch_bounds__(256) void k_bicg_start(LaunchCtx c, int nblk) {
  const int p = pair_of_block(c);
  if (p < 0) return;
  PairState& s = c.st[p];
  if (s.phase != PH_SOLVE) return;
  const PairDesc d = c.desc[p];
  __shared__ double scratch[4 * 2];
  const int kinds[2] = {0, 0};
  double t[2];
  fold_partials<2>(d.part + nblk, nblk, kinds, t, scratch);
  if (threadIdx.x == 0) {
    s.bi_rho[0] = t[0];
    s.bi_sum_p[0] = t[1];
    s.bi_sum_pt[0] = t[1];
    s.bi_break = 0;
    s.bnorm = sqrt(t[0]);
    s.gm_target = pair_eta(s, c) * s.bnorm;
    s.gm_running = s.bnorm > 0.0;
    s.gm_k = 0;
  }
}

// Iteration j >= 1: the test on r_j and the new directions, then q = tilde A p_j and
// q~ = tilde A^T p~_j.  j = 0 applies the operators to p_0 as stored (no test, no
// direction): the first iteration of a solve and the step entry point.
template <int TX>
__global__ __launch_bounds__(256) void k_bicg_matvec(LaunchCtx c, int j) {
  const int p = pair_of_block(c);
  if (p < 0) return;
  PairState& s = c.st[p];
  // the state flags are read once per block (block 0 of this launch may be writing
  // them), so that every wave of a block takes the same branch
  __shared__ int go;
  if (threadIdx.x == 0) go = s.phase != PH_SOLVE || !s.gm_running ? 0 : (s.bi_break ? 2 : 1);
  __syncthreads();
  if (go == 0) return;
  if (go == 2) {  // the last update met a zero denominator: stop with x as it is
    if (blockIdx.x == 0 && threadIdx.x == 0) s.gm_running = 0;
    return;
  }
  const PairDesc d = c.desc[p];
  const int n = d.n;
  const long nn = (long)n * n;
  const int nb = bicg_blocks_dev(n, TX);
  const int cur = j & 1, prev = cur ^ 1;
  constexpr int W = TX + 2, H = BI_TY + 2, NLD = (H * W + 255) / 256;
  const int tpr = n / TX;
  const int i0 = (int)(blockIdx.x / tpr) * BI_TY, j0 = (int)(blockIdx.x % tpr) * TX;
  // every load of the tile and its halo is issued before the fold below (a slot past
  // the tile reloads the tile's first point and is never stored; for j = 0 the r loads
  // repeat the p loads)
  const auto bv = gmem<double>(d.bv);
  const auto coef = gmem<const float>(d.coef);
  const auto Pin = bv + (j > 0 ? bv_p(prev) : BV_P0) * nn;
  const auto PTin = bv + (j > 0 ? bv_pt(prev) : BV_PT0) * nn;
  const auto R = j > 0 ? bv + BV_R * nn : Pin;
  const auto RT = j > 0 ? bv + BV_RT * nn : PTin;
  double lp[NLD], lpt[NLD], lr[NLD], lrt[NLD];
  float lc[NLD][5];
#pragma unroll
  for (int q = 0; q < NLD; ++q) {
    const int e0 = threadIdx.x + q * 256;
    const int e = e0 < H * W ? e0 : 0;
    const int a = e / W, b = e % W;
    int gi = i0 + a - 1, gj = j0 + b - 1;
    gi += gi < 0 ? n : (gi >= n ? -n : 0);
    gj += gj < 0 ? n : (gj >= n ? -n : 0);
    const long g = (long)gi * n + gj;
    lp[q] = Pin[g];
    lpt[q] = PTin[g];
    lr[q] = R[g];
    lrt[q] = RT[g];
#pragma unroll
    for (int k = 0; k < 5; ++k) lc[q][k] = coef[k * nn + g];
  }
  double beta = 0.0, S, ST;
  if (j == 0) {
    S = s.bi_sum_p[0];
    ST = s.bi_sum_pt[0];
  } else {
    double t[4];
    fold_all<4>(d.part + nb, nb, t);  // r~.r, r.r, sum r, sum r~ after the last update
    const double rho = t[0], rr = t[1];
    if (sqrt(rr) <= s.gm_target || j >= c.bicg_max || rho == 0.0 || !isfinite(rho) || !isfinite(rr)) {
      if (blockIdx.x == 0 && threadIdx.x == 0) s.gm_running = 0;
      return;
    }
    beta = rho / s.bi_rho[prev];
    S = t[2] + beta * s.bi_sum_p[prev];
    ST = t[3] + beta * s.bi_sum_pt[prev];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      s.bi_rho[cur] = rho;
      s.bi_sum_p[cur] = S;
      s.bi_sum_pt[cur] = ST;
    }
  }
  // algorithmic bytes per point: r, p, r~, p~ (FP64) and five FP32 coefficients read,
  // p, p~, q, q~ written; j = 0 reads only p, p~ and writes only q, q~
  count_bytes(c, j > 0 ? 84.0 : 52.0, n);
  __shared__ double sp[H][W], spt[H][W];
  __shared__ float sc[5][H][W];
#pragma unroll
  for (int q = 0; q < NLD; ++q) {
    const int e = threadIdx.x + q * 256;
    if (e >= H * W) continue;
    const int a = e / W, b = e % W;
    if (j > 0) {
      sp[a][b] = lr[q] + beta * lp[q];
      spt[a][b] = lrt[q] + beta * lpt[q];
    } else {
      sp[a][b] = lp[q];
      spt[a][b] = lpt[q];
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) sc[k][a][b] = lc[q][k];
  }
  __syncthreads();
  const double ih = (double)n, ih2 = (double)n * (double)n, hih = 0.5 * ih, hih2 = 0.5 * ih2;
  const auto Q = bv + BV_Q * nn;
  const auto QT = bv + BV_QT * nn;
  const auto Pout = bv + bv_p(cur) * nn;
  const auto PTout = bv + bv_pt(cur) * nn;
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
    if (j > 0) {
      Pout[g] = pc;
      PTout[g] = spt[a][b];
    }
    Q[g] = ap;
    QT[g] = atp;
    v[0] += spt[a][b] * ap;
  }
  __shared__ double scratch[4];
  const int kinds[1] = {0};
  block_reduce<1>(v, kinds, scratch);
  if (threadIdx.x == 0) d.part[blockIdx.x] = v[0];
}

// alpha_j = rho_j / (p~_j . q_j); x += alpha p_j, r -= alpha q, r~ -= alpha q~
template <int TX>
__global__ __launch_bounds__(256) void k_bicg_update(LaunchCtx c, int j) {
  const int p = pair_of_block(c);
  if (p < 0) return;
  PairState& s = c.st[p];
  __shared__ int go;  // read once per block, as in the matvec
  if (threadIdx.x == 0) go = s.phase == PH_SOLVE && s.gm_running && !s.bi_break;
  __syncthreads();
  if (!go) return;
  const PairDesc d = c.desc[p];
  const long nn = (long)d.n * d.n;
  const int nb = bicg_blocks_dev(d.n, TX);
  // the block's loads are issued before the fold of the p~.q partials
  constexpr int PER = BI_TY * TX / 256;
  const auto bv = gmem<double>(d.bv);
  const auto P_ = bv + bv_p(j) * nn;
  const long base = (long)blockIdx.x * (BI_TY * TX);
  double lx[PER], lp[PER], lr[PER], lq[PER], lrt[PER], lqt[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const long g = base + threadIdx.x + q * 256;
    lx[q] = bv[BV_X * nn + g];
    lp[q] = P_[g];
    lr[q] = bv[BV_R * nn + g];
    lq[q] = bv[BV_Q * nn + g];
    lrt[q] = bv[BV_RT * nn + g];
    lqt[q] = bv[BV_QT * nn + g];
  }
  double t[1];
  fold_all<1>(d.part, nb, t);
  const double sigma = t[0];
  if (sigma == 0.0 || !isfinite(sigma)) {  // breakdown: the next launch stops the pair
    if (blockIdx.x == 0 && threadIdx.x == 0) s.bi_break = 1;
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    s.gm_k = j + 1;
    s.gmres_iters++;
  }
  count_bytes(c, 72.0, d.n);  // x, p, r, q, r~, q~ read; x, r, r~ written (FP64)
  const double al = s.bi_rho[j & 1] / sigma;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const long g = base + threadIdx.x + q * 256;
    bv[BV_X * nn + g] = lx[q] + al * lp[q];
    const double r = lr[q] - al * lq[q];
    const double rt = lrt[q] - al * lqt[q];
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
    for (int k = 0; k < 4; ++k) d.part[nb + (long)blockIdx.x * 4 + k] = v[k];
}

// theta = x (kept for step halving), u += x
template <int TX>
__global__ __launch_bounds__(256) void k_bicg_finish(LaunchCtx c) {
  const int p = pair_of_block(c);
  if (p < 0) return;
  const PairState& s = c.st[p];
  if (s.phase != PH_SOLVE) return;
  const PairDesc d = c.desc[p];
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

#define MA_BICG_DISPATCH(EV, KERNEL, ...)                                           \
  do {                                                                              \
    const dim3 grid(bicg_blocks(n), npairs);                                        \
    switch (bicg_tx(n)) {                                                           \
      case 64: MA_LAUNCH(EV, KERNEL<64>, grid, dim3(256), st, __VA_ARGS__); break; \
      case 32: MA_LAUNCH(EV, KERNEL<32>, grid, dim3(256), st, __VA_ARGS__); break; \
      default: MA_LAUNCH(EV, KERNEL<16>, grid, dim3(256), st, __VA_ARGS__); break; \
    }                                                                               \
  } while (0)

// one step of the BiCG sequence for the pairs of a class (j: the iteration); ev times
// the direction+matvec launch only
void launch_bicg(const LaunchCtx& c, int n, int npairs, int step, int j, hipStream_t st, const TimedLaunch& ev) {
  const TimedLaunch none;
  switch (step) {
    case BI_INIT:
      MA_BICG_DISPATCH(none, k_bicg_init, c);
      hipLaunchKernelGGL(k_bicg_start, dim3(1, npairs), dim3(256), 0, st, c, bicg_blocks(n));
      break;
    case BI_MATVEC: MA_BICG_DISPATCH(ev, k_bicg_matvec, c, j); break;
    case BI_UPDATE: MA_BICG_DISPATCH(none, k_bicg_update, c, j); break;
    case BI_FINISH: MA_BICG_DISPATCH(none, k_bicg_finish, c); break;
    default: break;
  }
}
