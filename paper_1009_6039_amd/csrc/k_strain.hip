// The GMRES(m) cycle around Strain's operator (Section 4.2 of Saumier, Agueh,
// Khouider): the Arnoldi bookkeeping (Givens rotations, convergence test,
// least-squares solution, restart data), the per-pair finalize kernels that fold the
// passes' partial sums in a fixed order, and the pass launchers that append them.
#include "strain.h"

namespace {

// Arnoldi bookkeeping after ||w'|| is known (one thread): Givens rotations,
// convergence test, and at the end of a cycle the least-squares solution and the
// restart data.  Mirrors Saad's GMRES(m) with rotations.
__device__ void arnoldi_close(PairState& s, const LaunchCtx& c, int jn, double wnorm2) {
  const int j = jn - 1;
  double* col = &s.Hm[j * (MA_MMAX + 1)];
  const double hn = sqrt(fmax(wnorm2, 0.0));
  col[jn] = hn;
  s.vscale[jn] = hn > 0.0 ? 1.0 / hn : 0.0;
  for (int i = 0; i < j; ++i) {
    const double a = col[i], b = col[i + 1];
    col[i] = s.cs[i] * a + s.sn[i] * b;
    col[i + 1] = -s.sn[i] * a + s.cs[i] * b;
  }
  const double den = hypot(col[j], col[j + 1]);
  s.cs[j] = den > 0.0 ? col[j] / den : 1.0;
  s.sn[j] = den > 0.0 ? col[j + 1] / den : 0.0;
  col[j] = den;
  col[j + 1] = 0.0;
  s.gv[jn] = -s.sn[j] * s.gv[j];
  s.gv[j] = s.cs[j] * s.gv[j];
  s.gmres_iters++;
  const bool conv = fabs(s.gv[jn]) <= s.gm_target || hn == 0.0;
  if (!(conv || jn >= c.m)) return;
  const int k = jn;
  for (int i = k - 1; i >= 0; --i) {  // back substitution on the rotated Hessenberg matrix
    double t = s.gv[i];
    for (int l = i + 1; l < k; ++l) t -= s.Hm[l * (MA_MMAX + 1) + i] * s.y[l];
    const double di = s.Hm[i * (MA_MMAX + 1) + i];
    s.y[i] = di != 0.0 ? t / di : 0.0;
  }
  s.gm_k = k;
  s.gm_running = 0;
  if (!conv && s.gm_cycle < c.max_restarts) {
    // residual of the cycle: V_{k+1} Q^T (g_k e_k), Q the product of the rotations
    for (int l = 0; l <= k; ++l) s.q[l] = 0.0;
    s.q[k] = s.gv[k];
    for (int i = k - 1; i >= 0; --i) {
      const double a = s.q[i], b = s.q[i + 1];
      s.q[i] = s.cs[i] * a - s.sn[i] * b;
      s.q[i + 1] = s.sn[i] * a + s.cs[i] * b;
    }
    for (int l = 0; l <= k; ++l) s.q[l] *= s.vscale[l];
    for (int l = 0; l < k; ++l) s.y[l] *= s.vscale[l];
    const double beta = fabs(s.gv[k]);
    s.gv[0] = beta;
    s.vscale[0] = beta > 0.0 ? 1.0 / beta : 0.0;
    s.gm_restart = 1;
  } else {
    for (int l = 0; l < k; ++l) s.y[l] *= s.vscale[l];
    s.gm_restart = 0;
  }
}

// ||w'|| from the pass-A partials (at off, after pass C's), then the rotations and the
// convergence test (on a copy of the pair's state in LDS, loaded together with the
// partials)
__global__ __launch_bounds__(256) void k_arnoldi_finalize(LaunchCtx c, int jn, int nblk, long off) {
  const int p = pair_of_block(c);
  if (p < 0) return;
  const PairDesc d = c.desc[p];
  PairState& s = c.st[p];
  if (!(s.phase == PH_SOLVE && s.gm_running)) return;
  __shared__ double scratch[4];
  __shared__ PairState ls;
  StagedWords<PairState, 256> sw;
  sw.load(&s);
  const int kinds[1] = {0};
  double t[1];
  fold_partials<1>(d.part + off, nblk, kinds, t, scratch);
  sw.to_lds(&ls);
  __syncthreads();
  if (threadIdx.x == 0) arnoldi_close(ls, c, jn, t[0]);
  __syncthreads();
  sw.write_back(&ls, &s);
}

// the scaled right-hand side's norm (option MA_PRECOND_DIAG) from the pass-A partials:
// the GMRES start values that the residual's fold set for the unscaled system
__global__ __launch_bounds__(256) void k_rhs_finalize(LaunchCtx c, int nblk) {
  const int p = pair_of_block(c);
  if (p < 0) return;
  const PairDesc d = c.desc[p];
  PairState& s = c.st[p];
  if (!(s.phase == PH_SOLVE && s.gm_running && s.gm_cycle == 0)) return;
  __shared__ double scratch[4];
  const int kinds[1] = {0};
  double t[1];
  fold_partials<1>(d.part, nblk, kinds, t, scratch);
  if (threadIdx.x == 0) {
    const double bn = sqrt(fmax(t[0], 0.0));
    s.bnorm = bn;
    s.gm_target = pair_eta(s, c) * bn;
    s.gm_running = bn > 0.0;
    s.vscale[0] = bn > 0.0 ? 1.0 / bn : 0.0;
    s.gv[0] = bn;
  }
}

// a restarted cycle begins: its first vector has been transformed by pass A
__global__ void k_cycle_begin(LaunchCtx c) {
  const int p = pair_of_block(c);
  if (p < 0) return;
  PairState& s = c.st[p];
  if (threadIdx.x == 0 && s.phase == PH_SOLVE && s.gm_restart) {
    s.gm_running = 1;
    s.gm_restart = 0;
    s.gm_cycle++;
  }
}

// x += sum y_l v_l and V[0] = the cycle's residual, for a GMRES restart
__global__ __launch_bounds__(MA_BLOCK) void k_restart(LaunchCtx c) {
  const int p = pair_of_block(c);
  if (p < 0) return;
  const PairDesc d = c.desc[p];
  const PairState& s = c.st[p];
  if (!(s.phase == PH_SOLVE && s.gm_restart)) return;
  __shared__ float cy[MA_MMAX + 1], cq[MA_MMAX + 1];
  const int k = s.gm_k;
  const bool usex = s.gm_cycle > 0;
  if (threadIdx.x <= k) {
    cy[threadIdx.x] = threadIdx.x < k ? (float)s.y[threadIdx.x] : 0.f;
    cq[threadIdx.x] = (float)s.q[threadIdx.x];
  }
  __syncthreads();
  const long nn = (long)d.n * d.n;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (long)gridDim.x * blockDim.x) {
    float xs = usex ? d.x[e] : 0.f, r0 = 0.f;
    for (int l = 0; l <= k; ++l) {
      const float v = d.V[(long)l * nn + e];
      xs += cy[l] * v;
      r0 += cq[l] * v;
    }
    d.x[e] = xs;
    d.V[e] = r0;
  }
}

// ---------------------------------------------------------------------------
// Power iteration on the inverse operator (Section 5.1): the vector steps and their
// per-pair folds.  The right-hand side of the next solve lives in r, the solution
// theta = A^{-1} b of the last one in x.
// ---------------------------------------------------------------------------
// elementwise step, with per-block partial sums (FP64) of the value it writes (or reads)
__global__ __launch_bounds__(MA_BLOCK) void k_power_vec(LaunchCtx c, int mode, const float* b0) {
  const int p = pair_of_block(c);
  if (p < 0) return;
  const PairDesc d = c.desc[p];
  const PairState& s = c.st[p];
  const long nn = (long)d.n * d.n;
  double acc = 0.0;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (long)gridDim.x * blockDim.x) {
    if (mode == PW_SUM_B0) {
      acc += (double)b0[e];
    } else if (mode == PW_CENTER) {  // b = b_0 - mean(b_0)
      const float v = (float)((double)b0[e] - s.aux[0]);
      d.r[e] = v;
      acc += (double)v * v;
    } else if (mode == PW_SCALE) {  // b *= 1 / ||b|| (first vector)
      const float v = (float)((double)d.r[e] * s.aux[1]);
      d.r[e] = v;
      acc += (double)v * v;
    } else if (mode == PW_THETA) {  // ||theta||^2
      acc += (double)d.x[e] * d.x[e];
    } else {  // PW_NEXT: b = theta / ||theta||
      const float v = (float)((double)d.x[e] * s.aux[1]);
      d.r[e] = v;
      acc += (double)v * v;
    }
  }
  __shared__ double scratch[MA_BLOCK / 64];
  double v[1] = {acc};
  const int kinds[1] = {0};
  block_reduce<1>(v, kinds, scratch);
  if (threadIdx.x == 0) d.part[blockIdx.x] = v[0];
}

// one block per pair: folds the partial sums of the preceding k_power_vec launch
__global__ __launch_bounds__(256) void k_power_fold(LaunchCtx c, int mode, int nblk, int k, double* out) {
  const int p = pair_of_block(c);
  if (p < 0) return;
  const PairDesc d = c.desc[p];
  PairState& s = c.st[p];
  __shared__ double scratch[4];
  const int kinds[1] = {0};
  double t[1];
  fold_partials<1>(d.part, nblk, kinds, t, scratch);
  if (threadIdx.x != 0) return;
  const double nn = (double)d.n * d.n;
  if (mode == PW_SUM_B0) {
    s.aux[0] = t[0] / nn;
  } else if (mode == PW_CENTER) {
    const double nb = sqrt(fmax(t[0], 0.0));
    s.aux[1] = nb > 0.0 ? 1.0 / nb : 0.0;
  } else if (mode == PW_THETA) {  // rho_k = ||A^{-1} b_k|| for the unit b_k; the next b scales by 1 / rho_k
    const double rho = sqrt(fmax(t[0], 0.0));
    out[2 * k] = rho;
    out[2 * k + 1] = (double)s.gmres_iters;
    s.aux[1] = rho > 0.0 ? 1.0 / rho : 0.0;
  } else {  // PW_SCALE, PW_NEXT: a GMRES solve of A sigma = b starts from sigma = 0
    const double bn = sqrt(fmax(t[0], 0.0));
    s.phase = PH_SOLVE;
    s.bnorm = bn;
    s.gm_target = c.gmres_tol * bn;
    s.gm_running = bn > 0.0;
    s.gm_restart = 0;
    s.gm_cycle = 0;
    s.gm_k = 0;
    s.vscale[0] = bn > 0.0 ? 1.0 / bn : 0.0;
    s.gv[0] = bn;
  }
}

}  // namespace

void launch_power_vec(const LaunchCtx& c, int n, int mode, const float* b0, double* out, int k, hipStream_t st) {
  const int nb = power_blocks(n);
  hipLaunchKernelGGL(k_power_vec, dim3(nb, 1), dim3(MA_BLOCK), 0, st, c, mode, b0);
  hipLaunchKernelGGL(k_power_fold, dim3(1, 1), dim3(256), 0, st, c, mode, nb, k, out);
}

int power_blocks(int n) {
  long b = (long)n * n / (MA_BLOCK * 4);
  return b < 1 ? 1 : (int)(b > 1024 ? 1024 : b);
}

bool fft_size_supported(int n) {
  switch (n) {
#define X(NV) case NV:
    MA_FOR_EACH_N(X)
#undef X
    return true;
    default:
      return false;
  }
}

void launch_passA(const LaunchCtx& c, int n, int npairs, int mode, int jn, const float2* tw, hipStream_t st,
                  const TimedLaunch& ev) {
  // the Arnoldi step folds the inner products of the pass C before it itself (no
  // separate fold kernel) and writes its norm partials after pass C's
  LaunchCtx ca = c;
  ca.dots_nblk = mode == PA_ARNOLDI ? passC_blocks(n, c.var[2]) : 0;
  launch_passA_only(ca, n, npairs, mode, jn, tw, st, ev);
  if (mode == PA_ARNOLDI) {
    const long off = (long)ca.dots_nblk * (MA_MMAX + 1);
    hipLaunchKernelGGL(k_arnoldi_finalize, dim3(1, npairs), dim3(256), 0, st, ca, jn, passA_blocks(n, c.var[0]), off);
  }
  else if (mode == PA_INIT && c.precond == MA_PRECOND_DIAG)
    hipLaunchKernelGGL(k_rhs_finalize, dim3(1, npairs), dim3(256), 0, st, c, passA_blocks(n, c.var[0]));
  else if (mode == PA_PLAIN)
    hipLaunchKernelGGL(k_cycle_begin, dim3(1, npairs), dim3(64), 0, st, c);
}

void launch_passC(const LaunchCtx& c, int n, int npairs, int mode, int j, const float2* tw, hipStream_t st,
                  const TimedLaunch& ev) {
  // (the matvec's inner products are folded by the next pass A)
  launch_passC_only(c, n, npairs, mode, j, tw, st, ev);
}

void launch_restart(const LaunchCtx& c, int n, int npairs, hipStream_t st) {
  long b = (long)n * n / (MA_BLOCK * 4);
  const int nb = b < 1 ? 1 : (int)(b > 4096 ? 4096 : b);
  hipLaunchKernelGGL(k_restart, dim3(nb, npairs), dim3(MA_BLOCK), 0, st, c);
}
