// Strain's FFT operator and the GMRES(m) cycle (Section 4.2 of Saumier, Agueh,
// Khouider), in three passes over the grid per operator application:
//
//   pass A  row pass: builds the Krylov vector on the fly (right-hand side,
//           Gram-Schmidt update, or solution recovery), then a length-N FFT of two
//           real rows packed as one complex row, split into two half spectra.
//           Half-spectrum layout H[i][s], s < N/2: slot 0 packs the real DC and
//           Nyquist coefficients of row i as (Re X_i[0], Re X_i[N/2]).
//   pass B  column pass: FFT along x1 of each slot, multiply by rhobar(k) (and the
//           Krylov scale, and 1/N^2), then inverse FFTs of rhobar*sigmahat times
//           1, 2 pi i k1 and -(2 pi k1)^2 (three outputs T0, T1, T2).
//   pass C  row pass: five real inverse transforms along x2 taken as complex pairs
//           (alpha11 + i beta1, alpha12 + i beta2 per row, alpha22 of two rows),
//           the pointwise combination w = a11 alpha11 + 2 a12 alpha12 + a22 alpha22
//           + b1 beta1 + b2 beta2, and the Arnoldi inner products <w, v_l>.
//
// Wavenumber conventions (reading P8): k in -N/2 .. N/2-1; the first-derivative
// multiplier 2 pi i k is zero at k = -N/2, the second-derivative multiplier
// -(2 pi k)^2 is used for every k; rhobar(0) = 0.
#include "common.h"
#include "fft.h"
#include "kernels.h"
#include "ma_ot.h"

namespace {

__host__ __device__ constexpr int pow2_div(int limit, int m) {
  int p = 1;
  while (p * 2 <= limit && m % (p * 2) == 0) p *= 2;
  return p;
}
__host__ __device__ constexpr int round_block(int t, int cap = 256) {
  int b = ((t + 63) / 64) * 64;
  return b < 64 ? 64 : (b > cap ? cap : b);
}

// launch geometry per grid size
template <int N>
struct Cfg {
  static constexpr int NH = N / 2;
  static constexpr int A_PPB = pow2_div(1024 / N > 0 ? 1024 / N : 1, NH);   // row pairs per block
  static constexpr int A_BLOCK = round_block(A_PPB * N / 8);
  static constexpr int B_CPB = pow2_div(4096 / N > 0 ? 4096 / N : 1, NH);   // columns per block
  static constexpr int B_BLOCK = round_block(B_CPB * N / 8);
  static constexpr int C_PPB = pow2_div(512 / N > 0 ? 512 / N : 1, NH);     // row pairs per block
  static constexpr int C_BLOCK = round_block(5 * C_PPB * N / 8, 320);  // one butterfly per thread at 512
  static_assert((N * B_CPB) % B_BLOCK == 0, "column pass: whole elements per thread");
  static_assert(B_BLOCK % B_CPB == 0, "column pass: fixed column per thread");
};

// rhobar(k): inverse symbol of the averaged operator (Section 4.2), zero at k = 0.
// q: FFT index of k1; q2: FFT index of k2 (N/2 for the Nyquist column).
// mt[q] = (Im of the first-derivative multiplier, second-derivative multiplier).
template <int N>
__device__ __forceinline__ float2 rhobar(int q, int q2, const float (&ab)[5], const float2* __restrict__ mt) {
  if (q == 0 && q2 == 0) return make_float2(0.f, 0.f);
  const float2 m1 = mt[q], m2 = mt[q2];
  // S = a11 d2(k1) + 2 a12 (i d1(k1))(i d1(k2)) + a22 d2(k2) + i (b1 d1(k1) + b2 d1(k2))
  const float re = ab[0] * m1.y + ab[2] * m2.y - 2.f * ab[1] * m1.x * m2.x;
  const float im = ab[3] * m1.x + ab[4] * m2.x;
  const float den = re * re + im * im;
  return make_float2(re / den, -im / den);
}

// Z[k] = A + iB and Z[N-k] = conj(A) + i conj(B): the full spectrum of the complex
// signal whose real / imaginary parts have half spectra A / B
template <int N>
__device__ __forceinline__ void put_pair(float2* L, int k, float2 A, float2 B) {
  L[k] = make_float2(A.x - B.y, A.y + B.x);
  L[N - k] = make_float2(A.x + B.y, B.x - A.y);
}
__device__ __forceinline__ float2 times_i(float s, float2 a) { return make_float2(-s * a.y, s * a.x); }

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

// ---------------------------------------------------------------------------
// pass A
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(Cfg<N>::A_BLOCK) void k_passA(LaunchCtx c, int mode, int jn,
                                                           const float2* __restrict__ tw) {
  constexpr int PPB = Cfg<N>::A_PPB, BLOCK = Cfg<N>::A_BLOCK, NH = N / 2;
  constexpr long NN = (long)N * N;
  const int p = pair_of_block(c);
  const PairDesc& d = c.desc[p];
  PairState& s = c.st[p];
  bool run;
  if (mode == PA_INIT) run = s.phase == PH_SOLVE && s.gm_running && s.gm_cycle == 0;
  else if (mode == PA_PLAIN) run = s.phase == PH_SOLVE && s.gm_restart;
  else if (mode == PA_ARNOLDI) run = s.phase == PH_SOLVE && s.gm_running;
  else if (mode == PA_RECOVER) run = s.phase == PH_SOLVE;
  else run = true;
  if (!run) return;

  __shared__ float2 lds[PPB * N];
  __shared__ float cf[MA_MMAX + 1];
  __shared__ double scratch[BLOCK / 64];
  int nv = 0;
  bool usex = false;
  if (mode == PA_ARNOLDI) nv = jn;
  else if (mode == PA_RECOVER) { nv = s.gm_k; usex = s.gm_cycle > 0; }
  if (threadIdx.x < nv) {
    const int l = threadIdx.x;
    cf[l] = mode == PA_ARNOLDI ? (float)(s.Hm[(jn - 1) * (MA_MMAX + 1) + l] * s.vscale[l]) : (float)s.y[l];
  }
  const float cst = (float)s.mass_c, inv_tau = (float)(1.0 / s.tau);
  {  // algorithmic bytes per point: vectors read, Krylov vector written, half spectrum written
    const bool fft = !(mode == PA_ARNOLDI && jn >= c.m);
    double b = fft ? 4.0 : 0.0;
    if (mode == PA_INIT) b += 8.0;
    else if (mode == PA_PLAIN || mode == PA_STEP) b += 4.0;
    else if (mode == PA_ARNOLDI) b += 4.0 * (jn + 1) + 4.0;
    else b += 4.0 * (nv + (usex ? 1 : 0));
    count_bytes(c, b, N);
  }
  __syncthreads();

  const int row0 = 2 * blockIdx.x * PPB;
  float* V = d.V;
  float* Vj = V + (long)jn * NN;
  float nrm = 0.f;
  for (int e = threadIdx.x; e < PPB * N; e += BLOCK) {
    const int pp = e / N, jj = e % N;
    const long ea = (long)(row0 + 2 * pp) * N + jj, eb = ea + N;
    float va, vb;
    if (mode == PA_INIT) {
      va = (d.r[ea] + cst) * inv_tau;
      vb = (d.r[eb] + cst) * inv_tau;
      V[ea] = va;
      V[eb] = vb;
    } else if (mode == PA_PLAIN || mode == PA_STEP) {
      va = V[ea];
      vb = V[eb];
    } else if (mode == PA_ARNOLDI) {
      va = Vj[ea];
      vb = Vj[eb];
      for (int l = 0; l < nv; ++l) {
        const float* Vl = V + (long)l * NN;
        va -= cf[l] * Vl[ea];
        vb -= cf[l] * Vl[eb];
      }
      Vj[ea] = va;
      Vj[eb] = vb;
      nrm += va * va + vb * vb;
    } else {  // PA_RECOVER
      va = usex ? d.x[ea] : 0.f;
      vb = usex ? d.x[eb] : 0.f;
      for (int l = 0; l < nv; ++l) {
        const float* Vl = V + (long)l * NN;
        va += cf[l] * Vl[ea];
        vb += cf[l] * Vl[eb];
      }
    }
    lds[pp * N + jj] = make_float2(va, vb);
  }

  if (!(mode == PA_ARNOLDI && jn >= c.m)) {
    __syncthreads();
    fft_lds<N, PPB, BLOCK, false, LAYOUT_ROWS>(lds, tw);
    for (int e = threadIdx.x; e < PPB * NH; e += BLOCK) {
      const int pp = e / NH, k = e % NH;
      const long ia = (long)(row0 + 2 * pp) * NH + k, ib = ia + NH;
      const float2 zk = lds[pp * N + k];
      float2 oa, ob;
      if (k == 0) {
        const float2 zn = lds[pp * N + NH];
        oa = make_float2(zk.x, zn.x);
        ob = make_float2(zk.y, zn.y);
      } else {
        const float2 zm = lds[pp * N + N - k];
        oa = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
        ob = make_float2(0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x));
      }
      d.H[ia] = oa;
      d.H[ib] = ob;
    }
  }

  if (mode == PA_ARNOLDI) {  // partial ||w'||^2, folded by k_arnoldi_finalize
    double v[1] = {(double)nrm};
    const int kinds[1] = {0};
    block_reduce<1>(v, kinds, scratch);
    if (threadIdx.x == 0) d.part[blockIdx.x] = v[0];
  }
}

// ---------------------------------------------------------------------------
// pass B (columns)
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(Cfg<N>::B_BLOCK) void k_passB(LaunchCtx c, int mode, int j,
                                                           const float2* __restrict__ tw) {
  constexpr int CPB = Cfg<N>::B_CPB, BLOCK = Cfg<N>::B_BLOCK, NH = N / 2;
  const int p = pair_of_block(c);
  const PairDesc& d = c.desc[p];
  const PairState& s = c.st[p];
  bool run;
  if (mode == PB_MATVEC) run = s.phase == PH_SOLVE && s.gm_running;
  else if (mode == PB_RECOVER) run = s.phase == PH_SOLVE;
  else run = true;
  if (!run) return;
  count_bytes(c, mode == PB_MATVEC ? 16.0 : 8.0, N);  // half spectrum in, one or three out

  // S: the column spectra, then rhobar * sigmahat; W: work buffer for derived spectra.
  // Element (row or wavenumber e, column cc) sits at e * CPB + cc.
  __shared__ float2 S[N * CPB];
  __shared__ float2 Wb[N * CPB];
  const int s0 = blockIdx.x * CPB;
  for (int e = threadIdx.x; e < N * CPB; e += BLOCK) {
    const int i = e / CPB, cc = e % CPB;
    S[e] = d.H[(long)i * NH + s0 + cc];
  }
  __syncthreads();
  fft_lds<N, CPB, BLOCK, false, LAYOUT_COLS>(S, tw);
  if (mode == PB_FORWARD) {
    for (int e = threadIdx.x; e < N * CPB; e += BLOCK) {
      const int i = e / CPB, cc = e % CPB;
      d.T[(long)i * NH + s0 + cc] = S[e];
    }
    return;
  }
  const float scale = (float)((mode == PB_MATVEC ? s.vscale[j] : 1.0) / ((double)N * (double)N));
  float ab[5];
  for (int k = 0; k < 5; ++k) ab[k] = (float)s.abar[k];
  // wavenumbers q and N - q together: slot 0 packs the DC and Nyquist columns of the
  // rows, which separate with the partner coefficient; every later multiplier m(q)
  // then acts on the packed value P = sA + i sB directly
  for (int it = threadIdx.x; it < (NH + 1) * CPB; it += BLOCK) {
    const int q = it / CPB, cc = it % CPB;
    const int qm = (N - q) % N;
    const int slot = s0 + cc;
    const float2 z = S[q * CPB + cc], zm = S[qm * CPB + cc];
    float2 vq, vm;
    if (slot != 0) {
      vq = cscale(cmul(rhobar<N>(q, slot, ab, c.mt), z), scale);
      vm = cscale(cmul(rhobar<N>(qm, slot, ab, c.mt), zm), scale);
    } else {
      const float2 A = make_float2(0.5f * (z.x + zm.x), 0.5f * (z.y - zm.y));
      const float2 B = make_float2(0.5f * (z.y + zm.y), -0.5f * (z.x - zm.x));
      const float2 aq = cmul(rhobar<N>(q, 0, ab, c.mt), A), bq = cmul(rhobar<N>(q, NH, ab, c.mt), B);
      const float2 am = cmul(rhobar<N>(qm, 0, ab, c.mt), cconj(A));
      const float2 bm = cmul(rhobar<N>(qm, NH, ab, c.mt), cconj(B));
      vq = cscale(make_float2(aq.x - bq.y, aq.y + bq.x), scale);
      vm = cscale(make_float2(am.x - bm.y, am.y + bm.x), scale);
    }
    S[q * CPB + cc] = vq;
    if (qm != q) S[qm * CPB + cc] = vm;
  }
  __syncthreads();
  // derived spectra 2 pi i k1 and -(2 pi k1)^2 (matvec only), then the plain one in place
  const int nout = mode == PB_MATVEC ? 3 : 1;
  for (int oo = 0; oo < nout; ++oo) {
    const int o = (oo + 1) % 3 == 0 || nout == 1 ? 0 : oo + 1;  // order 1, 2, 0
    float2* L = (o == 0) ? S : Wb;
    if (o != 0) {
      for (int e = threadIdx.x; e < N * CPB; e += BLOCK) {
        const int q = e / CPB;
        const float2 m = c.mt[q];
        const float2 v = S[e];
        Wb[e] = (o == 1) ? times_i(m.x, v) : cscale(v, m.y);
      }
      __syncthreads();
    }
    fft_lds<N, CPB, BLOCK, true, LAYOUT_COLS>(L, tw);
    float2* To = d.T + (long)o * N * NH;
    for (int e = threadIdx.x; e < N * CPB; e += BLOCK) {
      const int i = e / CPB, c2 = e % CPB;
      To[(long)i * NH + s0 + c2] = L[e];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// pass C (rows)
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(Cfg<N>::C_BLOCK) void k_passC(LaunchCtx c, int mode, int j,
                                                           const float2* __restrict__ tw) {
  constexpr int PPB = Cfg<N>::C_PPB, BLOCK = Cfg<N>::C_BLOCK, NH = N / 2;
  constexpr long NN = (long)N * N;
  const int p = pair_of_block(c);
  const PairDesc& d = c.desc[p];
  PairState& s = c.st[p];
  const bool run = mode == PC_MATVEC ? (s.phase == PH_SOLVE && s.gm_running) : (s.phase == PH_SOLVE);
  if (!run) return;

  // three half spectra 12, coefficients 20, Krylov vectors for the dots, w 4 (matvec);
  // one half spectrum 4, theta 8, u read and written 16 (recovery)
  count_bytes(c, mode == PC_MATVEC ? 36.0 + 4.0 * (j + 1) : (mode == PC_RECOVER ? 28.0 : 8.0), N);
  __shared__ float2 lds[5 * PPB * N];
  __shared__ double red[(BLOCK / 64) * (MA_MMAX + 1)];
  const int row0 = 2 * blockIdx.x * PPB;
  const float2* T0 = d.T;
  const float2* T1 = d.T + NN / 2;
  const float2* T2 = d.T + NN;

  if (mode != PC_MATVEC) {
    // theta = Lbar^{-1} sigma: one complex inverse transform per row pair
    for (int e = threadIdx.x; e < PPB * NH; e += BLOCK) {
      const int pp = e / NH, k = e % NH;
      const long ia = (long)(row0 + 2 * pp) * NH + k;
      const float2 a = T0[ia], b = T0[ia + NH];
      float2* L = lds + pp * N;
      if (k == 0) {
        L[0] = make_float2(a.x, b.x);
        L[NH] = make_float2(a.y, b.y);
      } else {
        put_pair<N>(L, k, a, b);
      }
    }
    __syncthreads();
    fft_lds<N, PPB, BLOCK, true, LAYOUT_ROWS>(lds, tw);
    for (int e = threadIdx.x; e < PPB * N; e += BLOCK) {
      const int pp = e / N, jj = e % N;
      const long ea = (long)(row0 + 2 * pp) * N + jj, eb = ea + N;
      const float2 z = lds[pp * N + jj];
      if (mode == PC_RECOVER) {  // FP64 correction kept for step halving; u in FP64
        d.theta[ea] = (double)z.x;
        d.theta[eb] = (double)z.y;
        d.u[ea] += (double)z.x;
        d.u[eb] += (double)z.y;
      } else {  // single-step use: FP32 result in the x buffer
        d.x[ea] = z.x;
        d.x[eb] = z.y;
      }
    }
    return;
  }

  // five complex inverse transforms per row pair
  for (int e = threadIdx.x; e < PPB * NH; e += BLOCK) {
    const int pp = e / NH, k = e % NH;
    const long ia = (long)(row0 + 2 * pp) * NH + k, ib = ia + NH;
    const float2 t0a = T0[ia], t1a = T1[ia], t2a = T2[ia];
    const float2 t0b = T0[ib], t1b = T1[ib], t2b = T2[ib];
    float2* L = lds + 5 * pp * N;
    if (k == 0) {
      // DC (.x) and Nyquist (.y) are real; the first-derivative multiplier vanishes at
      // both, the second-derivative one at DC
      const float d2n = c.mt[NH].y;
      L[0] = make_float2(t2a.x, t1a.x);
      L[NH] = make_float2(t2a.y, t1a.y);
      L[N] = make_float2(0.f, 0.f);
      L[N + NH] = make_float2(0.f, 0.f);
      L[2 * N] = make_float2(t2b.x, t1b.x);
      L[2 * N + NH] = make_float2(t2b.y, t1b.y);
      L[3 * N] = make_float2(0.f, 0.f);
      L[3 * N + NH] = make_float2(0.f, 0.f);
      L[4 * N] = make_float2(0.f, 0.f);
      L[4 * N + NH] = make_float2(d2n * t0a.y, d2n * t0b.y);
    } else {
      const float2 m = c.mt[k];
      put_pair<N>(L, k, t2a, t1a);
      put_pair<N>(L + N, k, times_i(m.x, t1a), times_i(m.x, t0a));
      put_pair<N>(L + 2 * N, k, t2b, t1b);
      put_pair<N>(L + 3 * N, k, times_i(m.x, t1b), times_i(m.x, t0b));
      put_pair<N>(L + 4 * N, k, cscale(t0a, m.y), cscale(t0b, m.y));
    }
  }
  __syncthreads();
  fft_lds<N, 5 * PPB, BLOCK, true, LAYOUT_ROWS>(lds, tw);

  float* W = d.V + (long)(j + 1) * NN;
  const float* coef = d.coef;
  float dots[MA_MMAX + 1];
#pragma unroll
  for (int l = 0; l <= MA_MMAX; ++l) dots[l] = 0.f;
  for (int e = threadIdx.x; e < PPB * N; e += BLOCK) {
    const int pp = e / N, jj = e % N;
    const long ea = (long)(row0 + 2 * pp) * N + jj, eb = ea + N;
    const float2* L = lds + 5 * pp * N + jj;
    const float2 z0 = L[0], z1 = L[N], z2 = L[2 * N], z3 = L[3 * N], z4 = L[4 * N];
    const float wa = coef[ea] * z0.x + 2.f * coef[NN + ea] * z1.x + coef[2 * NN + ea] * z4.x +
                     coef[3 * NN + ea] * z0.y + coef[4 * NN + ea] * z1.y;
    const float wb = coef[eb] * z2.x + 2.f * coef[NN + eb] * z3.x + coef[2 * NN + eb] * z4.y +
                     coef[3 * NN + eb] * z2.y + coef[4 * NN + eb] * z3.y;
    W[ea] = wa;
    W[eb] = wb;
#pragma unroll
    for (int l = 0; l <= MA_MMAX; ++l)
      if (l <= j) {
        const float* Vl = d.V + (long)l * NN;
        dots[l] += wa * Vl[ea] + wb * Vl[eb];
      }
  }
  // block reduction of the j+1 inner products (fixed order); folded by k_dots_finalize
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int l = 0; l <= MA_MMAX; ++l)
    if (l <= j) {
      double v = wave_sum((double)dots[l]);
      if (lane == 0) red[wid * (MA_MMAX + 1) + l] = v;
    }
  __syncthreads();
  if (threadIdx.x <= j) {
    double t = 0.0;
    for (int w = 0; w < BLOCK / 64; ++w) t += red[w * (MA_MMAX + 1) + threadIdx.x];
    d.part[(long)blockIdx.x * (MA_MMAX + 1) + threadIdx.x] = t;
  }
}

// h[l][j] = <w, v_l> for l <= j from the pass-C partials (one block per pair).
// Lane l of group g sums blocks g, g + 8, ...; the loads are independent.
__global__ __launch_bounds__(256) void k_dots_finalize(LaunchCtx c, int j, int nblk) {
  const int p = pair_of_block(c);
  const PairDesc& d = c.desc[p];
  PairState& s = c.st[p];
  if (!(s.phase == PH_SOLVE && s.gm_running)) return;
  __shared__ double red[8][32];
  const int l = threadIdx.x & 31, grp = threadIdx.x >> 5;
  double t = 0.0;
  if (l <= j) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int b = grp;
    for (; b + 24 < nblk; b += 32) {
      a0 += d.part[(long)b * (MA_MMAX + 1) + l];
      a1 += d.part[(long)(b + 8) * (MA_MMAX + 1) + l];
      a2 += d.part[(long)(b + 16) * (MA_MMAX + 1) + l];
      a3 += d.part[(long)(b + 24) * (MA_MMAX + 1) + l];
    }
    for (; b < nblk; b += 8) a0 += d.part[(long)b * (MA_MMAX + 1) + l];
    t = (a0 + a1) + (a2 + a3);
  }
  red[grp][l] = t;
  __syncthreads();
  if (threadIdx.x <= j) {
    double u = 0.0;
    for (int g2 = 0; g2 < 8; ++g2) u += red[g2][threadIdx.x];
    s.Hm[j * (MA_MMAX + 1) + threadIdx.x] = u * s.vscale[threadIdx.x];
  }
}

// ||w'|| from the pass-A partials, then the rotations and the convergence test
__global__ __launch_bounds__(256) void k_arnoldi_finalize(LaunchCtx c, int jn, int nblk) {
  const int p = pair_of_block(c);
  const PairDesc& d = c.desc[p];
  PairState& s = c.st[p];
  if (!(s.phase == PH_SOLVE && s.gm_running)) return;
  __shared__ double scratch[4];
  const int kinds[1] = {0};
  double t[1];
  fold_partials<1>(d.part, nblk, kinds, t, scratch);
  if (threadIdx.x == 0) arnoldi_close(s, c, jn, t[0]);
}

// a restarted cycle begins: its first vector has been transformed by pass A
__global__ void k_cycle_begin(LaunchCtx c) {
  const int p = pair_of_block(c);
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
  const PairDesc& d = c.desc[p];
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

}  // namespace

#define MA_FOR_EACH_N(X) \
  X(16) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024) X(1536) X(2048)

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

int passA_blocks(int n) {
  switch (n) {
#define X(NV) case NV: return NV / 2 / Cfg<NV>::A_PPB;
    MA_FOR_EACH_N(X)
#undef X
    default: return 0;
  }
}

int passC_blocks(int n) {
  switch (n) {
#define X(NV) case NV: return NV / 2 / Cfg<NV>::C_PPB;
    MA_FOR_EACH_N(X)
#undef X
    default: return 0;
  }
}

void launch_passA(const LaunchCtx& c, int n, int npairs, int mode, int jn, const float2* tw, hipStream_t st,
                  const TimedLaunch& ev) {
  launch_passA_only(c, n, npairs, mode, jn, tw, st, ev);
  if (mode == PA_ARNOLDI)
    hipLaunchKernelGGL(k_arnoldi_finalize, dim3(1, npairs), dim3(256), 0, st, c, jn, passA_blocks(n));
  else if (mode == PA_PLAIN)
    hipLaunchKernelGGL(k_cycle_begin, dim3(1, npairs), dim3(64), 0, st, c);
}

void launch_passA_only(const LaunchCtx& c, int n, int npairs, int mode, int jn, const float2* tw, hipStream_t st,
                       const TimedLaunch& ev) {
  switch (n) {
#define X(NV)                                                                                  \
  case NV:                                                                                     \
    MA_LAUNCH(ev, k_passA<NV>, dim3(NV / 2 / Cfg<NV>::A_PPB, npairs), dim3(Cfg<NV>::A_BLOCK), st, c, \
              mode, jn, tw);                                                                   \
    break;
    MA_FOR_EACH_N(X)
#undef X
    default: break;
  }
}

void launch_passB(const LaunchCtx& c, int n, int npairs, int mode, int j, const float2* tw, hipStream_t st,
                  const TimedLaunch& ev) {
  switch (n) {
#define X(NV)                                                                                  \
  case NV:                                                                                     \
    MA_LAUNCH(ev, k_passB<NV>, dim3(NV / 2 / Cfg<NV>::B_CPB, npairs), dim3(Cfg<NV>::B_BLOCK), st, c, \
              mode, j, tw);                                                                    \
    break;
    MA_FOR_EACH_N(X)
#undef X
    default: break;
  }
}

void launch_passC(const LaunchCtx& c, int n, int npairs, int mode, int j, const float2* tw, hipStream_t st,
                  const TimedLaunch& ev) {
  launch_passC_only(c, n, npairs, mode, j, tw, st, ev);
  if (mode == PC_MATVEC)
    hipLaunchKernelGGL(k_dots_finalize, dim3(1, npairs), dim3(256), 0, st, c, j, passC_blocks(n));
}

void launch_passC_only(const LaunchCtx& c, int n, int npairs, int mode, int j, const float2* tw, hipStream_t st,
                       const TimedLaunch& ev) {
  switch (n) {
#define X(NV)                                                                                  \
  case NV:                                                                                     \
    MA_LAUNCH(ev, k_passC<NV>, dim3(NV / 2 / Cfg<NV>::C_PPB, npairs), dim3(Cfg<NV>::C_BLOCK), st, c, \
              mode, j, tw);                                                                    \
    break;
    MA_FOR_EACH_N(X)
#undef X
    default: break;
  }
}

void launch_restart(const LaunchCtx& c, int n, int npairs, hipStream_t st) {
  long b = (long)n * n / (MA_BLOCK * 4);
  const int nb = b < 1 ? 1 : (int)(b > 4096 ? 4096 : b);
  hipLaunchKernelGGL(k_restart, dim3(nb, npairs), dim3(MA_BLOCK), 0, st, c);
}
