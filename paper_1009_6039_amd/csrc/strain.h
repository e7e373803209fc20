// Strain's FFT operator (Section 4.2 of Saumier, Agueh, Khouider): the kernels of
// the three passes over the grid per operator application, templated on the grid
// size and a launch-geometry variant; instantiated by k_pass_a/b/c.hip:
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
#pragma once
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

// Launch geometry per grid size N and variant V (the autotuner's choices):
//   V = 0  the default: rows (pass A, C) or columns (pass B) per block as below,
//          about one radix-8 butterfly per thread
//   V = 1  half as many rows / columns per block (more, smaller blocks)
//   V = 2  twice as many (fewer, larger blocks; only if the LDS tile stays within 64 KiB)
//   V = 3  the default tile with half the threads (two butterflies per thread)
// A variant that does not change the geometry is reported as a duplicate of V = 0.
__host__ __device__ constexpr int vary_units(int base, int V, int limit, int bytes_per_unit) {
  return V == 1 ? (base >= 2 ? base / 2 : base)
                : (V == 2 ? ((limit % (2 * base) == 0 && 2 * base * bytes_per_unit <= 65536) ? 2 * base : base)
                          : base);
}
__host__ __device__ constexpr int vary_block(int block, int V) {
  return V == 3 ? (block / 2 >= 64 ? ((block / 2 + 63) / 64) * 64 : 64) : block;
}

template <int N, int V>
struct Cfg {
  static constexpr int NH = N / 2;
  static constexpr int A0 = pow2_div(1024 / N > 0 ? 1024 / N : 1, NH);  // default row pairs per block
  static constexpr int B0 = pow2_div(4096 / N > 0 ? 4096 / N : 1, NH);  // default columns per block
  static constexpr int C0 = pow2_div(512 / N > 0 ? 512 / N : 1, NH);    // default row pairs per block
  static constexpr int A_PPB = vary_units(A0, V, NH, 8 * N);
  static constexpr int A_BLOCK = vary_block(round_block(A_PPB * N / 8, V == 2 ? 512 : 256), V);
  static constexpr int B_CPB = vary_units(B0, V, NH, 16 * N);
  static constexpr int B_BLOCK = vary_block(round_block(B_CPB * N / 8, V == 2 ? 512 : 256), V);
  static constexpr int C_PPB = vary_units(C0, V, NH, 40 * N);
  static constexpr int C_BLOCK = vary_block(round_block(5 * C_PPB * N / 8, V == 2 ? 640 : 320), V);
  static_assert((N * B_CPB) % B_BLOCK == 0, "column pass: whole elements per thread");
  static_assert(B_BLOCK % B_CPB == 0, "column pass: fixed column per thread");
};

// the smallest variant index with the same geometry (duplicates share one kernel)
template <int N, int V>
struct Canon {
  static constexpr int A = (V > 0 && Cfg<N, V>::A_PPB == Cfg<N, 0>::A_PPB && Cfg<N, V>::A_BLOCK == Cfg<N, 0>::A_BLOCK) ? 0 : V;
  static constexpr int B = (V > 0 && Cfg<N, V>::B_CPB == Cfg<N, 0>::B_CPB && Cfg<N, V>::B_BLOCK == Cfg<N, 0>::B_BLOCK) ? 0 : V;
  static constexpr int C = (V > 0 && Cfg<N, V>::C_PPB == Cfg<N, 0>::C_PPB && Cfg<N, V>::C_BLOCK == Cfg<N, 0>::C_BLOCK) ? 0 : V;
};

// rhobar(k): inverse symbol of the averaged operator (Section 4.2), zero at k = 0.
// q: FFT index of k1; q2: FFT index of k2 (N/2 for the Nyquist column).
// mt[q] = (Im of the first-derivative multiplier, second-derivative multiplier).
template <int N>
__device__ __forceinline__ float2 rhobar_m(int q, int q2, float2 m1, float2 m2, const float (&ab)[5]) {
  if (q == 0 && q2 == 0) return make_float2(0.f, 0.f);
  // S = a11 d2(k1) + 2 a12 (i d1(k1))(i d1(k2)) + a22 d2(k2) + i (b1 d1(k1) + b2 d1(k2))
  const float re = ab[0] * m1.y + ab[2] * m2.y - 2.f * ab[1] * m1.x * m2.x;
  const float im = ab[3] * m1.x + ab[4] * m2.x;
  const float den = re * re + im * im;
  const float inv = 1.f / den;  // one division for both parts
  return make_float2(re * inv, -im * inv);
}
// the same with the multipliers read from the table mt
template <int N>
__device__ __forceinline__ float2 rhobar(int q, int q2, const float (&ab)[5], const float2* __restrict__ mt) {
  return rhobar_m<N>(q, q2, mt[q], mt[q2], ab);
}

// Z[k] = A + iB and Z[N-k] = conj(A) + i conj(B): the full spectrum of the complex
// signal whose real / imaginary parts have half spectra A / B
template <int N>
__device__ __forceinline__ void put_pair(float2* L, int k, float2 A, float2 B) {
  L[k] = make_float2(A.x - B.y, A.y + B.x);
  L[N - k] = make_float2(A.x + B.y, B.x - A.y);
}
__device__ __forceinline__ float2 times_i(float s, float2 a) { return make_float2(-s * a.y, s * a.x); }

// h_l = <w, v_l>, l < nv, from pass C's block partials (nblk blocks of MA_MMAX + 1
// slots), in an order that does not depend on the block size: item (l, g), g < 32, sums
// blocks g, g + 32, ... (strided_sum<4>); the 32 items of one l sit in one half of a
// wave and are added by DPP prefix sums within rows of 16 and the two row totals.  The
// block size is a multiple of 64.  out (LDS) receives h_l; ends with a barrier.
__device__ __forceinline__ void fold_inner_products(const double* part, int nblk, int nv, double* out) {
  const int lane = threadIdx.x & 63;
  for (int base = 0; base < 32 * nv; base += blockDim.x) {  // the same trip count in every thread
    const int t = base + threadIdx.x, l = t >> 5, g = t & 31;
    double x = l < nv ? strided_sum<4>(part, MA_MMAX + 1, l, g, 32, nblk) : 0.0;
    x += row_shr<1>(x);
    x += row_shr<2>(x);
    x += row_shr<4>(x);
    x += row_shr<8>(x);
    const double h0 = read_lane(x, 15) + read_lane(x, 31), h1 = read_lane(x, 47) + read_lane(x, 63);
    const int l0 = (base + (threadIdx.x & ~63)) >> 5;  // the wave's first l
    if (lane == 0 && l0 < nv) out[l0] = h0;
    if (lane == 0 && l0 + 1 < nv) out[l0 + 1] = h1;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// pass A
// ---------------------------------------------------------------------------
// PL: the radix plan of the transforms (fft.h)
template <int N, int G, int PL = 0>
__global__ __launch_bounds__((Cfg<N, G>::A_BLOCK)) void k_passA(LaunchCtx c, int mode, int jn,
                                                           const float2* __restrict__ tw) {
  constexpr int PPB = Cfg<N, G>::A_PPB, BLOCK = Cfg<N, G>::A_BLOCK, NH = N / 2;
  constexpr long NN = (long)N * N;
  const int p = pair_of_block(c);
  if (p < 0) return;
  const PairDesc d = c.desc[p];
  const PairState& s = c.st[p];
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
  if (mode == PA_ARNOLDI && c.dots_nblk > 0) {
    // the column h[.][jn - 1] of the Hessenberg matrix from pass C's partials (every
    // block folds them the same way; block 0 records the column)
    __shared__ double hl[MA_MMAX + 1];
    fold_inner_products(d.part, c.dots_nblk, nv, hl);
    if (threadIdx.x < nv) {
      const int l = threadIdx.x;
      const double h = hl[l] * s.vscale[l];
      cf[l] = (float)(h * s.vscale[l]);
      if (blockIdx.x == 0) c.st[p].Hm[(jn - 1) * (MA_MMAX + 1) + l] = h;
    }
  } else if (threadIdx.x < nv) {
    const int l = threadIdx.x;
    cf[l] = mode == PA_ARNOLDI ? (float)(s.Hm[(jn - 1) * (MA_MMAX + 1) + l] * s.vscale[l]) : (float)s.y[l];
  }
  const float cst = (float)s.mass_c, inv_tau = (float)(1.0 / s.tau);
  // left scaling of the GMRES system (option): h / D with D = (a11 + a22) / (abar11 + abar22)
  const bool scaled = mode == PA_INIT && c.precond == MA_PRECOND_DIAG;
  const float trbar = (float)(s.abar[0] + s.abar[2]);
  {  // algorithmic bytes per point: vectors read, Krylov vector written, half spectrum written
    const bool fft = !(mode == PA_ARNOLDI && jn >= c.m);
    double b = fft ? 4.0 : 0.0;
    if (mode == PA_INIT) b += scaled ? 16.0 : 8.0;
    else if (mode == PA_PLAIN || mode == PA_STEP) b += 4.0;
    else if (mode == PA_ARNOLDI) b += 4.0 * (jn + 1) + 4.0;
    else b += 4.0 * (nv + (usex ? 1 : 0));
    count_bytes(c, b, N);
  }
  __syncthreads();

  const int row0 = 2 * blockIdx.x * PPB;
  const auto V = gmem<float>(d.V);
  const auto Vj = V + (long)jn * NN;
  const auto R = gmem<const float>(d.r);
  const auto coef = gmem<const float>(d.coef);
  const auto X = gmem<const float>(d.x);
  // The thread's points first (their values in registers), then the Krylov vectors
  // one at a time with all of the thread's loads of that vector in flight together,
  // and those of the next vector issued before the current one is used.
  constexpr int PER = (PPB * N + BLOCK - 1) / BLOCK;
  constexpr bool FULL = (PPB * N) % BLOCK == 0;
  float va[PER], vb[PER];
  int ea_[PER];  // offset of the first row's point (n * n < 2^31); a point past the end
                 // reads the block's first point (in bounds) and is never stored
  float nrm = 0.f;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = threadIdx.x + q * BLOCK;
    va[q] = vb[q] = 0.f;
    ea_[q] = row0 * N;
    if (!FULL && e >= PPB * N) continue;
    const int pp = e / N, jj = e % N;
    const int ea = (row0 + 2 * pp) * N + jj, eb = ea + N;
    ea_[q] = ea;
    if (mode == PA_INIT) {
      va[q] = (R[ea] + cst) * inv_tau;
      vb[q] = (R[eb] + cst) * inv_tau;
      if (scaled) {
        va[q] *= trbar / (coef[ea] + coef[2 * NN + ea]);
        vb[q] *= trbar / (coef[eb] + coef[2 * NN + eb]);
      }
    } else if (mode == PA_PLAIN || mode == PA_STEP) {
      va[q] = V[ea];
      vb[q] = V[eb];
    } else if (mode == PA_ARNOLDI) {
      va[q] = Vj[ea];
      vb[q] = Vj[eb];
    } else {  // PA_RECOVER
      va[q] = usex ? X[ea] : 0.f;
      vb[q] = usex ? X[eb] : 0.f;
    }
  }
  if (mode == PA_ARNOLDI || mode == PA_RECOVER) {
    // v -= sum_l c_l V_l (Arnoldi) or x += sum_l y_l V_l (recovery), l in order
    const float sg = mode == PA_ARNOLDI ? -1.f : 1.f;
    stream_vectors<2 * PER>(
        nv,
        [&](int l, float* x) {
          const auto Vl = V + (long)l * NN;
#pragma unroll
          for (int q = 0; q < PER; ++q) {
            x[q] = Vl[ea_[q]];
            x[PER + q] = Vl[ea_[q] + N];
          }
        },
        [&](int l, const float* x) {
          const float cl = sg * cf[l];
#pragma unroll
          for (int q = 0; q < PER; ++q) {
            va[q] += cl * x[q];
            vb[q] += cl * x[PER + q];
          }
        });
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = threadIdx.x + q * BLOCK;
    if (!FULL && e >= PPB * N) continue;
    const int pp = e / N, jj = e % N;
    const int ea = ea_[q], eb = ea + N;
    if (mode == PA_INIT) {
      if (scaled) nrm += va[q] * va[q] + vb[q] * vb[q];
      V[ea] = va[q];
      V[eb] = vb[q];
    } else if (mode == PA_ARNOLDI) {
      Vj[ea] = va[q];
      Vj[eb] = vb[q];
      nrm += va[q] * va[q] + vb[q] * vb[q];
    }
    lds[pp * N + jj] = make_float2(va[q], vb[q]);
  }

  if (!(mode == PA_ARNOLDI && jn >= c.m)) {
    __syncthreads();
    fft_lds<N, PPB, BLOCK, false, LAYOUT_ROWS, PL>(lds, tw);
    const auto H = gmem<float2>(d.H);
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
      H[ia] = oa;
      H[ib] = ob;
    }
  }

  if (mode == PA_ARNOLDI || scaled) {  // partial ||w'||^2 (or ||h / D||^2), folded per pair
    double v[1] = {(double)nrm};
    const int kinds[1] = {0};
    block_reduce<1>(v, kinds, scratch);
    // after pass C's partials when pass A folds those itself
    const long off = mode == PA_ARNOLDI ? (long)c.dots_nblk * (MA_MMAX + 1) : 0;
    if (threadIdx.x == 0) d.part[off + blockIdx.x] = v[0];
  }
}

// ---------------------------------------------------------------------------
// pass B (columns)
// ---------------------------------------------------------------------------
template <int N, int G, int PL = 0>
__global__ __launch_bounds__((Cfg<N, G>::B_BLOCK)) void k_passB(LaunchCtx c, int mode, int j,
                                                           const float2* __restrict__ tw) {
  constexpr int CPB = Cfg<N, G>::B_CPB, BLOCK = Cfg<N, G>::B_BLOCK, NH = N / 2;
  const int p = pair_of_block(c);
  if (p < 0) return;
  const PairDesc d = c.desc[p];
  const PairState& s = c.st[p];
  bool run;
  if (mode == PB_MATVEC) run = s.phase == PH_SOLVE && s.gm_running;
  else if (mode == PB_RECOVER) run = s.phase == PH_SOLVE;
  else run = true;
  if (!run) return;
  count_bytes(c, mode == PB_MATVEC ? 16.0 : 8.0, N);  // half spectrum in, one or three out

  // S: the column spectra, then rhobar * sigmahat, then each output spectrum in turn.
  // Element (row or wavenumber e, column cc) sits at e * CPB + cc.
  __shared__ float2 S[N * CPB];
  constexpr int PT = PL | TW_FULL;  // the transforms read every twiddle power from twl
  __shared__ float2 twl[tw_span(N, PT)];
  const int s0 = blockIdx.x * CPB;
  const auto H = gmem<const float2>(d.H);
  const auto T = gmem<float2>(d.T);
  // With one first-stage butterfly per thread, the thread's elements (rows e / CPB
  // for e = threadIdx.x + q BLOCK of column threadIdx.x % CPB) are that butterfly's
  // inputs: every transform starts from registers (one LDS pass and two barriers
  // fewer each); other geometries stage everything through LDS.
  constexpr int R0 = pick_radix(N, PL);
  constexpr bool REG1 = BLOCK == CPB * (N / R0);
  // the multipliers the thread uses below, loaded with its columns (so that no wait on
  // a table load stalls the transforms): at the wavenumbers q and N - q of its rhobar
  // items, at its column's wavenumber, and at the rows of its elements
  constexpr int NI = ((NH + 1) * CPB + BLOCK - 1) / BLOCK;  // rhobar items per thread
  constexpr int PER = N * CPB / BLOCK;                      // elements per thread (whole)
  float2 mq[NI], mqm[NI], mo[PER];
  const int cc0 = threadIdx.x % CPB;  // the thread's column (BLOCK is a multiple of CPB)
  float2 mslot, m0, mnh;
  // the scale and the averaged coefficients, read with the loads below (the scale's
  // load is unconditional so that no branch waits on it before the column loads)
  const double vsj = s.vscale[mode == PB_MATVEC ? j : 0];
  float ab[5];
  for (int k = 0; k < 5; ++k) ab[k] = (float)s.abar[k];
  {  // every column load of the thread in flight before the first LDS write; the
     // twiddles first, so that their copy into LDS waits for them alone
    TwiddleStage<N, BLOCK, PT> tws;
    tws.load(tw);
    float2 h[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = threadIdx.x + q * BLOCK;
      h[q] = H[(long)(e / CPB) * NH + s0 + e % CPB];
    }
#pragma unroll
    for (int r = 0; r < NI; ++r) {
      const int it = threadIdx.x + r * BLOCK;
      const int q = it < (NH + 1) * CPB ? it / CPB : 0;
      mq[r] = c.mt[q];
      mqm[r] = c.mt[(N - q) % N];
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) mo[k] = c.mt[(threadIdx.x + k * BLOCK) / CPB];
    mslot = c.mt[s0 + cc0];
    m0 = c.mt[0];
    mnh = c.mt[NH];
    tws.store(twl);
    if constexpr (REG1) {
      fft_cols_from_regs<N, CPB, BLOCK, false, PT>(S, twl, h);
    } else {
#pragma unroll
      for (int q = 0; q < PER; ++q) S[threadIdx.x + q * BLOCK] = h[q];
      __syncthreads();
      fft_lds<N, CPB, BLOCK, false, LAYOUT_COLS, PT>(S, twl);
    }
  }
  const float scale = (float)((mode == PB_MATVEC ? vsj : 1.0) / ((double)N * (double)N));
  if (mode == PB_FORWARD) {
    for (int e = threadIdx.x; e < N * CPB; e += BLOCK) {
      const int i = e / CPB, cc = e % CPB;
      T[(long)i * NH + s0 + cc] = S[e];
    }
    return;
  }
  // wavenumbers q and N - q together: slot 0 packs the DC and Nyquist columns of the
  // rows, which separate with the partner coefficient; every later multiplier m(q)
  // then acts on the packed value P = sA + i sB directly
#pragma unroll
  for (int r = 0; r < NI; ++r) {
    const int it = threadIdx.x + r * BLOCK;
    if (it >= (NH + 1) * CPB) break;
    const int q = it / CPB, cc = cc0;
    const int qm = (N - q) % N;
    const int slot = s0 + cc;
    const float2 z = S[q * CPB + cc], zm = S[qm * CPB + cc];
    float2 vq, vm;
    if (slot != 0) {
      vq = cscale(cmul(rhobar_m<N>(q, slot, mq[r], mslot, ab), z), scale);
      vm = cscale(cmul(rhobar_m<N>(qm, slot, mqm[r], mslot, ab), zm), scale);
    } else {
      const float2 A = make_float2(0.5f * (z.x + zm.x), 0.5f * (z.y - zm.y));
      const float2 B = make_float2(0.5f * (z.y + zm.y), -0.5f * (z.x - zm.x));
      const float2 aq = cmul(rhobar_m<N>(q, 0, mq[r], m0, ab), A), bq = cmul(rhobar_m<N>(q, NH, mq[r], mnh, ab), B);
      const float2 am = cmul(rhobar_m<N>(qm, 0, mqm[r], m0, ab), cconj(A));
      const float2 bm = cmul(rhobar_m<N>(qm, NH, mqm[r], mnh, ab), cconj(B));
      vq = cscale(make_float2(aq.x - bq.y, aq.y + bq.x), scale);
      vm = cscale(make_float2(am.x - bm.y, am.y + bm.x), scale);
    }
    S[q * CPB + cc] = vq;
    if (qm != q) S[qm * CPB + cc] = vm;
  }
  __syncthreads();
  // derived spectra 2 pi i k1 and -(2 pi k1)^2 (matvec only), then the plain one.  The
  // multiplied spectrum stays in registers (each thread's own elements), and every
  // output is written back into S from them and transformed in place: one LDS buffer
  // per block instead of two, so twice the blocks fit on a CU.
  float2 sv[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) sv[k] = S[threadIdx.x + k * BLOCK];
  // the register path writes elements other threads are still reading here
  if constexpr (REG1) __syncthreads();
  const int nout = mode == PB_MATVEC ? 3 : 1;
  for (int oo = 0; oo < nout; ++oo) {
    const int o = (oo + 1) % 3 == 0 || nout == 1 ? 0 : oo + 1;  // order 1, 2, 0
    // the last radix stage stores its outputs (row e of column t) straight to memory
    const auto To = T + (long)o * N * NH + s0;
    auto store = [&](int t, int e, float2 v) { To[(long)e * NH + t] = v; };
    if constexpr (REG1) {
      float2 x[PER];
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const float2 m = mo[k];
        x[k] = o == 0 ? sv[k] : ((o == 1) ? times_i(m.x, sv[k]) : cscale(sv[k], m.y));
      }
      fft_cols_from_regs_out<N, CPB, BLOCK, true, PT>(S, twl, x, store);
    } else {
      if (oo > 0 || o != 0) {  // S still holds the plain spectrum for a lone output 0
#pragma unroll
        for (int k = 0; k < PER; ++k) {
          const int e = threadIdx.x + k * BLOCK;
          const float2 m = mo[k];
          S[e] = o == 0 ? sv[k] : ((o == 1) ? times_i(m.x, sv[k]) : cscale(sv[k], m.y));
        }
        __syncthreads();
      }
      fft_stages_out<N, 1, CPB, BLOCK, true, LAYOUT_COLS, PT>(S, twl, store);
    }
    __syncthreads();  // the last stage has read S before the next output overwrites it
  }
}

// The coefficients at the thread's points of the block's row pairs (all loads issued
// together, with no branch) and the points' offsets; a point past the end takes the
// block's first point (in bounds) and is never used.
template <int N, int PPB, int BLOCK>
struct PassCCoef {
  static constexpr int PER = (PPB * N + BLOCK - 1) / BLOCK;
  float ca[PER][5], cb[PER][5];
  int ea[PER];
};
template <int N, int PPB, int BLOCK>
__device__ __forceinline__ void passC_load_coef(const PairDesc& d, int row0, PassCCoef<N, PPB, BLOCK>& k5) {
  constexpr long NN = (long)N * N;
  constexpr int PER = PassCCoef<N, PPB, BLOCK>::PER;
  constexpr bool FULL = (PPB * N) % BLOCK == 0;
  const auto coef = gmem<const float>(d.coef);
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = threadIdx.x + q * BLOCK;
    const bool in = FULL || e < PPB * N;
    const int pp = in ? e / N : 0, jj = in ? e % N : 0;
    k5.ea[q] = (row0 + 2 * pp) * N + jj;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      k5.ca[q][k] = coef[k * NN + k5.ea[q]];
      k5.cb[q][k] = coef[k * NN + k5.ea[q] + N];
    }
  }
}

// Pass C's epilogue: w = a11 alpha11 + 2 a12 alpha12 + a22 alpha22 + b1 beta1 + b2 beta2 at
// the block's points (left-scaled if the option is on), stored as V[j+1], and the
// block's partial inner products <w, v_l>, l <= j, which the next pass A folds.  zat(pp, t, jj)
// is element jj of derived transform t of the block's row pair pp: t = 0 alpha11 + i
// beta1 of row a, 1 alpha12 + i beta2 of row a, 2 and 3 the same for row b, 4 alpha22 of
// row a (.x) and row b (.y).  The caller synchronises the block before the call.
// k5: the coefficients at the thread's points (passC_load_coef); trbar = abar11 + abar22.
// d is the caller's register copy of the pair's descriptor, so that no pointer is
// reloaded from memory after the block barriers.
template <int N, int PPB, int BLOCK, class ZAT>
__device__ __forceinline__ void passC_combine(const LaunchCtx& c, const PairDesc& d, float trbar, int j,
                                              int row0, double* red, ZAT zat,
                                              const PassCCoef<N, PPB, BLOCK>& k5) {
  constexpr long NN = (long)N * N;
  const auto V = gmem<float>(d.V);
  const auto W = V + (long)(j + 1) * NN;
  const bool scaled = c.precond == MA_PRECOND_DIAG;
  // w at the thread's points, then the inner products <w, v_l>
  constexpr int PER = PassCCoef<N, PPB, BLOCK>::PER;
  constexpr bool FULL = (PPB * N) % BLOCK == 0;
  float wa[PER], wb[PER];
  const auto& ca = k5.ca;
  const auto& cb = k5.cb;
  const auto& ea_ = k5.ea;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = threadIdx.x + q * BLOCK;
    wa[q] = wb[q] = 0.f;
    if (!FULL && e >= PPB * N) continue;
    const int pp = e / N, jj = e % N;
    const int ea = ea_[q], eb = ea + N;
    const float2 z0 = zat(pp, 0, jj), z1 = zat(pp, 1, jj), z2 = zat(pp, 2, jj), z3 = zat(pp, 3, jj),
                 z4 = zat(pp, 4, jj);
    float a = ca[q][0] * z0.x + 2.f * ca[q][1] * z1.x + ca[q][2] * z4.x + ca[q][3] * z0.y + ca[q][4] * z1.y;
    float b = cb[q][0] * z2.x + 2.f * cb[q][1] * z3.x + cb[q][2] * z4.y + cb[q][3] * z2.y + cb[q][4] * z3.y;
    if (scaled) {  // left scaling by 1 / D(x), D = (a11 + a22) / (abar11 + abar22)
      a *= trbar / (ca[q][0] + ca[q][2]);
      b *= trbar / (cb[q][0] + cb[q][2]);
    }
    W[ea] = a;
    W[eb] = b;
    wa[q] = a;
    wb[q] = b;
  }
  // block reduction of the j+1 inner products (fixed order); folded by the next pass A
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  stream_vectors<2 * PER>(
      j + 1,
      [&](int l, float* x) {
        const auto Vl = V + (long)l * NN;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
          x[q] = Vl[ea_[q]];
          x[PER + q] = Vl[ea_[q] + N];
        }
      },
      [&](int l, const float* x) {
        float acc = 0.f;
#pragma unroll
        for (int q = 0; q < PER; ++q) acc += wa[q] * x[q] + wb[q] * x[PER + q];
        const double v = wave_sum((double)acc);
        if (lane == 0) red[wid * (MA_MMAX + 1) + l] = v;
      });
  __syncthreads();
  if (threadIdx.x <= j) {
    double t = 0.0;
    for (int w = 0; w < BLOCK / 64; ++w) t += red[w * (MA_MMAX + 1) + threadIdx.x];
    d.part[(long)blockIdx.x * (MA_MMAX + 1) + threadIdx.x] = t;
  }
}

// ---------------------------------------------------------------------------
// pass C (rows)
// ---------------------------------------------------------------------------
// PF: the coefficients of the combination are loaded right after the spectra, before
// the transforms, and the transforms read their twiddles from an LDS copy (so that no
// vector-memory wait inside them holds the coefficient loads back)
template <int N, int G, bool PF = false, int PL = 0>
__global__ __launch_bounds__((Cfg<N, G>::C_BLOCK)) void k_passC(LaunchCtx c, int mode, int j,
                                                           const float2* __restrict__ tw) {
  constexpr int PPB = Cfg<N, G>::C_PPB, BLOCK = Cfg<N, G>::C_BLOCK, NH = N / 2;
  constexpr long NN = (long)N * N;
  const int p = pair_of_block(c);
  if (p < 0) return;
  const PairDesc d = c.desc[p];
  const PairState& s = c.st[p];
  const bool run = mode == PC_MATVEC ? (s.phase == PH_SOLVE && s.gm_running) : (s.phase == PH_SOLVE);
  if (!run) return;
  const float trbar = (float)(s.abar[0] + s.abar[2]);

  // three half spectra 12, coefficients 20, Krylov vectors for the dots, w 4 (matvec);
  // one half spectrum 4, theta 8, u read and written 16 (recovery)
  count_bytes(c, mode == PC_MATVEC ? 36.0 + 4.0 * (j + 1) : (mode == PC_RECOVER ? 28.0 : 8.0), N);
  __shared__ float2 lds[5 * PPB * N];
  __shared__ double red[(BLOCK / 64) * (MA_MMAX + 1)];
  const int row0 = 2 * blockIdx.x * PPB;
  const auto T0 = gmem<const float2>(d.T);
  const auto T1 = T0 + NN / 2;
  const auto T2 = T0 + NN;

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
    fft_lds<N, PPB, BLOCK, true, LAYOUT_ROWS, PL>(lds, tw);
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

  // five complex inverse transforms per row pair; every spectrum load of the thread
  // is issued before the first LDS write
  constexpr int PT = PF ? (PL | TW_FULL) : PL;  // with the LDS copy, every twiddle power from it
  __shared__ float2 twl[PF ? tw_span(N, PT) : 1];
  TwiddleStage<N, BLOCK, PT> tws;
  if constexpr (PF) tws.load(tw);
  constexpr int IT1 = (PPB * NH + BLOCK - 1) / BLOCK;
  constexpr bool FULL1 = (PPB * NH) % BLOCK == 0;
  float2 tl[IT1][7];  // three spectra of each row, the multipliers at k
  const float d2n = c.mt[NH].y;
#pragma unroll
  for (int q = 0; q < IT1; ++q) {
    const int e = threadIdx.x + q * BLOCK;
    if (!FULL1 && e >= PPB * NH) continue;
    const int pp = e / NH, k = e % NH;
    const long ia = (long)(row0 + 2 * pp) * NH + k, ib = ia + NH;
    tl[q][6] = c.mt[k];
    tl[q][0] = T0[ia];
    tl[q][1] = T1[ia];
    tl[q][2] = T2[ia];
    tl[q][3] = T0[ib];
    tl[q][4] = T1[ib];
    tl[q][5] = T2[ib];
  }
  PassCCoef<N, PPB, BLOCK> pre;
  if constexpr (PF) {
    passC_load_coef<N, PPB, BLOCK>(d, row0, pre);
    tws.store(twl);
  }
#pragma unroll
  for (int q = 0; q < IT1; ++q) {
    const int e = threadIdx.x + q * BLOCK;
    if (!FULL1 && e >= PPB * NH) continue;
    const int pp = e / NH, k = e % NH;
    const float2 t0a = tl[q][0], t1a = tl[q][1], t2a = tl[q][2];
    const float2 t0b = tl[q][3], t1b = tl[q][4], t2b = tl[q][5];
    float2* L = lds + 5 * pp * N;
    if (k == 0) {
      // DC (.x) and Nyquist (.y) are real; the first-derivative multiplier vanishes at
      // both, the second-derivative one at DC
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
      const float2 m = tl[q][6];
      put_pair<N>(L, k, t2a, t1a);
      put_pair<N>(L + N, k, times_i(m.x, t1a), times_i(m.x, t0a));
      put_pair<N>(L + 2 * N, k, t2b, t1b);
      put_pair<N>(L + 3 * N, k, times_i(m.x, t1b), times_i(m.x, t0b));
      put_pair<N>(L + 4 * N, k, cscale(t0a, m.y), cscale(t0b, m.y));
    }
  }
  __syncthreads();
  fft_lds<N, 5 * PPB, BLOCK, true, LAYOUT_ROWS, PT>(lds, PF ? twl : tw);
  // the coefficients at all of the thread's points are loaded before the first is used
  if constexpr (!PF) passC_load_coef<N, PPB, BLOCK>(d, row0, pre);
  passC_combine<N, PPB, BLOCK>(c, d, trbar, j, row0, red,
                               [&](int pp, int t, int jj) { return lds[(5 * pp + t) * N + jj]; }, pre);
}

// Pass C with wave-owned transforms: 5 PPB waves per block, wave (pp, t) builds derived
// transform t of row pair pp straight from the column pass's spectra and inverts it in
// its private LDS region; one block barrier before the pointwise combination.  The
// recovery modes use wave (pp, 0) only.
template <int N, int PPB>
__global__ __launch_bounds__(320 * PPB) void k_passC_w(LaunchCtx c, int mode, int j, const float2* tw) {
  constexpr int NH = N / 2, WB = WaveBuf<N>::size, BLOCK = 320 * PPB;
  constexpr long NN = (long)N * N;
  const int p = pair_of_block(c);
  if (p < 0) return;
  const PairDesc d = c.desc[p];
  const PairState& s = c.st[p];
  const bool run = mode == PC_MATVEC ? (s.phase == PH_SOLVE && s.gm_running) : (s.phase == PH_SOLVE);
  if (!run) return;
  const float trbar = (float)(s.abar[0] + s.abar[2]);
  count_bytes(c, mode == PC_MATVEC ? 36.0 + 4.0 * (j + 1) : (mode == PC_RECOVER ? 28.0 : 8.0), N);
  __shared__ float2 lds[5 * PPB * WB];
  __shared__ double red[(BLOCK / 64) * (MA_MMAX + 1)];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int pp = wv / 5, t = wv % 5;
  const int row0 = 2 * blockIdx.x * PPB;
  float2* L = lds + wv * WB;
  const auto T0 = gmem<const float2>(d.T);
  const auto T1 = T0 + NN / 2;
  const auto T2 = T0 + NN;
  const long ra = (long)(row0 + 2 * pp) * NH;  // half-spectrum row a of this row pair; row b follows

  if (mode != PC_MATVEC) {
    if (t != 0) return;
    // theta = Lbar^{-1} sigma: rows a and b as the real and imaginary parts of one transform
    for (int k = lane; k < NH; k += 64) {
      const float2 a = T0[ra + k], b = T0[ra + NH + k];
      if (k == 0) {
        L[wpad(0)] = make_float2(a.x, b.x);
        L[wpad(NH)] = make_float2(a.y, b.y);
      } else {
        L[wpad(k)] = make_float2(a.x - b.y, a.y + b.x);
        L[wpad(N - k)] = make_float2(a.x + b.y, b.x - a.y);
      }
    }
    wave_sync();
    wfft<N, true>(L, tw, lane);
    for (int jj = lane; jj < N; jj += 64) {
      const long ea = (long)(row0 + 2 * pp) * N + jj, eb = ea + N;
      const float2 z = L[wpad(jj)];
      if (mode == PC_RECOVER) {  // FP64 correction kept for step halving; u in FP64
        d.theta[ea] = (double)z.x;
        d.theta[eb] = (double)z.y;
        d.u[ea] += (double)z.x;
        d.u[eb] += (double)z.y;
      } else {
        d.x[ea] = z.x;
        d.x[eb] = z.y;
      }
    }
    return;
  }

  // derived transform t of this row pair: every spectrum load of the lane first
  constexpr int IT = (NH + 63) / 64;
  float2 A[IT], B[IT];
#pragma unroll
  for (int q = 0; q < IT; ++q) {
    const int k = lane + 64 * q;
    if (NH % 64 != 0 && k >= NH) continue;
    const long ia = ra + k, ib = ia + NH;
    if (t == 0) { A[q] = T2[ia]; B[q] = T1[ia]; }
    else if (t == 1) { A[q] = T1[ia]; B[q] = T0[ia]; }
    else if (t == 2) { A[q] = T2[ib]; B[q] = T1[ib]; }
    else if (t == 3) { A[q] = T1[ib]; B[q] = T0[ib]; }
    else { A[q] = T0[ia]; B[q] = T0[ib]; }
  }
#pragma unroll
  for (int q = 0; q < IT; ++q) {
    const int k = lane + 64 * q;
    if (NH % 64 != 0 && k >= NH) continue;
    if (k == 0) {
      // DC (.x) and Nyquist (.y) are real; the first-derivative multiplier vanishes at
      // both, the second-derivative one at DC
      if (t == 0 || t == 2) {
        L[wpad(0)] = make_float2(A[q].x, B[q].x);
        L[wpad(NH)] = make_float2(A[q].y, B[q].y);
      } else if (t == 4) {
        const float d2n = c.mt[NH].y;
        L[wpad(0)] = make_float2(0.f, 0.f);
        L[wpad(NH)] = make_float2(d2n * A[q].y, d2n * B[q].y);
      } else {
        L[wpad(0)] = make_float2(0.f, 0.f);
        L[wpad(NH)] = make_float2(0.f, 0.f);
      }
    } else {
      const float2 m = c.mt[k];
      float2 a = A[q], b = B[q];
      if (t == 1 || t == 3) {
        a = times_i(m.x, a);
        b = times_i(m.x, b);
      } else if (t == 4) {
        a = cscale(a, m.y);
        b = cscale(b, m.y);
      }
      L[wpad(k)] = make_float2(a.x - b.y, a.y + b.x);
      L[wpad(N - k)] = make_float2(a.x + b.y, b.x - a.y);
    }
  }
  wave_sync();
  wfft<N, true>(L, tw, lane);
  __syncthreads();
  PassCCoef<N, PPB, BLOCK> k5;
  passC_load_coef<N, PPB, BLOCK>(d, row0, k5);
  passC_combine<N, PPB, BLOCK>(c, d, trbar, j, row0, red,
                               [&](int q, int tt, int jj) { return lds[(5 * q + tt) * WB + wpad(jj)]; }, k5);
}

// region stride of a block's wave-owned transforms: at least the padded length, and
// 8 modulo 32 elements, so that the transposing accesses of eight regions at once
// spread over the LDS banks
template <int N>
struct WaveRegion {
  static constexpr int size = WaveBuf<N>::size + ((8 - WaveBuf<N>::size % 32) + 32) % 32;
};

// Pass B with wave-owned columns: a block of W waves takes W adjacent half-spectrum
// columns; rows are read with coalesced loads and transposed into the waves' regions
// (one block barrier), then each wave runs its column's forward transform, the
// multiplication by rhobar and the inverse transforms in its own region with wave-level
// synchronisation only; each output is stored with coalesced row writes (two block
// barriers around the transposing read).
template <int N, int W>
__global__ __launch_bounds__(64 * W) void k_passB_w(LaunchCtx c, int mode, int j, const float2* tw) {
  constexpr int NH = N / 2, RS = WaveRegion<N>::size, BLOCK = 64 * W;
  constexpr int ROWS = BLOCK / W;      // rows per cooperative pass (64)
  constexpr int PER = N / ROWS;        // cooperative passes over the rows
  constexpr int OWN = (N + 63) / 64;   // elements per lane of a column
  const int p = pair_of_block(c);
  if (p < 0) return;
  const PairDesc d = c.desc[p];
  const PairState& s = c.st[p];
  bool run;
  if (mode == PB_MATVEC) run = s.phase == PH_SOLVE && s.gm_running;
  else if (mode == PB_RECOVER) run = s.phase == PH_SOLVE;
  else run = true;
  if (!run) return;
  count_bytes(c, mode == PB_MATVEC ? 16.0 : 8.0, N);
  __shared__ float2 lds[W * RS];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tc = threadIdx.x % W, tr = threadIdx.x / W;  // cooperative role: column, first row
  const int s0 = blockIdx.x * W;
  float2* L = lds + wv * RS;  // this wave's column: slot s0 + wv
  const auto H = gmem<const float2>(d.H);
  const auto T = gmem<float2>(d.T);
  {  // rows in, transposed into the regions
    float2 h[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) h[q] = H[(long)(tr + ROWS * q) * NH + s0 + tc];
#pragma unroll
    for (int q = 0; q < PER; ++q) lds[tc * RS + wpad(tr + ROWS * q)] = h[q];
  }
  __syncthreads();
  wfft<N, false>(L, tw, lane);
  auto store = [&](int o) {  // the regions' columns out as rows of T_o
    __syncthreads();
    const auto To = T + (long)o * N * NH;
#pragma unroll
    for (int q = 0; q < PER; ++q) To[(long)(tr + ROWS * q) * NH + s0 + tc] = lds[tc * RS + wpad(tr + ROWS * q)];
    __syncthreads();
  };
  if (mode == PB_FORWARD) {
    store(0);
    return;
  }
  const float scale = (float)((mode == PB_MATVEC ? s.vscale[j] : 1.0) / ((double)N * (double)N));
  float ab[5];
  for (int k = 0; k < 5; ++k) ab[k] = (float)s.abar[k];
  const int slot = s0 + wv;
  // wavenumbers q and N - q together (slot 0 packs the DC and Nyquist columns of the rows)
  for (int q = lane; q <= NH; q += 64) {
    const int qm = (N - q) % N;
    const float2 z = L[wpad(q)], zm = L[wpad(qm)];
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
    L[wpad(q)] = vq;
    if (qm != q) L[wpad(qm)] = vm;
  }
  wave_sync();
  // the multiplied spectrum stays in registers (the lane's elements e = lane + 64 r)
  float2 sv[OWN];
#pragma unroll
  for (int r = 0; r < OWN; ++r) {
    const int e = lane + 64 * r;
    sv[r] = (N % 64 == 0 || e < N) ? L[wpad(e)] : make_float2(0.f, 0.f);
  }
  const int nout = mode == PB_MATVEC ? 3 : 1;
  for (int oo = 0; oo < nout; ++oo) {
    const int o = (oo + 1) % 3 == 0 || nout == 1 ? 0 : oo + 1;  // order 1, 2, 0
    wave_sync();
#pragma unroll
    for (int r = 0; r < OWN; ++r) {
      const int e = lane + 64 * r;
      if (N % 64 != 0 && e >= N) continue;
      const float2 m = c.mt[e];
      L[wpad(e)] = o == 0 ? sv[r] : ((o == 1) ? times_i(m.x, sv[r]) : cscale(sv[r], m.y));
    }
    wave_sync();
    wfft<N, true>(L, tw, lane);
    store(o);
  }
}

// Pass A with wave-owned row pairs: a block of W waves, wave w builds the Krylov vector
// on row pair w of the block (lane l takes the columns l, l + 64, ...), packs the two
// rows as one complex row in its region, transforms it and writes the two half
// spectra; the only block barrier is the final reduction of ||w'||^2.
template <int N, int W>
__global__ __launch_bounds__(64 * W) void k_passA_w(LaunchCtx c, int mode, int jn, const float2* tw) {
  constexpr int NH = N / 2, WB = WaveBuf<N>::size, BLOCK = 64 * W;
  constexpr long NN = (long)N * N;
  constexpr int OWN = (N + 63) / 64;
  const int p = pair_of_block(c);
  if (p < 0) return;
  const PairDesc d = c.desc[p];
  const PairState& s = c.st[p];
  bool run;
  if (mode == PA_INIT) run = s.phase == PH_SOLVE && s.gm_running && s.gm_cycle == 0;
  else if (mode == PA_PLAIN) run = s.phase == PH_SOLVE && s.gm_restart;
  else if (mode == PA_ARNOLDI) run = s.phase == PH_SOLVE && s.gm_running;
  else if (mode == PA_RECOVER) run = s.phase == PH_SOLVE;
  else run = true;
  if (!run) return;
  __shared__ float2 lds[W * WB];
  __shared__ float cf[MA_MMAX + 1];
  __shared__ double scratch[BLOCK / 64];
  int nv = 0;
  bool usex = false;
  if (mode == PA_ARNOLDI) nv = jn;
  else if (mode == PA_RECOVER) { nv = s.gm_k; usex = s.gm_cycle > 0; }
  if (mode == PA_ARNOLDI && c.dots_nblk > 0) {
    // the column h[.][jn - 1] of the Hessenberg matrix from pass C's partials (every
    // block folds them the same way; block 0 records the column)
    __shared__ double hl[MA_MMAX + 1];
    fold_inner_products(d.part, c.dots_nblk, nv, hl);
    if (threadIdx.x < nv) {
      const int l = threadIdx.x;
      const double h = hl[l] * s.vscale[l];
      cf[l] = (float)(h * s.vscale[l]);
      if (blockIdx.x == 0) c.st[p].Hm[(jn - 1) * (MA_MMAX + 1) + l] = h;
    }
  } else if (threadIdx.x < nv) {
    const int l = threadIdx.x;
    cf[l] = mode == PA_ARNOLDI ? (float)(s.Hm[(jn - 1) * (MA_MMAX + 1) + l] * s.vscale[l]) : (float)s.y[l];
  }
  const float cst = (float)s.mass_c, inv_tau = (float)(1.0 / s.tau);
  const bool scaled = mode == PA_INIT && c.precond == MA_PRECOND_DIAG;
  const float trbar = (float)(s.abar[0] + s.abar[2]);
  {
    const bool fft = !(mode == PA_ARNOLDI && jn >= c.m);
    double b = fft ? 4.0 : 0.0;
    if (mode == PA_INIT) b += scaled ? 16.0 : 8.0;
    else if (mode == PA_PLAIN || mode == PA_STEP) b += 4.0;
    else if (mode == PA_ARNOLDI) b += 4.0 * (jn + 1) + 4.0;
    else b += 4.0 * (nv + (usex ? 1 : 0));
    count_bytes(c, b, N);
  }
  __syncthreads();  // cf
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float2* L = lds + wv * WB;
  const int ra = 2 * (blockIdx.x * W + wv);  // the wave's row pair
  const auto V = gmem<float>(d.V);
  const auto Vj = V + (long)jn * NN;
  const auto R = gmem<const float>(d.r);
  const auto coef = gmem<const float>(d.coef);
  const auto X = gmem<const float>(d.x);
  float va[OWN], vb[OWN];
  int ea_[OWN];
  float nrm = 0.f;
#pragma unroll
  for (int q = 0; q < OWN; ++q) {
    const int jj = lane + 64 * q;
    va[q] = vb[q] = 0.f;
    ea_[q] = ra * N;
    if (N % 64 != 0 && jj >= N) continue;
    const int ea = ra * N + jj, eb = ea + N;
    ea_[q] = ea;
    if (mode == PA_INIT) {
      va[q] = (R[ea] + cst) * inv_tau;
      vb[q] = (R[eb] + cst) * inv_tau;
      if (scaled) {
        va[q] *= trbar / (coef[ea] + coef[2 * NN + ea]);
        vb[q] *= trbar / (coef[eb] + coef[2 * NN + eb]);
      }
    } else if (mode == PA_PLAIN || mode == PA_STEP) {
      va[q] = V[ea];
      vb[q] = V[eb];
    } else if (mode == PA_ARNOLDI) {
      va[q] = Vj[ea];
      vb[q] = Vj[eb];
    } else {
      va[q] = usex ? X[ea] : 0.f;
      vb[q] = usex ? X[eb] : 0.f;
    }
  }
  if (mode == PA_ARNOLDI || mode == PA_RECOVER) {
    // v -= sum_l c_l V_l (Arnoldi) or x += sum_l y_l V_l (recovery), l in order
    const float sg = mode == PA_ARNOLDI ? -1.f : 1.f;
    stream_vectors<2 * OWN>(
        nv,
        [&](int l, float* x) {
          const auto Vl = V + (long)l * NN;
#pragma unroll
          for (int q = 0; q < OWN; ++q) {
            x[q] = Vl[ea_[q]];
            x[OWN + q] = Vl[ea_[q] + N];
          }
        },
        [&](int l, const float* x) {
          const float cl = sg * cf[l];
#pragma unroll
          for (int q = 0; q < OWN; ++q) {
            va[q] += cl * x[q];
            vb[q] += cl * x[OWN + q];
          }
        });
  }
#pragma unroll
  for (int q = 0; q < OWN; ++q) {
    const int jj = lane + 64 * q;
    if (N % 64 != 0 && jj >= N) continue;
    const int ea = ea_[q], eb = ea + N;
    if (mode == PA_INIT) {
      if (scaled) nrm += va[q] * va[q] + vb[q] * vb[q];
      V[ea] = va[q];
      V[eb] = vb[q];
    } else if (mode == PA_ARNOLDI) {
      Vj[ea] = va[q];
      Vj[eb] = vb[q];
      nrm += va[q] * va[q] + vb[q] * vb[q];
    }
    L[wpad(jj)] = make_float2(va[q], vb[q]);
  }
  if (!(mode == PA_ARNOLDI && jn >= c.m)) {
    wave_sync();
    wfft<N, false>(L, tw, lane);
    const auto Hs = gmem<float2>(d.H);
    for (int k = lane; k < NH; k += 64) {
      const long ia = (long)ra * NH + k, ib = ia + NH;
      const float2 zk = L[wpad(k)];
      float2 oa, ob;
      if (k == 0) {
        const float2 zn = L[wpad(NH)];
        oa = make_float2(zk.x, zn.x);
        ob = make_float2(zk.y, zn.y);
      } else {
        const float2 zm = L[wpad(N - k)];
        oa = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
        ob = make_float2(0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x));
      }
      Hs[ia] = oa;
      Hs[ib] = ob;
    }
  }
  if (mode == PA_ARNOLDI || scaled) {  // partial ||w'||^2 (or ||h / D||^2), folded per pair
    double v[1] = {(double)nrm};
    const int kinds[1] = {0};
    block_reduce<1>(v, kinds, scratch);
    // after pass C's partials when pass A folds those itself
    const long off = mode == PA_ARNOLDI ? (long)c.dots_nblk * (MA_MMAX + 1) : 0;
    if (threadIdx.x == 0) d.part[off + blockIdx.x] = v[0];
  }
}

}  // namespace

#define MA_FOR_EACH_N(X) \
  X(16) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024) X(1536) X(2048)
// the sizes with wave-owned variants
#define MA_FOR_EACH_N_WAVE(X) X(128) X(192) X(256) X(384) X(512) X(768) X(1024) X(1536) X(2048)
