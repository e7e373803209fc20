// Mixed-radix (2, 3, 4, 8, 16) self-sorting Stockham FFT on data resident in LDS.
//
// A block runs NF independent length-N complex transforms that sit in LDS.
// LAYOUT_ROWS:  element e of transform t at lds[t * N + e]   (row FFTs)
// LAYOUT_COLS:  element e of transform t at lds[e * NF + t]  (column FFTs; the
//               transform index varies fastest so neighbouring lanes hit
//               neighbouring LDS words)
// Stage with radix R after sub-length Ns (Ns = product of earlier radices): the
// butterfly j reads x[j + r N/R], r < R, multiplies by w^(r (j mod Ns)) with
// w = exp(-+2 pi i / (Ns R)), runs a length-R DFT and writes
// x[(j / Ns) Ns R + (j mod Ns) + r Ns].  The output is in natural order.
// Twiddles come from a table tw[m] = exp(-2 pi i m / N) built on the host in FP64.
// The radix sequence (the plan) is a compile-time choice: plan 0 takes a factor 3
// first, then eights; plan 1 fours; plan 2 sixteens where they save a stage.
#pragma once
#include <hip/hip_runtime.h>

enum { LAYOUT_ROWS = 0, LAYOUT_COLS = 1 };

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 rot90(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

template <bool INV>
__device__ __forceinline__ void dft2(float2& a, float2& b) {
  float2 t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <bool INV>
__device__ __forceinline__ void dft3(float2& a, float2& b, float2& c) {
  const float s3 = 0.86602540378443864676f;  // sin(pi/3)
  float2 t1 = cadd(b, c);
  float2 t2 = make_float2(a.x - 0.5f * t1.x, a.y - 0.5f * t1.y);
  float2 d = csub(b, c);
  // (b - c) * (-+ i sqrt(3)/2)
  float2 t3 = rot90<INV>(make_float2(d.x * s3, d.y * s3));
  a = cadd(a, t1);
  b = cadd(t2, t3);
  c = csub(t2, t3);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2& v0, float2& v1, float2& v2, float2& v3) {
  float2 t0 = cadd(v0, v2), t1 = csub(v0, v2);
  float2 t2 = cadd(v1, v3), t3 = rot90<INV>(csub(v1, v3));
  v0 = cadd(t0, t2);
  v2 = csub(t0, t2);
  v1 = cadd(t1, t3);
  v3 = csub(t1, t3);
}

template <bool INV>
__device__ __forceinline__ void dft8(float2 (&v)[8]) {
  const float r2 = 0.70710678118654752440f;
  float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<INV>(e0, e1, e2, e3);
  dft4<INV>(o0, o1, o2, o3);
  // o_k *= w8^k, w8 = exp(-+ 2 pi i / 8)
  o1 = INV ? make_float2(r2 * (o1.x - o1.y), r2 * (o1.x + o1.y))
           : make_float2(r2 * (o1.x + o1.y), r2 * (o1.y - o1.x));
  o2 = rot90<INV>(o2);
  o3 = INV ? make_float2(-r2 * (o3.x + o3.y), r2 * (o3.x - o3.y))
           : make_float2(r2 * (o3.y - o3.x), -r2 * (o3.x + o3.y));
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, o1);
  v[5] = csub(e1, o1);
  v[2] = cadd(e2, o2);
  v[6] = csub(e2, o2);
  v[3] = cadd(e3, o3);
  v[7] = csub(e3, o3);
}

// x * exp(-+ 2 pi i m / 16) for a fixed m in 1..9 (cos and sin of multiples of pi / 8)
template <int M, bool INV>
__device__ __forceinline__ float2 w16(float2 a) {
  constexpr float c1 = 0.92387953251128675613f, s1 = 0.38268343236508977173f, r2 = 0.70710678118654752440f;
  constexpr float cr = M == 1 ? c1 : M == 2 ? r2 : M == 3 ? s1 : M == 4 ? 0.f : M == 6 ? -r2 : -c1;
  constexpr float si = M == 1 ? s1 : M == 2 ? r2 : M == 3 ? c1 : M == 4 ? 1.f : M == 6 ? r2 : -s1;
  static_assert(M == 1 || M == 2 || M == 3 || M == 4 || M == 6 || M == 9, "twiddle index");
  // w = cr - +i si (forward: minus)
  const float sg = INV ? si : -si;
  return make_float2(a.x * cr - a.y * sg, a.x * sg + a.y * cr);
}

// 16-point DFT as 4 x 4: element 4 n1 + n2; length-4 transforms over n1, the twiddles
// w16^(n2 k1), length-4 transforms over n2; output k1 + 4 k2 in natural order
template <bool INV>
__device__ __forceinline__ void dft16(float2 (&v)[16]) {
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) dft4<INV>(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
  // v[4 k1 + n2] now holds y[n2][k1]
  v[5] = w16<1, INV>(v[5]);
  v[9] = w16<2, INV>(v[9]);
  v[13] = w16<3, INV>(v[13]);
  v[6] = w16<2, INV>(v[6]);
  v[10] = w16<4, INV>(v[10]);
  v[14] = w16<6, INV>(v[14]);
  v[7] = w16<3, INV>(v[7]);
  v[11] = w16<6, INV>(v[11]);
  v[15] = w16<9, INV>(v[15]);
  float2 o[16];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    float2 a = v[4 * k1], b = v[4 * k1 + 1], c = v[4 * k1 + 2], d = v[4 * k1 + 3];
    dft4<INV>(a, b, c, d);
    o[k1] = a;
    o[k1 + 4] = b;
    o[k1 + 8] = c;
    o[k1 + 12] = d;
  }
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = o[k];
}

template <int R, bool INV>
__device__ __forceinline__ void dft(float2 (&v)[R]) {
  if constexpr (R == 2) dft2<INV>(v[0], v[1]);
  else if constexpr (R == 3) dft3<INV>(v[0], v[1], v[2]);
  else if constexpr (R == 4) dft4<INV>(v[0], v[1], v[2], v[3]);
  else if constexpr (R == 8) dft8<INV>(v);
  else dft16<INV>(v);
}

// radix used for the remaining length REM under a plan.  Plan 0: a factor 3 first,
// then eights, with sixteen split as 4 x 4 and leftovers as 4 or 2.  Plan 1: a factor 3
// first, then fours, with a last eight or two.  Plan 2: a factor 3 first, then sixteens
// (thirty-two as 8 x 4), then 8, 4 or 2.
// Flag of a plan argument: the stages read every twiddle power w^r, r < R, from the
// table (an LDS copy, so the extra reads cost no memory traffic) instead of forming the
// higher powers as products of two or three table values, which saves their complex
// multiplications.  The radix sequence is the plan's.
constexpr int TW_FULL = 4;

__host__ __device__ constexpr int pick_radix(int rem, int plan = 0) {
  plan &= 3;
  if (rem % 3 == 0) return 3;
  if (plan == 1) return rem == 8 ? 8 : (rem % 4 == 0 ? 4 : 2);
  if (plan == 2 && rem % 16 == 0 && rem != 32) return 16;
  return rem == 16 ? 4 : (rem % 8 == 0 ? 8 : (rem % 4 == 0 ? 4 : 2));
}

// whether a plan's radix sequence for length n differs from plan 0's
__host__ __device__ constexpr bool plan_differs(int n, int plan) {
  int ns = 1;
  while (ns < n) {
    const int r = pick_radix(n / ns, plan);
    if (r != pick_radix(n / ns, 0)) return true;
    ns *= r;
  }
  return false;
}

// One more than the largest twiddle-table index a length-N transform reads: a stage
// of radix R after sub-length NS > 1 reads tw[m k TWS], k < NS, TWS = N / (NS R), with
// m up to 8 (R = 16), 4 (R = 8), 2 (R = 4, 3) or 1 (R = 2), or up to R - 1 under
// TW_FULL.
__host__ __device__ constexpr int tw_span(int n, int plan = 0) {
  int need = 1, ns = 1;
  while (ns < n) {
    const int r = pick_radix(n / ns, plan);
    if (ns > 1) {
      const int top = (plan & TW_FULL) ? r - 1 : (r == 16 ? 8 : (r == 8 ? 4 : (r == 2 ? 1 : 2)));
      const int idx = top * (ns - 1) * (n / (ns * r)) + 1;
      need = need > idx ? need : idx;
    }
    ns *= r;
  }
  return need;
}

// The part of the twiddle table that a length-N transform reads, copied into LDS so
// that the stages read twiddles without vector-memory loads (whose in-order counter
// would also hold every other load in flight).  load() issues the thread's share of
// the table into registers; a caller that issues it before its data loads can store()
// the copy while those are still in flight.  The caller's barrier before its first
// transform makes the copy visible.
template <int N, int BLOCK, int PLAN = 0>
struct TwiddleStage {
  static constexpr int SPAN = tw_span(N, PLAN);
  static constexpr int IT = (SPAN + BLOCK - 1) / BLOCK;
  float2 v[IT];
  __device__ __forceinline__ void load(const float2* __restrict__ tw) {
#pragma unroll
    for (int q = 0; q < IT; ++q) {
      const int e = threadIdx.x + q * BLOCK;
      if (SPAN % BLOCK == 0 || e < SPAN) v[q] = tw[e];
    }
  }
  __device__ __forceinline__ void store(float2* twl) const {
#pragma unroll
    for (int q = 0; q < IT; ++q) {
      const int e = threadIdx.x + q * BLOCK;
      if (SPAN % BLOCK == 0 || e < SPAN) twl[e] = v[q];
    }
  }
};
template <int N, int BLOCK, int PLAN = 0>
__device__ __forceinline__ void stage_twiddles(float2* twl, const float2* __restrict__ tw) {
  TwiddleStage<N, BLOCK, PLAN> t;
  t.load(tw);
  t.store(twl);
}

template <int N, int NF, int LAYOUT>
__device__ __forceinline__ int lds_index(int t, int e) {
  if constexpr (LAYOUT == LAYOUT_ROWS) return t * N + e;
  else return e * NF + t;
}

// w[r] = tw[r k TWS] for 0 < r < R.  FULL: every power read from the table; otherwise
// from at most three table entries (k r < NS R, so indices stay below N), products of
// two table values keeping the error within a few ulp.
template <int R, bool FULL>
__device__ __forceinline__ void stage_powers(const float2* __restrict__ tw, int k, int TWS, float2 (&w)[R]) {
  if constexpr (FULL) {
#pragma unroll
    for (int r = 1; r < R; ++r) w[r] = tw[r * k * TWS];
  } else {
    w[1] = tw[k * TWS];
    if constexpr (R >= 3) w[2] = tw[2 * k * TWS];
    if constexpr (R == 4) w[3] = cmul(w[1], w[2]);
    if constexpr (R >= 8) {
      w[4] = tw[4 * k * TWS];
      w[3] = cmul(w[1], w[2]);
      w[5] = cmul(w[4], w[1]);
      w[6] = cmul(w[4], w[2]);
      w[7] = cmul(w[4], w[3]);
    }
    if constexpr (R == 16) {  // w^8 from the table, the rest as w^8 w^(r - 8)
      w[8] = tw[8 * k * TWS];
#pragma unroll
      for (int r = 9; r < 16; ++r) w[r] = cmul(w[8], w[r - 8]);
    }
  }
}

template <int N, int NS, int R, int NF, int BLOCK, bool INV, int LAYOUT, bool FULL = false>
__device__ __forceinline__ void fft_stage(float2* lds, const float2* __restrict__ tw) {
  constexpr int NB = N / R;                  // butterflies per transform
  constexpr int ITEMS = NF * NB;
  constexpr int PER = (ITEMS + BLOCK - 1) / BLOCK;
  constexpr int TWS = N / (NS * R);          // twiddle stride in the length-N table
  float2 v[PER][R];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int it = threadIdx.x + q * BLOCK;
    if (ITEMS % BLOCK == 0 || it < ITEMS) {
      int t, j;
      if constexpr (LAYOUT == LAYOUT_ROWS) { t = it / NB; j = it % NB; }
      else { t = it % NF; j = it / NF; }
      const int k = j % NS;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = lds[lds_index<N, NF, LAYOUT>(t, j + r * NB)];
      if (NS > 1) {
        float2 w[R];
        stage_powers<R, FULL>(tw, k, TWS, w);
#pragma unroll
        for (int r = 1; r < R; ++r) v[q][r] = cmul(v[q][r], INV ? cconj(w[r]) : w[r]);
      }
      dft<R, INV>(v[q]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int it = threadIdx.x + q * BLOCK;
    if (ITEMS % BLOCK == 0 || it < ITEMS) {
      int t, j;
      if constexpr (LAYOUT == LAYOUT_ROWS) { t = it / NB; j = it % NB; }
      else { t = it % NF; j = it / NF; }
      const int k = j % NS;
      const int base = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) lds[lds_index<N, NF, LAYOUT>(t, base + r * NS)] = v[q][r];
    }
  }
  __syncthreads();
}

template <int N, int NS, int NF, int BLOCK, bool INV, int LAYOUT, int PLAN = 0>
__device__ __forceinline__ void fft_stages(float2* lds, const float2* __restrict__ tw) {
  if constexpr (NS < N) {
    constexpr int R = pick_radix(N / NS, PLAN);
    fft_stage<N, NS, R, NF, BLOCK, INV, LAYOUT, (PLAN & TW_FULL) != 0>(lds, tw);
    fft_stages<N, NS * R, NF, BLOCK, INV, LAYOUT, PLAN>(lds, tw);
  }
}

// The last stage of a transform (NS R = N) handing its outputs to out(t, e, value),
// element e of sequence t, instead of writing them back to LDS: the caller's stores go
// straight to memory.  It reads LDS and ends without a barrier, so the caller
// synchronises before anything writes `lds` again.
template <int N, int NS, int R, int NF, int BLOCK, bool INV, int LAYOUT, bool FULL, class OUT>
__device__ __forceinline__ void fft_stage_out(const float2* lds, const float2* __restrict__ tw, OUT out) {
  static_assert(NS * R == N, "the last stage");
  constexpr int NB = N / R;
  constexpr int ITEMS = NF * NB;
  constexpr int PER = (ITEMS + BLOCK - 1) / BLOCK;
  constexpr int TWS = N / (NS * R);
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int it = threadIdx.x + q * BLOCK;
    if (ITEMS % BLOCK == 0 || it < ITEMS) {
      int t, j;
      if constexpr (LAYOUT == LAYOUT_ROWS) { t = it / NB; j = it % NB; }
      else { t = it % NF; j = it / NF; }
      const int k = j % NS;  // = j: the last stage has NB = NS butterflies per sequence
      float2 v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = lds[lds_index<N, NF, LAYOUT>(t, j + r * NB)];
      if (NS > 1) {
        float2 w[R];
        stage_powers<R, FULL>(tw, k, TWS, w);
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = cmul(v[r], INV ? cconj(w[r]) : w[r]);
      }
      dft<R, INV>(v);
#pragma unroll
      for (int r = 0; r < R; ++r) out(t, k + r * NS, v[r]);
    }
  }
}

// All stages in LDS but the last, which hands its outputs to out (fft_stage_out)
template <int N, int NS, int NF, int BLOCK, bool INV, int LAYOUT, int PLAN, class OUT>
__device__ __forceinline__ void fft_stages_out(float2* lds, const float2* __restrict__ tw, OUT out) {
  constexpr int R = pick_radix(N / NS, PLAN);
  if constexpr (NS * R < N) {
    fft_stage<N, NS, R, NF, BLOCK, INV, LAYOUT, (PLAN & TW_FULL) != 0>(lds, tw);
    fft_stages_out<N, NS * R, NF, BLOCK, INV, LAYOUT, PLAN>(lds, tw, out);
  } else {
    fft_stage_out<N, NS, R, NF, BLOCK, INV, LAYOUT, (PLAN & TW_FULL) != 0>(lds, tw, out);
  }
}

// Column transforms whose first stage starts from registers.  Valid when every thread
// runs exactly one butterfly of the first stage (BLOCK = NF * N / R0, R0 the first
// radix) and holds its inputs: x[r] = element j + r N/R0 of column t, with
// t = threadIdx.x % NF and j = threadIdx.x / NF (the element order e * NF + t read
// with stride BLOCK).  The first stage has no twiddles; its outputs go to LDS in the
// Stockham order and the later stages run in LDS as in fft_lds.  The caller makes
// sure no thread still reads `lds` before the call; the routine ends with a barrier.
template <int N, int NF, int BLOCK, bool INV, int PLAN = 0>
__device__ __forceinline__ void fft_cols_from_regs(float2* lds, const float2* __restrict__ tw,
                                                   float2 (&x)[pick_radix(N, PLAN)]) {
  constexpr int R0 = pick_radix(N, PLAN);
  static_assert(BLOCK == NF * (N / R0), "one first-stage butterfly per thread");
  const int t = threadIdx.x % NF, j = threadIdx.x / NF;
  dft<R0, INV>(x);
#pragma unroll
  for (int r = 0; r < R0; ++r) lds[lds_index<N, NF, LAYOUT_COLS>(t, j * R0 + r)] = x[r];
  __syncthreads();
  fft_stages<N, R0, NF, BLOCK, INV, LAYOUT_COLS, PLAN>(lds, tw);
}

// fft_cols_from_regs whose last stage hands its outputs to out(t, e, value) (see
// fft_stage_out); ends without a barrier.
template <int N, int NF, int BLOCK, bool INV, int PLAN, class OUT>
__device__ __forceinline__ void fft_cols_from_regs_out(float2* lds, const float2* __restrict__ tw,
                                                       float2 (&x)[pick_radix(N, PLAN)], OUT out) {
  constexpr int R0 = pick_radix(N, PLAN);
  static_assert(BLOCK == NF * (N / R0), "one first-stage butterfly per thread");
  const int t = threadIdx.x % NF, j = threadIdx.x / NF;
  dft<R0, INV>(x);
  if constexpr (R0 == N) {  // a single stage: the outputs are the thread's registers
#pragma unroll
    for (int r = 0; r < R0; ++r) out(t, r, x[r]);
  } else {
#pragma unroll
    for (int r = 0; r < R0; ++r) lds[lds_index<N, NF, LAYOUT_COLS>(t, j * R0 + r)] = x[r];
    __syncthreads();
    fft_stages_out<N, R0, NF, BLOCK, INV, LAYOUT_COLS, PLAN>(lds, tw, out);
  }
}

// In-place transforms of NF sequences in LDS.  Caller synchronises before (data
// written) — the routine ends with a barrier so results are visible on return.
template <int N, int NF, int BLOCK, bool INV, int LAYOUT, int PLAN = 0>
__device__ __forceinline__ void fft_lds(float2* lds, const float2* __restrict__ tw) {
  fft_stages<N, 1, NF, BLOCK, INV, LAYOUT, PLAN>(lds, tw);
}

// ---------------------------------------------------------------------------
// Transforms owned by one wavefront.  The sequence sits in an LDS region private to
// the wave, element e at wpad(e) = e + e / 8 (one pad word pair after every eight
// elements: the strided writes of a radix-8 stage then spread over the banks), and a
// stage synchronises only its own wave: a wave's LDS operations execute in order, so a
// compiler barrier between a stage's writes and the next stage's reads is enough.
// Lane l runs butterflies l, l + 64, ... of each stage (any N; lanes idle where a
// stage has fewer than 64 butterflies).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wpad(int e) { return e + (e >> 3); }
template <int N>
struct WaveBuf {
  static constexpr int size = N + N / 8;
};
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int N, int NS, int R, bool INV>
__device__ __forceinline__ void wfft_stage(float2* L, const float2* __restrict__ tw, int lane) {
  constexpr int NB = N / R;
  constexpr int PER = (NB + 63) / 64;
  constexpr int TWS = N / (NS * R);
  float2 v[PER][R];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int j = lane + 64 * q;
    if (NB % 64 == 0 || j < NB) {
      const int k = j % NS;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = L[wpad(j + r * NB)];
      if (NS > 1) {
        float2 w[R];
        w[1] = tw[k * TWS];
        if constexpr (R >= 3) w[2] = tw[2 * k * TWS];
        if constexpr (R == 4) w[3] = cmul(w[1], w[2]);
        if constexpr (R == 8) {
          w[4] = tw[4 * k * TWS];
          w[3] = cmul(w[1], w[2]);
          w[5] = cmul(w[4], w[1]);
          w[6] = cmul(w[4], w[2]);
          w[7] = cmul(w[4], w[3]);
        }
#pragma unroll
        for (int r = 1; r < R; ++r) v[q][r] = cmul(v[q][r], INV ? cconj(w[r]) : w[r]);
      }
      dft<R, INV>(v[q]);
    }
  }
  wave_sync();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int j = lane + 64 * q;
    if (NB % 64 == 0 || j < NB) {
      const int k = j % NS;
      const int base = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) L[wpad(base + r * NS)] = v[q][r];
    }
  }
  wave_sync();
}

template <int N, int NS, bool INV>
__device__ __forceinline__ void wfft_stages(float2* L, const float2* __restrict__ tw, int lane) {
  if constexpr (NS < N) {
    constexpr int R = pick_radix(N / NS);
    wfft_stage<N, NS, R, INV>(L, tw, lane);
    wfft_stages<N, NS * R, INV>(L, tw, lane);
  }
}

// In-place transform of the wave's sequence (written by the wave before the call);
// ends synchronised, the result in natural order at wpad(e).
template <int N, bool INV>
__device__ __forceinline__ void wfft(float2* L, const float2* __restrict__ tw, int lane) {
  wfft_stages<N, 1, INV>(L, tw, lane);
}
