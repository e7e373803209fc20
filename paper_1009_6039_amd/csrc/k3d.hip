// The damped Newton method in three dimensions (the method is stated for any dimension
// d; Section 4.2 counts d(d+1) inverse transforms per product): the set-up, the FP64
// residual and coefficient kernel, Strain's operator as five line-transform passes, the
// Arnoldi steps and their per-pair folds.
//
// Operator passes for a product w = L Lbar^{-1} v (complex FP32 spectra, full length):
//   P1  along x3 (contiguous): v (real) -> forward transform -> S
//   P2  along x2: S -> forward transform -> S (in place)
//   P3  along x1: S -> forward transform, times rhobar(k) (Section 4.2) and the Krylov
//       scale / N^3, then inverse transforms of Z, i k1 Z and -k1^2 Z -> T0, T1, T2
//   P4  along x2: inverse transforms of T2, T1, i k2 T1, T0, i k2 T0, -k2^2 T0 -> U_a..U_f
//   P5  along x3: the nine real results alpha_ab, beta_a as five complex inverse
//       transforms (two real signals per transform: X + iY -> x + iy), the combination
//       w = sum a_aa alpha_aa + 2 sum a_ab alpha_ab + sum b_a beta_a, the inner products
//       <w, V_l> (partial sums per block)
// For theta = Lbar^{-1} x only Z -> T0 -> U_d -> theta is formed.
#include "common.h"
#include "fft.h"
#include "k3d.h"

namespace {

constexpr int LINES_ELEMS = 2048;  // complex elements per block in the x3 passes (16 KB of LDS)
constexpr int COLS = 16;           // lines per block in the x1 / x2 passes (128-byte row segments)

// the largest power of two <= max(1, lim): lines per block of the x3 passes, a divisor of
// N^2 (N is a multiple of 16), so that the blocks cover every line exactly once
__host__ __device__ constexpr int pow2_floor(int lim) {
  int p = 1;
  while (2 * p <= lim) p *= 2;
  return p;
}
template <int N>
struct Lines3 {
  static constexpr int P1 = pow2_floor(LINES_ELEMS / N);        // P1: one transform per line
  static constexpr int P5 = pow2_floor((LINES_ELEMS / 2) / N);  // P5: five transforms per line
  static_assert((N * N) % P1 == 0 && (N * N) % P5 == 0, "whole lines per block");
};

__device__ __forceinline__ int wrap3(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// periodic index of an integer-valued double (|f| < 2^50), in [0, n)
__device__ __forceinline__ int wrapf(double f, int n, double invn) {
  int a = (int)(f - (double)n * floor(f * invn));
  return a < 0 ? a + n : (a >= n ? a - n : a);
}

// ---------------------------------------------------------------------------
// set-up: means of f and g, then the scaled fields and the gradient of g
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(MA3_BLOCK) void k3_sums(Desc3 d) {
  const long nn = (long)d.n * d.n * d.n;
  double v[4] = {0.0, 0.0, 1e300, 0.0};
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (long)gridDim.x * blockDim.x) {
    const double a = d.f_in[e], b = d.g_in[e];
    v[0] += a;
    v[1] += b;
    v[2] = fmin(v[2], fmin(a, b));
    v[3] += (isfinite(a) && isfinite(b)) ? 0.0 : 1.0;
  }
  __shared__ double scratch[4 * 4];
  const int kinds[4] = {0, 0, 1, 0};
  block_reduce<4>(v, kinds, scratch);
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) d.part[(long)blockIdx.x * 4 + k] = v[k];
}

__global__ __launch_bounds__(256) void k3_sums_fold(Desc3 d, State3* s, int nblk) {
  __shared__ double scratch[4 * 4];
  const int kinds[4] = {0, 0, 1, 0};
  double t[4];
  fold_partials<4>(d.part, nblk, kinds, t, scratch);
  if (threadIdx.x == 0) {
    const double nn = (double)d.n * d.n * d.n;
    s->mean_f = t[0] / nn;
    s->mean_g = t[1] / nn;
    s->sums[0] = t[2];  // smallest density value (positive required)
    s->sums[1] = t[3];  // non-finite values
  }
}

__global__ __launch_bounds__(MA3_BLOCK) void k3_fields(Desc3 d, const State3* s) {
  const int n = d.n;
  const long nn = (long)n * n * n;
  const double ig = 1.0 / s->mean_g, i12h = (double)n / 12.0;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e / ((long)n * n)), j = (int)((e / n) % n), k = (int)(e % n);
    auto G = [&](int a, int b, int c) { return d.g_in[((long)wrap3(a, n) * n + wrap3(b, n)) * n + wrap3(c, n)]; };
    const double g1 = (G(i - 2, j, k) - 8.0 * G(i - 1, j, k) + 8.0 * G(i + 1, j, k) - G(i + 2, j, k)) * i12h * ig;
    const double g2 = (G(i, j - 2, k) - 8.0 * G(i, j - 1, k) + 8.0 * G(i, j + 1, k) - G(i, j + 2, k)) * i12h * ig;
    const double g3 = (G(i, j, k - 2) - 8.0 * G(i, j, k - 1) + 8.0 * G(i, j, k + 1) - G(i, j, k + 2)) * i12h * ig;
    d.gg[e] = make_float4((float)g1, (float)g2, (float)g3, 0.f);
    d.g[e] = d.g_in[e] * ig;
    d.f[e] = d.f_in[e] / s->mean_f;
    d.u[e] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// residual and coefficients (eq. ma2, eq. linearmaeq in 3-D; Section 4)
// ---------------------------------------------------------------------------

// The residual and coefficients at point (i, j, k) (ei its offset) from u at offsets
// |a|, |b|, |c| <= 2 (U(a, b, c)), accumulated into the block's partials
template <class UF>
__device__ __forceinline__ void res_point(const Desc3& d, int op_mode, int i, int j, int k, int ei, UF&& U,
                                          double (&acc)[MA3_NPART]) {
  const int n = d.n;
  const long nn = (long)n * n * n;
  const double N = (double)n, invn = 1.0 / N, h1 = N, h2 = N * N;
  const double u0 = U(0, 0, 0);
  // first and second derivatives along each axis, fourth order
  double g[3], s2[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int di = a == 0, dj = a == 1, dk = a == 2;
    const double m2 = U(-2 * di, -2 * dj, -2 * dk), m1 = U(-di, -dj, -dk);
    const double p1 = U(di, dj, dk), p2 = U(2 * di, 2 * dj, 2 * dk);
    g[a] = (m2 - 8.0 * m1 + 8.0 * p1 - p2) * (h1 / 12.0);
    s2[a] = (-m2 + 16.0 * m1 - 30.0 * u0 + 16.0 * p1 - p2) * (h2 / 12.0);
  }
  // mixed derivatives: the first-derivative formula along a applied to the one along b
  // (the sixteen values of each loaded before the first is used)
  constexpr double w1[4] = {1.0 / 12.0, -8.0 / 12.0, 8.0 / 12.0, -1.0 / 12.0};  // offsets -2, -1, 1, 2
  constexpr int off[4] = {-2, -1, 1, 2};
  double mx[3];
  const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    double v[4][4];
#pragma unroll
    for (int ia = 0; ia < 4; ++ia)
#pragma unroll
      for (int ib = 0; ib < 4; ++ib) {
        int o[3] = {0, 0, 0};
        o[pa[q]] = off[ia];
        o[pb[q]] = off[ib];
        v[ia][ib] = U(o[0], o[1], o[2]);
      }
    double outer = 0.0;
#pragma unroll
    for (int ia = 0; ia < 4; ++ia) {
      double inner = 0.0;
#pragma unroll
      for (int ib = 0; ib < 4; ++ib) inner += w1[ib] * v[ia][ib];
      outer += w1[ia] * (inner * h1);
    }
    mx[q] = outer * h1;
  }
  // g and grad g at y = x + grad u, trilinear and periodic
  const double y[3] = {i * invn + g[0], j * invn + g[1], k * invn + g[2]};
  int lo[3], hi[3];
  double fr[3];
  for (int a = 0; a < 3; ++a) {
    const double t = y[a] * N, fl = floor(t);
    fr[a] = t - fl;
    lo[a] = wrapf(fl, n, invn);
    hi[a] = lo[a] + 1 == n ? 0 : lo[a] + 1;
  }
  double gy = 0.0, gy1 = 0.0, gy2 = 0.0, gy3 = 0.0;
  const auto G = gmem<const double>(d.g);
  const auto GG = gmem<const float4>(d.gg);
  double gc[8];  // the eight corners' values, all loaded before the first is used
  float4 gg[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int c1 = c >> 2, c2 = (c >> 1) & 1, c3 = c & 1;
    const int idx = ((c1 ? hi[0] : lo[0]) * n + (c2 ? hi[1] : lo[1])) * n + (c3 ? hi[2] : lo[2]);
    gc[c] = G[idx];
    gg[c] = GG[idx];
  }
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int c1 = c >> 2, c2 = (c >> 1) & 1, c3 = c & 1;
    const double w = (c1 ? fr[0] : 1.0 - fr[0]) * (c2 ? fr[1] : 1.0 - fr[1]) * (c3 ? fr[2] : 1.0 - fr[2]);
    gy = gy + w * gc[c];
    gy1 = gy1 + w * (double)gg[c].x;
    gy2 = gy2 + w * (double)gg[c].y;
    gy3 = gy3 + w * (double)gg[c].z;
  }
  // det and cofactors of M = I + D^2 u
  const double m11 = 1.0 + s2[0], m22 = 1.0 + s2[1], m33 = 1.0 + s2[2];
  const double m12 = mx[0], m13 = mx[1], m23 = mx[2];
  const double c11 = m22 * m33 - m23 * m23, c22 = m11 * m33 - m13 * m13, c33 = m11 * m22 - m12 * m12;
  const double c12 = m13 * m23 - m12 * m33, c13 = m12 * m23 - m13 * m22, c23 = m12 * m13 - m11 * m23;
  const double det = m11 * c11 + m12 * c12 + m13 * c13;
  const double fn = gy * det;
  const double fe = gmem<const double>(d.f)[ei];
  const double rr = fe - fn;
  gmem<float>(d.r)[ei] = (float)rr;
  double cf[9] = {gy * c11, gy * c22, gy * c33, gy * c12, gy * c13, gy * c23, 0.0, 0.0, 0.0};
  if (op_mode == 0) {
    cf[6] = det * gy1;
    cf[7] = det * gy2;
    cf[8] = det * gy3;
  }
  // periodic Simpson weights (2/3 at even, 4/3 at odd indices, times 1/N per axis)
  const double ws = ((i & 1) ? 4.0 : 2.0) * ((j & 1) ? 4.0 : 2.0) * ((k & 1) ? 4.0 : 2.0) / (27.0 * N * N * N);
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    gmem<float>(d.coef)[q * (int)nn + ei] = (float)cf[q];
    acc[3 + q] += ws * cf[q];
  }
  acc[0] += fn;
  acc[1] += rr;
  acc[2] += rr * rr;
  acc[12] += (g[0] * g[0] + g[1] * g[1] + g[2] * g[2]) * fe;
  acc[13] += u0;
  acc[14] = fmin(acc[14], det);
  acc[15] = fmin(acc[15], m11);
  acc[16] = fmin(acc[16], m11 * m22 - m12 * m12);
  acc[17] = fmax(acc[17], rr);
  acc[18] = fmin(acc[18], rr);
  acc[19] += isfinite(rr) ? 0.0 : 1.0;
}

__device__ __forceinline__ void res_acc_init(double (&acc)[MA3_NPART]) {
  for (int k = 0; k < 14; ++k) acc[k] = 0.0;
  acc[14] = acc[15] = acc[16] = 1e300;
  acc[17] = -1e300;
  acc[18] = 1e300;
  acc[19] = 0.0;
}

__device__ __forceinline__ void res_acc_store(const Desc3& d, double (&acc)[MA3_NPART]) {
  __shared__ double scratch[4 * MA3_NPART];
  const int kinds[MA3_NPART] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 2, 1, 0};
  block_reduce<MA3_NPART>(acc, kinds, scratch);
  if (threadIdx.x == 0)
    for (int q = 0; q < MA3_NPART; ++q) d.part[(long)blockIdx.x * MA3_NPART + q] = acc[q];
}

// u read directly (cached) at every stencil point: any n
__global__ __launch_bounds__(MA3_BLOCK) void k3_res(Desc3 d, int op_mode) {
  const int n = d.n;
  const long nn = (long)n * n * n;
  double acc[MA3_NPART];
  res_acc_init(acc);
  // n^3 (and 9 n^3) stay below 2^31 for the supported sizes: 32-bit offsets
  const auto u = gmem<const double>(d.u);
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (long)gridDim.x * blockDim.x) {
    const int ei = (int)e, n2 = n * n;
    const int i = ei / n2, j = (ei / n) % n, k = ei % n;
    // wrapped offsets of the planes i - 2..i + 2, rows j - 2..j + 2, columns k - 2..k + 2
    int oi[5], oj[5], ok[5];
#pragma unroll
    for (int t = 0; t < 5; ++t) {
      oi[t] = wrap3(i + t - 2, n) * n2;
      oj[t] = wrap3(j + t - 2, n) * n;
      ok[t] = wrap3(k + t - 2, n);
    }
    res_point(d, op_mode, i, j, k, ei, [&](int a, int b, int c) { return u[oi[a + 2] + oj[b + 2] + ok[c + 2]]; },
              acc);
  }
  res_acc_store(d, acc);
}

// Streaming form (64 | n): a block takes a tile of R3_TJ rows x 64 columns of (j, k) and
// walks R3_TI planes along i with the five planes i - 2 .. i + 2 of u (tile plus a halo
// of two) in LDS; the next plane's loads are issued before the current plane is
// computed.  Wave w takes row j0 + w, lane l column k0 + l.
constexpr int R3_TJ = 4, R3_TI = 8, R3_W = 64 + 4, R3_H = R3_TJ + 4, R3_PLANE = R3_W * R3_H;
constexpr int R3_PER = (R3_PLANE + MA3_BLOCK - 1) / MA3_BLOCK;
static_assert(R3_TJ * 64 == MA3_BLOCK, "one point per thread and plane");

__global__ __launch_bounds__(MA3_BLOCK) void k3_res_s(Desc3 d, int op_mode) {
  const int n = d.n, n2 = n * n;
  const int ntk = n / 64, ntj = n / R3_TJ;
  const int b = blockIdx.x;
  const int k0 = (b % ntk) * 64, j0 = ((b / ntk) % ntj) * R3_TJ, i0 = (b / (ntk * ntj)) * R3_TI;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __shared__ double L[5 * R3_PLANE];
  const auto u = gmem<const double>(d.u);
  // tile element e of plane i: row jt = e / R3_W (j = j0 - 2 + jt), column kt = e % R3_W
  int toff[R3_PER];  // (j, k) offset of the thread's tile elements (elements past the tile: 0)
#pragma unroll
  for (int q = 0; q < R3_PER; ++q) {
    const int e = threadIdx.x + q * MA3_BLOCK;
    const int jt = e / R3_W, kt = e % R3_W;
    toff[q] = e < R3_PLANE ? wrap3(j0 - 2 + jt, n) * n + wrap3(k0 - 2 + kt, n) : 0;
  }
  auto slot = [&](int i) { return ((i - i0 + 2) % 5) * R3_PLANE; };  // i >= i0 - 2
  auto fetch = [&](int i, double (&v)[R3_PER]) {
    const int po = wrap3(i, n) * n2;
#pragma unroll
    for (int q = 0; q < R3_PER; ++q) v[q] = u[po + toff[q]];
  };
  auto put = [&](int i, const double (&v)[R3_PER]) {
#pragma unroll
    for (int q = 0; q < R3_PER; ++q) {
      const int e = threadIdx.x + q * MA3_BLOCK;
      if (e < R3_PLANE) L[slot(i) + e] = v[q];
    }
  };
  {  // planes i0 - 2 .. i0 + 2
    double v[5][R3_PER];
#pragma unroll
    for (int t = 0; t < 5; ++t) fetch(i0 - 2 + t, v[t]);
#pragma unroll
    for (int t = 0; t < 5; ++t) put(i0 - 2 + t, v[t]);
  }
  __syncthreads();
  double acc[MA3_NPART];
  res_acc_init(acc);
  const int j = j0 + w, k = k0 + lane;
  const int cell = (w + 2) * R3_W + lane + 2;  // the point's position in a plane tile
#pragma unroll 1
  for (int s = 0; s < R3_TI; ++s) {
    const int i = i0 + s;
    double nv[R3_PER];
    if (s + 1 < R3_TI) fetch(i + 3, nv);
    int so[5];
#pragma unroll
    for (int t = 0; t < 5; ++t) so[t] = slot(i - 2 + t) + cell;
    res_point(d, op_mode, i, j, k, (i * n + j) * n + k,
              [&](int a, int bb, int c) { return L[so[a + 2] + bb * R3_W + c]; }, acc);
    if (s + 1 < R3_TI) {
      __syncthreads();  // every read of plane i - 2 is done
      put(i + 3, nv);
      __syncthreads();
    }
  }
  res_acc_store(d, acc);
}

bool res_streams(int n) { return n % 64 == 0 && n % R3_TI == 0; }
int res_blocks(int n) { return res_streams(n) ? (n / 64) * (n / R3_TJ) * (n / R3_TI) : k3_blocks(n); }

__global__ __launch_bounds__(256) void k3_res_fold(Desc3 d, State3* s, int nblk) {
  __shared__ double scratch[4 * MA3_NPART];
  const int kinds[MA3_NPART] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 2, 1, 0};
  double t[MA3_NPART];
  fold_partials<MA3_NPART>(d.part, nblk, kinds, t, scratch);
  if (threadIdx.x == 0) {
    for (int q = 0; q < MA3_NPART; ++q) s->sums[q] = t[q];
    for (int q = 0; q < 9; ++q) s->abar[q] = t[3 + q];
    s->mass_c = t[0] / ((double)d.n * d.n * d.n) - 1.0;
  }
}

__global__ __launch_bounds__(MA3_BLOCK) void k3_upd(Desc3 d, double a) {
  const long nn = (long)d.n * d.n * d.n;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (long)gridDim.x * blockDim.x)
    d.u[e] += a * d.theta[e];
}

// psi = u - mean(u); map = x + D_h u (fourth order), unwrapped
__global__ __launch_bounds__(MA3_BLOCK) void k3_out(Desc3 d, const State3* s, double* psi, double* map) {
  const int n = d.n;
  const long nn = (long)n * n * n;
  const double mu = s->sums[13] / (double)nn, i12h = (double)n / 12.0, h = 1.0 / n;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e / ((long)n * n)), j = (int)((e / n) % n), k = (int)(e % n);
    psi[e] = d.u[e] - mu;
    if (map) {
      auto U = [&](int a, int b, int c) { return d.u[((long)wrap3(a, n) * n + wrap3(b, n)) * n + wrap3(c, n)]; };
      map[e] = i * h + (U(i - 2, j, k) - 8.0 * U(i - 1, j, k) + 8.0 * U(i + 1, j, k) - U(i + 2, j, k)) * i12h;
      map[nn + e] = j * h + (U(i, j - 2, k) - 8.0 * U(i, j - 1, k) + 8.0 * U(i, j + 1, k) - U(i, j + 2, k)) * i12h;
      map[2 * nn + e] = k * h + (U(i, j, k - 2) - 8.0 * U(i, j, k - 1) + 8.0 * U(i, j, k + 1) - U(i, j, k + 2)) * i12h;
    }
  }
}

// ---------------------------------------------------------------------------
// Arnoldi bookkeeping (one thread): as in the 2-D solver's GMRES(m) with Givens
// rotations, on the 3-D state
// ---------------------------------------------------------------------------
__device__ void arnoldi_close3(State3& s, int jn, double wnorm2) {
  const int j = jn - 1;
  double* col = &s.Hm[j * (MA3_MMAX + 1)];
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
  if (!(conv || jn >= s.m)) return;
  const int k = jn;
  for (int i = k - 1; i >= 0; --i) {
    double t = s.gv[i];
    for (int l = i + 1; l < k; ++l) t -= s.Hm[l * (MA3_MMAX + 1) + i] * s.y[l];
    const double di = s.Hm[i * (MA3_MMAX + 1) + i];
    s.y[i] = di != 0.0 ? t / di : 0.0;
  }
  s.gm_k = k;
  s.gm_running = 0;
  if (!conv && s.gm_cycle < s.max_restarts) {
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

// Krylov vector build, with the per-block partial sums of its square
__global__ __launch_bounds__(MA3_BLOCK) void k3_vec(Desc3 d, const State3* s, int mode, int jn) {
  const bool run = mode == V3_INIT ? true : (mode == V3_ARNOLDI ? (bool)s->gm_running : true);
  if (!run) return;
  __shared__ float cf[MA3_MMAX + 1];
  int nv = 0;
  if (mode == V3_ARNOLDI) nv = jn;
  else if (mode == V3_RECOVER) nv = s->gm_k;
  if (threadIdx.x < nv)
    cf[threadIdx.x] = mode == V3_ARNOLDI ? (float)(s->Hm[(jn - 1) * (MA3_MMAX + 1) + threadIdx.x] * s->vscale[threadIdx.x])
                                         : (float)s->y[threadIdx.x];
  __syncthreads();
  const long nn = (long)d.n * d.n * d.n;
  const float cst = (float)s->mass_c, itau = (float)(1.0 / s->tau);
  const bool usex = mode == V3_RECOVER && s->gm_cycle > 0;
  double acc = 0.0;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (long)gridDim.x * blockDim.x) {
    float v;
    if (mode == V3_INIT) {
      v = (d.r[e] + cst) * itau;
      d.V[e] = v;
    } else if (mode == V3_ARNOLDI) {
      v = d.V[(long)jn * nn + e];
      for (int l = 0; l < nv; ++l) v -= cf[l] * d.V[(long)l * nn + e];
      d.V[(long)jn * nn + e] = v;
    } else {  // recovery: x = (x of earlier cycles) + sum y_l V_l
      v = usex ? d.x[e] : 0.f;
      for (int l = 0; l < nv; ++l) v += cf[l] * d.V[(long)l * nn + e];
      d.x[e] = v;
    }
    acc += (double)v * v;
  }
  __shared__ double scratch[4];
  double t[1] = {acc};
  const int kinds[1] = {0};
  block_reduce<1>(t, kinds, scratch);
  if (threadIdx.x == 0) d.part[blockIdx.x] = t[0];
}

// the fold after k3_vec: the right-hand side's norm (init) or ||w'|| and the rotations
__global__ __launch_bounds__(256) void k3_vec_fold(Desc3 d, State3* s, int mode, int jn, int nblk) {
  if (mode == V3_ARNOLDI && !s->gm_running) return;
  __shared__ double scratch[4];
  const int kinds[1] = {0};
  double t[1];
  if (mode == V3_ARNOLDI) {  // the rotations run on a copy of the state in LDS
    __shared__ State3 ls;
    StagedWords<State3, 256> sw;
    sw.load(s);
    fold_partials<1>(d.part, nblk, kinds, t, scratch);
    sw.to_lds(&ls);
    __syncthreads();
    if (threadIdx.x == 0) arnoldi_close3(ls, jn, t[0]);
    __syncthreads();
    sw.write_back(&ls, s);
    return;
  }
  fold_partials<1>(d.part, nblk, kinds, t, scratch);
  if (threadIdx.x != 0) return;
  if (mode == V3_INIT) {
    const double bn = sqrt(fmax(t[0], 0.0));
    s->bnorm = bn;
    s->gm_target = s->gmres_tol * bn;
    s->gm_running = bn > 0.0;
    s->gm_restart = 0;
    s->gm_cycle = 0;
    s->gm_k = 0;
    s->vscale[0] = bn > 0.0 ? 1.0 / bn : 0.0;
    s->gv[0] = bn;
  }
}

// x += sum y_l V_l and V0 = the cycle's residual; then the next cycle begins
__global__ __launch_bounds__(MA3_BLOCK) void k3_rst(Desc3 d, const State3* s) {
  __shared__ float cy[MA3_MMAX + 1], cq[MA3_MMAX + 1];
  const int k = s->gm_k;
  const bool usex = s->gm_cycle > 0;
  if (threadIdx.x <= k) {
    cy[threadIdx.x] = threadIdx.x < k ? (float)s->y[threadIdx.x] : 0.f;
    cq[threadIdx.x] = (float)s->q[threadIdx.x];
  }
  __syncthreads();
  const long nn = (long)d.n * d.n * d.n;
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

__global__ void k3_cycle_begin(State3* s) {
  if (threadIdx.x == 0 && s->gm_restart) {
    s->gm_running = 1;
    s->gm_restart = 0;
    s->gm_cycle++;
  }
}

// ---------------------------------------------------------------------------
// line-transform passes
// ---------------------------------------------------------------------------
// The line passes below issue every global load of a phase before the phase's first
// LDS write, and read their twiddles from an LDS copy of the table (so that no
// in-order wait on a twiddle load holds back the other loads in flight).

// P1: real input along x3 -> complex forward transform -> S.  Input: V[j] (matvec) or x.
template <int N>
__global__ __launch_bounds__(MA3_BLOCK) void k3_p1(Desc3 d, const State3* s, int mode, int j) {
  if (mode == P3_MATVEC && !s->gm_running) return;
  constexpr int R = Lines3<N>::P1;  // lines per block
  constexpr int PER = R * N / MA3_BLOCK;
  static_assert((R * N) % MA3_BLOCK == 0, "whole elements per thread");
  __shared__ float2 L[R * N];
  __shared__ float2 twl[tw_span(N, TW_FULL)];
  const long nn = (long)N * N * N;
  const float* in = mode == P3_MATVEC ? d.V + (long)j * nn : d.x;
  const long base = (long)blockIdx.x * R * N;
  TwiddleStage<N, MA3_BLOCK, TW_FULL> tws;  // issued before the data loads
  tws.load(d.tw);
  float x[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) x[q] = in[base + threadIdx.x + q * MA3_BLOCK];
  tws.store(twl);
#pragma unroll
  for (int q = 0; q < PER; ++q) L[threadIdx.x + q * MA3_BLOCK] = make_float2(x[q], 0.f);
  __syncthreads();
  fft_lds<N, R, MA3_BLOCK, false, LAYOUT_ROWS, TW_FULL>(L, twl);
  for (int e = threadIdx.x; e < R * N; e += MA3_BLOCK) d.S[base + e] = L[e];
}

// element e of a block's tile in the x1 / x2 passes: line e % C, position e / C along it
template <int N, int C>
__device__ __forceinline__ long col_index(long plane_or_row_base, long stride, int e) {
  return plane_or_row_base + (long)(e / C) * stride + (e % C);
}

// P2: forward transform along x2, in place; a block takes COLS consecutive x3 indices
// of one x1 plane
template <int N>
__global__ __launch_bounds__(MA3_BLOCK) void k3_p2(Desc3 d, const State3* s, int mode) {
  if (mode == P3_MATVEC && !s->gm_running) return;
  constexpr int C = COLS < N ? COLS : N;
  constexpr int PER = N * C / MA3_BLOCK;
  static_assert((N * C) % MA3_BLOCK == 0, "whole elements per thread");
  __shared__ float2 L[N * C];
  __shared__ float2 twl[tw_span(N, TW_FULL)];
  const int i = blockIdx.x / (N / C), k0 = (blockIdx.x % (N / C)) * C;
  const long b0 = (long)i * N * N + k0;  // element (i, jj, k0 + t) at b0 + jj N + t
  TwiddleStage<N, MA3_BLOCK, TW_FULL> tws;  // issued before the data loads
  tws.load(d.tw);
  float2 v[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) v[q] = d.S[col_index<N, C>(b0, N, threadIdx.x + q * MA3_BLOCK)];
  tws.store(twl);
#pragma unroll
  for (int q = 0; q < PER; ++q) L[threadIdx.x + q * MA3_BLOCK] = v[q];
  __syncthreads();
  fft_lds<N, C, MA3_BLOCK, false, LAYOUT_COLS, TW_FULL>(L, twl);
  for (int e = threadIdx.x; e < N * C; e += MA3_BLOCK) d.S[col_index<N, C>(b0, N, e)] = L[e];
}

// rhobar(k) from the multipliers of the wavenumber indices (q1, q2, q3): the inverse
// symbol of the averaged operator, zero where it vanishes (k = 0)
__device__ __forceinline__ float2 rhobar3(int q1, int q2, int q3, float2 m1, float2 m2, float2 m3,
                                          const float (&ab)[9]) {
  // S = sum a_aa d2(k_a) + 2 sum_{a<b} a_ab (i d1(k_a))(i d1(k_b)) + i sum b_a d1(k_a)
  const float re = ab[0] * m1.y + ab[1] * m2.y + ab[2] * m3.y -
                   2.f * (ab[3] * m1.x * m2.x + ab[4] * m1.x * m3.x + ab[5] * m2.x * m3.x);
  const float im = ab[6] * m1.x + ab[7] * m2.x + ab[8] * m3.x;
  const float den = re * re + im * im;
  if ((q1 == 0 && q2 == 0 && q3 == 0) || den == 0.f) return make_float2(0.f, 0.f);
  const float inv = 1.f / den;  // one division for both parts
  return make_float2(re * inv, -im * inv);
}

// P3: forward transform along x1, times rhobar and the scale, inverse transforms of
// Z, i k1 Z, -k1^2 Z -> T0, T1, T2 (theta: Z -> T0 only).  A block takes COLS
// consecutive x3 indices of one x2 row.
template <int N>
__global__ __launch_bounds__(MA3_BLOCK) void k3_p3(Desc3 d, const State3* s, int mode, int j) {
  if (mode == P3_MATVEC && !s->gm_running) return;
  constexpr int C = COLS < N ? COLS : N;
  constexpr long NN = (long)N * N * N;
  constexpr int PER = N * C / MA3_BLOCK;
  static_assert((N * C) % MA3_BLOCK == 0, "whole elements per thread");
  __shared__ float2 L[N * C];
  __shared__ float2 twl[tw_span(N, TW_FULL)];
  const int jj = blockIdx.x / (N / C), k0 = (blockIdx.x % (N / C)) * C;
  const long b0 = (long)jj * N + k0;  // element (i, jj, k0 + t) at b0 + i N^2 + t
  TwiddleStage<N, MA3_BLOCK, TW_FULL> tws;  // issued before the data loads
  tws.load(d.tw);
  float2 v[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) v[q] = d.S[col_index<N, C>(b0, (long)N * N, threadIdx.x + q * MA3_BLOCK)];
  float2 m[PER];  // multipliers at the thread's wavenumbers k1 = e / C
#pragma unroll
  for (int q = 0; q < PER; ++q) m[q] = d.mt[(threadIdx.x + q * MA3_BLOCK) / C];
  const int t = threadIdx.x % C;  // the thread's x3 index k0 + t (the same for every q)
  const float2 m2 = d.mt[jj], m3 = d.mt[k0 + t];
  float ab[9];
  for (int q = 0; q < 9; ++q) ab[q] = (float)s->abar[q];
  const float scale = (float)((mode == P3_MATVEC ? s->vscale[j] : 1.0) / ((double)N * N * N));
  tws.store(twl);
#pragma unroll
  for (int q = 0; q < PER; ++q) L[threadIdx.x + q * MA3_BLOCK] = v[q];
  __syncthreads();
  fft_lds<N, C, MA3_BLOCK, false, LAYOUT_COLS, TW_FULL>(L, twl);
  // Z = rhobar * spectrum * scale, kept in registers (each thread its own elements)
  float2 z[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = threadIdx.x + q * MA3_BLOCK;
    const float2 rb = rhobar3(e / C, jj, k0 + t, m[q], m2, m3, ab);
    z[q] = cscale(cmul(rb, L[e]), scale);
  }
  const int outs = mode == P3_MATVEC ? 3 : 1;
  for (int o = 0; o < outs; ++o) {
    __syncthreads();  // the previous transform's results have been stored
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      // o = 0: Z; o = 1: i d1(k1) Z; o = 2: d2(k1) Z
      L[threadIdx.x + q * MA3_BLOCK] =
          o == 0 ? z[q] : (o == 1 ? make_float2(-m[q].x * z[q].y, m[q].x * z[q].x) : cscale(z[q], m[q].y));
    }
    __syncthreads();
    fft_lds<N, C, MA3_BLOCK, true, LAYOUT_COLS, TW_FULL>(L, twl);
    float2* T = d.T + (long)o * NN;
    for (int e = threadIdx.x; e < N * C; e += MA3_BLOCK) T[col_index<N, C>(b0, (long)N * N, e)] = L[e];
  }
}

// P4: inverse transforms along x2 of T2, T1, i k2 T1, T0, i k2 T0, -k2^2 T0 -> U_a..U_f
// (theta: T0 -> U_d only).  A block takes COLS consecutive x3 indices of one x1 plane.
// Each source plane is loaded once (the next one's loads issued before the current
// one's transforms) and every output derived from it is transformed in turn.
template <int N>
__global__ __launch_bounds__(MA3_BLOCK) void k3_p4(Desc3 d, const State3* s, int mode) {
  if (mode == P3_MATVEC && !s->gm_running) return;
  constexpr int C = COLS < N ? COLS : N;
  constexpr long NN = (long)N * N * N;
  constexpr int PER = N * C / MA3_BLOCK;
  static_assert((N * C) % MA3_BLOCK == 0, "whole elements per thread");
  __shared__ float2 L[N * C];
  __shared__ float2 twl[tw_span(N, TW_FULL)];
  const int i = blockIdx.x / (N / C), k0 = (blockIdx.x % (N / C)) * C;
  const long b0 = (long)i * N * N + k0;
  // sources in order (T plane, first output, outputs): T2 -> U_a; T1 -> U_b, U_c (i d1);
  // T0 -> U_d, U_e (i d1), U_f (d2); theta: T0 -> U_d
  const bool mv = mode == P3_MATVEC;
  const int nsrc = mv ? 3 : 1;
  auto src_plane = [&](int si) { return mv ? 2 - si : 0; };
  TwiddleStage<N, MA3_BLOCK, TW_FULL> tws;  // issued before the data loads
  tws.load(d.tw);
  float2 cur[PER], nxt[PER], m[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) cur[q] = d.T[src_plane(0) * NN + col_index<N, C>(b0, N, threadIdx.x + q * MA3_BLOCK)];
#pragma unroll
  for (int q = 0; q < PER; ++q) m[q] = d.mt[(threadIdx.x + q * MA3_BLOCK) / C];
  tws.store(twl);
  int out = mv ? 0 : 3;
  for (int si = 0; si < nsrc; ++si) {
    if (si + 1 < nsrc) {
#pragma unroll
      for (int q = 0; q < PER; ++q)
        nxt[q] = d.T[src_plane(si + 1) * NN + col_index<N, C>(b0, N, threadIdx.x + q * MA3_BLOCK)];
    }
    const int nmul = mv ? si + 1 : 1;  // multipliers 0 .. nmul - 1: one, i d1(k2), d2(k2)
    for (int mu = 0; mu < nmul; ++mu, ++out) {
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const float2 v = cur[q];
        L[threadIdx.x + q * MA3_BLOCK] =
            mu == 0 ? v : (mu == 1 ? make_float2(-m[q].x * v.y, m[q].x * v.x) : cscale(v, m[q].y));
      }
      __syncthreads();
      fft_lds<N, C, MA3_BLOCK, true, LAYOUT_COLS, TW_FULL>(L, twl);
      float2* Uo = d.U + (long)out * NN;
      for (int e = threadIdx.x; e < N * C; e += MA3_BLOCK) Uo[col_index<N, C>(b0, N, e)] = L[e];
      __syncthreads();  // the stores have read L before the next transform overwrites it
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) cur[q] = nxt[q];
  }
}

// P5: along x3, the nine real results as five complex inverse transforms, then the
// combination and the inner products (matvec), or theta and u += theta.  A block takes
// R5 whole x3 lines.
template <int N>
__global__ __launch_bounds__(MA3_BLOCK) void k3_p5(Desc3 d, const State3* s, int mode, int j) {
  if (mode == P3_MATVEC && !s->gm_running) return;
  constexpr long NN = (long)N * N * N;
  constexpr int R5 = Lines3<N>::P5;  // lines per block
  constexpr int NT = 5;              // transforms per line
  constexpr int PER = R5 * N / MA3_BLOCK;
  static_assert((R5 * N) % MA3_BLOCK == 0, "whole elements per thread");
  __shared__ float2 L[NT * R5 * N];
  __shared__ float2 twl[tw_span(N, TW_FULL)];
  __shared__ double red[(MA3_BLOCK / 64) * (MA3_MMAX + 1)];
  const long base = (long)blockIdx.x * R5 * N;  // first element of the block's lines
  TwiddleStage<N, MA3_BLOCK, TW_FULL> tws;  // issued before the data loads
  tws.load(d.tw);
  if (mode != P3_MATVEC) {
    const float2* Ud = d.U + 3 * NN;
    float2 v[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) v[q] = Ud[base + threadIdx.x + q * MA3_BLOCK];
    tws.store(twl);
#pragma unroll
    for (int q = 0; q < PER; ++q) L[threadIdx.x + q * MA3_BLOCK] = v[q];
    __syncthreads();
    fft_lds<N, R5, MA3_BLOCK, true, LAYOUT_ROWS, TW_FULL>(L, twl);
    for (int e = threadIdx.x; e < R5 * N; e += MA3_BLOCK) {
      const double th = (double)L[e].x;
      if (mode == P3_THETA) {
        d.theta[base + e] = th;
        d.u[base + e] += th;
      } else {
        d.x[base + e] = L[e].x;
      }
    }
    return;
  }
  // transform t of line l at L[(t * R5 + l) * N + k]:
  //   0: U_a + i U_b        -> alpha11, beta1
  //   1: U_c + i (i d1 U_b) -> alpha12, alpha13
  //   2: U_f + i U_e        -> alpha22, beta2
  //   3: i d1 U_e + i d2 U_d -> alpha23, alpha33
  //   4: i d1 U_d           -> beta3
  float2 uv[6][PER], m[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const long g = base + threadIdx.x + q * MA3_BLOCK;
#pragma unroll
    for (int c = 0; c < 6; ++c) uv[c][q] = d.U[c * NN + g];
    m[q] = d.mt[(threadIdx.x + q * MA3_BLOCK) % N];
  }
  tws.store(twl);
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = threadIdx.x + q * MA3_BLOCK;
    const int l = e / N, k = e % N;
    const float2 ua = uv[0][q], ub = uv[1][q], uc = uv[2][q], ud = uv[3][q], ue = uv[4][q], uf = uv[5][q];
    const float2 mk = m[q];
    const float2 ib = make_float2(-mk.x * ub.y, mk.x * ub.x);  // i d1(k3) U_b
    const float2 ie = make_float2(-mk.x * ue.y, mk.x * ue.x);
    const float2 id = make_float2(-mk.x * ud.y, mk.x * ud.x);
    const float2 qd = cscale(ud, mk.y);
    // X + i Y for spectra X, Y of real signals
    L[(0 * R5 + l) * N + k] = make_float2(ua.x - ub.y, ua.y + ub.x);
    L[(1 * R5 + l) * N + k] = make_float2(uc.x - ib.y, uc.y + ib.x);
    L[(2 * R5 + l) * N + k] = make_float2(uf.x - ue.y, uf.y + ue.x);
    L[(3 * R5 + l) * N + k] = make_float2(ie.x - qd.y, ie.y + qd.x);
    L[(4 * R5 + l) * N + k] = id;
  }
  __syncthreads();
  fft_lds<N, NT * R5, MA3_BLOCK, true, LAYOUT_ROWS, TW_FULL>(L, twl);
  float* W = d.V + (long)(j + 1) * NN;
  // the nine coefficients at all of the thread's points, loaded before the first is used
  float cf[9][PER];
#pragma unroll
  for (int q = 0; q < PER; ++q)
#pragma unroll
    for (int c = 0; c < 9; ++c) cf[c][q] = d.coef[c * NN + base + threadIdx.x + q * MA3_BLOCK];
  float w[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = threadIdx.x + q * MA3_BLOCK;
    const int l = e / N, k = e % N;
    const long g = base + e;
    const float2 z0 = L[(0 * R5 + l) * N + k], z1 = L[(1 * R5 + l) * N + k], z2 = L[(2 * R5 + l) * N + k];
    const float2 z3 = L[(3 * R5 + l) * N + k], z4 = L[(4 * R5 + l) * N + k];
    // a11 a11 + a22 a22 + a33 a33 + 2 (a12 a12 + a13 a13 + a23 a23) + b . beta
    const float v = cf[0][q] * z0.x + cf[1][q] * z2.x + cf[2][q] * z3.y +
                    2.f * (cf[3][q] * z1.x + cf[4][q] * z1.y + cf[5][q] * z3.x) + cf[6][q] * z0.y +
                    cf[7][q] * z2.y + cf[8][q] * z4.x;
    W[g] = v;
    w[q] = v;
  }
  // inner products <w, V_l>, l <= j, per block (fixed order); folded by k3_dots_fold
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  stream_vectors<PER>(
      j + 1,
      [&](int lv, float* x) {
#pragma unroll
        for (int q = 0; q < PER; ++q) x[q] = d.V[(long)lv * NN + base + threadIdx.x + q * MA3_BLOCK];
      },
      [&](int lv, const float* x) {
        float acc = 0.f;
#pragma unroll
        for (int q = 0; q < PER; ++q) acc += w[q] * x[q];
        const double v = wave_sum((double)acc);
        if (lane == 0) red[wid * (MA3_MMAX + 1) + lv] = v;
      });
  __syncthreads();
  if (threadIdx.x <= j) {
    double t = 0.0;
    for (int ww = 0; ww < MA3_BLOCK / 64; ++ww) t += red[ww * (MA3_MMAX + 1) + threadIdx.x];
    d.part[(long)blockIdx.x * (MA3_MMAX + 1) + threadIdx.x] = t;
  }
}

// h[l][j] = <w, v_l> from the P5 partials (one block of 1024 threads): lane l of group g
// sums blocks g, g + 32, ... with 16 loads in flight per round, then the groups are
// summed in order (a fixed order throughout)
__global__ __launch_bounds__(1024) void k3_dots_fold(Desc3 d, State3* s, int j, int nblk) {
  if (!s->gm_running) return;
  __shared__ double red[32][32];
  const int l = threadIdx.x & 31, grp = threadIdx.x >> 5;
  const double t = l <= j ? strided_sum<16>(d.part, MA3_MMAX + 1, l, grp, 32, nblk) : 0.0;
  red[grp][l] = t;
  __syncthreads();
  if (threadIdx.x <= j) {
    double u = 0.0;
    for (int g2 = 0; g2 < 32; ++g2) u += red[g2][threadIdx.x];
    s->Hm[j * (MA3_MMAX + 1) + threadIdx.x] = u * s->vscale[threadIdx.x];
  }
}

template <int N>
void forward_rest_n(const Desc3& d, State3* s, int mode, hipStream_t st) {
  constexpr int C = COLS < N ? COLS : N;
  hipLaunchKernelGGL(k3_p2<N>, dim3(N * (N / C)), dim3(MA3_BLOCK), 0, st, d, s, mode);
}

template <int N>
void first_pass_n(const Desc3& d, State3* s, int mode, int j, hipStream_t st) {
  constexpr int R = Lines3<N>::P1;
  hipLaunchKernelGGL(k3_p1<N>, dim3((N * N) / R), dim3(MA3_BLOCK), 0, st, d, s, mode, j);
}

template <int N>
void inverse_n(const Desc3& d, State3* s, int mode, int j, hipStream_t st) {
  constexpr int C = COLS < N ? COLS : N;
  constexpr int R5 = Lines3<N>::P5;
  hipLaunchKernelGGL(k3_p3<N>, dim3(N * (N / C)), dim3(MA3_BLOCK), 0, st, d, s, mode, j);
  hipLaunchKernelGGL(k3_p4<N>, dim3(N * (N / C)), dim3(MA3_BLOCK), 0, st, d, s, mode);
  hipLaunchKernelGGL(k3_p5<N>, dim3((N * N) / R5), dim3(MA3_BLOCK), 0, st, d, s, mode, j);
  if (mode == P3_MATVEC)
    hipLaunchKernelGGL(k3_dots_fold, dim3(1), dim3(1024), 0, st, d, s, j, (N * N) / R5);
}

#define MA3_FOR_EACH_N(X) X(16) X(32) X(48) X(64) X(96) X(128) X(192) X(256)

}  // namespace

bool n3_supported(int n) {
  switch (n) {
#define X(NV) case NV:
    MA3_FOR_EACH_N(X)
#undef X
    return true;
    default:
      return false;
  }
}

int k3_blocks(int n) {
  const long b = (long)n * n * n / (MA3_BLOCK * 4);
  return b < 1 ? 1 : (int)(b > 8192 ? 8192 : b);
}

int k3_dot_blocks(int n) { return n * n / pow2_floor((LINES_ELEMS / 2) / n); }

void k3_setup(const Desc3& d, State3* s, bool scale, hipStream_t st) {
  const int nb = k3_blocks(d.n);
  if (scale) {
    hipLaunchKernelGGL(k3_sums, dim3(nb), dim3(MA3_BLOCK), 0, st, d);
    hipLaunchKernelGGL(k3_sums_fold, dim3(1), dim3(256), 0, st, d, s, nb);
  }
  hipLaunchKernelGGL(k3_fields, dim3(nb), dim3(MA3_BLOCK), 0, st, d, s);
}

void k3_residual(const Desc3& d, State3* s, int op_mode, hipStream_t st) {
  const int nb = res_blocks(d.n);
  if (res_streams(d.n))
    hipLaunchKernelGGL(k3_res_s, dim3(nb), dim3(MA3_BLOCK), 0, st, d, op_mode);
  else
    hipLaunchKernelGGL(k3_res, dim3(nb), dim3(MA3_BLOCK), 0, st, d, op_mode);
  hipLaunchKernelGGL(k3_res_fold, dim3(1), dim3(256), 0, st, d, s, nb);
}

void k3_update(const Desc3& d, double a, hipStream_t st) {
  hipLaunchKernelGGL(k3_upd, dim3(k3_blocks(d.n)), dim3(MA3_BLOCK), 0, st, d, a);
}

void k3_outputs(const Desc3& d, const State3* s, double* psi, double* map, hipStream_t st) {
  hipLaunchKernelGGL(k3_out, dim3(k3_blocks(d.n)), dim3(MA3_BLOCK), 0, st, d, s, psi, map);
}

void k3_vector(const Desc3& d, State3* s, int mode, int jn, hipStream_t st) {
  const int nb = k3_blocks(d.n);
  hipLaunchKernelGGL(k3_vec, dim3(nb), dim3(MA3_BLOCK), 0, st, d, s, mode, jn);
  if (mode == V3_INIT || mode == V3_ARNOLDI)
    hipLaunchKernelGGL(k3_vec_fold, dim3(1), dim3(256), 0, st, d, s, mode, jn, nb);
}

void k3_restart(const Desc3& d, State3* s, hipStream_t st) {
  hipLaunchKernelGGL(k3_rst, dim3(k3_blocks(d.n)), dim3(MA3_BLOCK), 0, st, d, s);
  hipLaunchKernelGGL(k3_cycle_begin, dim3(1), dim3(64), 0, st, s);
}

// the first pass: mode P3_* with the input V[j] (matvec) or x
void k3_forward_rest(const Desc3& d, State3* s, int mode, hipStream_t st) {
  switch (d.n) {
#define X(NV) \
  case NV: forward_rest_n<NV>(d, s, mode, st); break;
    MA3_FOR_EACH_N(X)
#undef X
    default: break;
  }
}

void k3_first_pass(const Desc3& d, State3* s, int mode, int j, hipStream_t st) {
  switch (d.n) {
#define X(NV) \
  case NV: first_pass_n<NV>(d, s, mode, j, st); break;
    MA3_FOR_EACH_N(X)
#undef X
    default: break;
  }
}

void k3_inverse(const Desc3& d, State3* s, int mode, int j, hipStream_t st) {
  switch (d.n) {
#define X(NV) \
  case NV: inverse_n<NV>(d, s, mode, j, st); break;
    MA3_FOR_EACH_N(X)
#undef X
    default: break;
  }
}
