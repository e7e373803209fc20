// Warm-start network kernels: periodic 3x3 convolutions in BF16 on MFMA with FP32
// accumulation, and what inference and training need around them.
//
// Activations are BF16, channels last ([sample][row][column][channel]); the
// network input has 8 stored channels (log f, log g of the mean-one densities, six
// zeros), hidden layers 32.
// A layer may be dilated by d (taps d pixels apart): a block then works on a 16 x 16
// tile of one of the d^2 interleaved subgrids (pixels with the same row and column
// residues mod d), where the taps are nearest neighbours, periodic with side n/d.
// A convolution is an implicit GEMM per 16-pixel strip: D[co][pixel] =
// sum_k A[co][k] B[k][pixel] with k = tap * C_in + ci, computed by
// v_mfma_f32_16x16x32_bf16 (lane l holds A[l%16][8(l/16)..+7], B[8(l/16)..+7][l%16]
// and D[4(l/16)..+3][l%16]).  The backward pass through the input is the same
// kernel with the kernel transposed over channels and flipped in space; the weight
// gradient reduces over pixels with the pixel index as the MFMA k dimension, from
// channel-major LDS copies of the tiles, followed by a fixed-order sum over blocks.
#include <hip/hip_runtime.h>

#include "cnn.h"

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// ---------------------------------------------------------------------------
// convolution: one block = a 16 x 16 pixel tile, 4 waves x 4 strips of 16 pixels
// ---------------------------------------------------------------------------
template <int CIN, int COUT_PAD, int MODE>
__global__ __launch_bounds__(256) void k_conv(const bf16* __restrict__ in, const bf16x8* __restrict__ wp,
                                              const float* __restrict__ bias, const bf16* __restrict__ mask,
                                              bf16* __restrict__ out_bf, float* __restrict__ out_f, int H, int W,
                                              int dil) {
  constexpr int KB = (9 * CIN + 31) / 32;  // k blocks of 32
  constexpr int MB = COUT_PAD / 16;        // 16-channel output blocks
  constexpr int TW = 16, TH = 16, LW = TW + 2, LH = TH + 2;
  constexpr int CH8 = CIN / 8;             // 16-byte channel chunks per pixel
  __shared__ bf16x8 tile[LH * LW * CH8];
  const int b = blockIdx.z;
  const int Hd = H / dil, Wd = W / dil;  // subgrid sides
  const int res = blockIdx.x % (dil * dil), t = blockIdx.x / (dil * dil);
  const int ry = res / dil, rx = res % dil;
  const int tiles_x = Wd / TW;
  const int ty0 = (t / tiles_x) * TH, tx0 = (t % tiles_x) * TW;
  const bf16x8* inb = reinterpret_cast<const bf16x8*>(in) + (size_t)b * H * W * CH8;
  for (int e = threadIdx.x; e < LH * LW * CH8; e += 256) {
    const int chunk = e % CH8, pix = e / CH8;
    const int ly = pix / LW, lx = pix % LW;
    const int gy = wrap(ty0 + ly - 1, Hd) * dil + ry, gx = wrap(tx0 + lx - 1, Wd) * dil + rx;
    tile[e] = inb[((size_t)gy * W + gx) * CH8 + chunk];
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  bf16x8 wreg[MB][KB];
#pragma unroll
  for (int cb = 0; cb < MB; ++cb)
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) wreg[cb][kb] = wp[(cb * KB + kb) * 64 + lane];
  __syncthreads();

  const int px = lane & 15, kq = lane >> 4;
  const bf16x8 zero8 = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll 1
  for (int rr = 0; rr < 4; ++rr) {
    const int row = wave * 4 + rr;
    f32x4 acc[MB];
#pragma unroll
    for (int cb = 0; cb < MB; ++cb) acc[cb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      const int tap = (CIN == 32) ? kb : kb * 4 + kq;
      const int chunk = (CIN == 32) ? kq : 0;
      bf16x8 bop = zero8;
      if (tap < 9) bop = tile[((row + tap / 3) * LW + px + tap % 3) * CH8 + chunk];
#pragma unroll
      for (int cb = 0; cb < MB; ++cb)
        acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wreg[cb][kb], bop, acc[cb], 0, 0, 0);
    }
    const size_t pixel = ((size_t)b * H + (ty0 + row) * dil + ry) * W + (tx0 + px) * dil + rx;
    if constexpr (MODE == CV_FWD_LAST) {
      if (kq == 0) out_f[pixel] = acc[0][0] + bias[0];
    } else {
#pragma unroll
      for (int cb = 0; cb < MB; ++cb) {
        const int co0 = cb * 16 + kq * 4;
        bf16x4 o;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          float v = acc[cb][e];
          if constexpr (MODE == CV_FWD_RELU) v = fmaxf(v + bias[co0 + e], 0.f);
          if constexpr (MODE == CV_BWD_DATA) v = ((float)mask[pixel * 32 + co0 + e] > 0.f) ? v : 0.f;
          o[e] = (bf16)v;
        }
        *reinterpret_cast<bf16x4*>(out_bf + pixel * 32 + co0) = o;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// weight gradient: D[co][ci] += sum over 32 pixels (two 16-pixel rows of a tile) of
// dz[p][co] h[p+off][ci]
// ---------------------------------------------------------------------------
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_conv_wgrad(const bf16* __restrict__ h, const bf16* __restrict__ dz, int B,
                                                    int H, int W, int dil, int cout_real, int cin_real,
                                                    float* __restrict__ part, float* __restrict__ partb) {
  constexpr int TR = 16, TC = 16, LW = TC + 2, LH = TR + 2;
  constexpr int RPK = 32 / TC;  // tile rows per MFMA k block
  constexpr int MB = (COUT + 15) / 16, NB = (CIN + 15) / 16;
  constexpr int NCOMBO = 9 * MB * NB, PERW = (NCOMBO + 3) / 4;
  __shared__ __attribute__((aligned(16))) bf16 dzT[COUT * TR * TC];  // [co][r][c]
  __shared__ bf16 hT[CIN * LH * LW];                                  // [ci][ly][lx]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kq = lane >> 4, l16 = lane & 15;
  const int Hd = H / dil, Wd = W / dil;  // subgrid sides
  const int tiles_y = Hd / TR, tiles_x = Wd / TC;
  const int per_sample = dil * dil * tiles_y * tiles_x;
  const int ntiles = B * per_sample;
  f32x4 acc[PERW];
#pragma unroll
  for (int i = 0; i < PERW; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;
  const bf16x8 zero8 = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int s = t / per_sample, rem = t % per_sample;
    const int res = rem % (dil * dil), tt = rem / (dil * dil);
    const int ry = res / dil, rx = res % dil;
    const int y0 = (tt / tiles_x) * TR, x0 = (tt % tiles_x) * TC;
    const bf16x8* dz8 = reinterpret_cast<const bf16x8*>(dz) + (size_t)s * H * W * (COUT / 8);
    const bf16x8* h8 = reinterpret_cast<const bf16x8*>(h) + (size_t)s * H * W * (CIN / 8);
    __syncthreads();  // the previous tile is no longer read
    for (int e = threadIdx.x; e < TR * TC * (COUT / 8); e += 256) {
      const int chunk = e % (COUT / 8), pix = e / (COUT / 8);
      const int r = pix / TC, c = pix % TC;
      const bf16x8 v = dz8[((size_t)((y0 + r) * dil + ry) * W + (x0 + c) * dil + rx) * (COUT / 8) + chunk];
#pragma unroll
      for (int k = 0; k < 8; ++k) dzT[((chunk * 8 + k) * TR + r) * TC + c] = v[k];
    }
    for (int e = threadIdx.x; e < LH * LW * (CIN / 8); e += 256) {
      const int chunk = e % (CIN / 8), pix = e / (CIN / 8);
      const int ly = pix / LW, lx = pix % LW;
      const int gy = wrap(y0 + ly - 1, Hd) * dil + ry, gx = wrap(x0 + lx - 1, Wd) * dil + rx;
      const bf16x8 v = h8[((size_t)gy * W + gx) * (CIN / 8) + chunk];
#pragma unroll
      for (int k = 0; k < 8; ++k) hT[((chunk * 8 + k) * LH + ly) * LW + lx] = v[k];
    }
    __syncthreads();
    if (threadIdx.x < COUT)
      for (int q = 0; q < TR * TC; ++q) bsum += (float)dzT[threadIdx.x * TR * TC + q];
#pragma unroll
    for (int i = 0; i < PERW; ++i) {
      const int combo = wave + 4 * i;
      if (combo < NCOMBO) {
        const int tap = combo / (MB * NB), cb = (combo / NB) % MB, nb = combo % NB;
        const int dy = tap / 3, dx = tap % 3;
        const int co = cb * 16 + l16, ci = nb * 16 + l16;
        // lane group kq takes 8 consecutive pixels: row r, columns c0..c0+7
        const int rq = kq / (TC / 8), c0 = 8 * (kq % (TC / 8));
#pragma unroll 1
        for (int rb = 0; rb < TR / RPK; ++rb) {
          const int r = rb * RPK + rq;
          bf16x8 aop = zero8, bop = zero8;
          if (co < COUT) aop = *reinterpret_cast<const bf16x8*>(&dzT[(co * TR + r) * TC + c0]);
          if (ci < CIN) {
            const bf16* src = &hT[(ci * LH + r + dy) * LW + c0 + dx];
#pragma unroll
            for (int k = 0; k < 8; ++k) bop[k] = src[k];
          }
          acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop, bop, acc[i], 0, 0, 0);
        }
      }
    }
  }
  // partial gradients of this block: [co][ci][tap]
  float* pw = part + (size_t)blockIdx.x * cout_real * cin_real * 9;
#pragma unroll
  for (int i = 0; i < PERW; ++i) {
    const int combo = wave + 4 * i;
    if (combo < NCOMBO) {
      const int tap = combo / (MB * NB), cb = (combo / NB) % MB, nb = combo % NB;
      const int ci = nb * 16 + l16;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int co = cb * 16 + kq * 4 + e;
        if (co < cout_real && ci < cin_real) pw[((size_t)co * cin_real + ci) * 9 + tap] = acc[i][e];
      }
    }
  }
  if (threadIdx.x < cout_real) partb[(size_t)blockIdx.x * cout_real + threadIdx.x] = bsum;
}

// fixed-order sum of the per-block partial gradients
__global__ void k_wgrad_reduce(const float* __restrict__ part, const float* __restrict__ partb, int nblk, int nw,
                               int nb, float* __restrict__ gw, float* __restrict__ gb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nw) {
    float s = 0.f;
    for (int b = 0; b < nblk; ++b) s += part[(size_t)b * nw + i];
    gw[i] = s;
  } else if (i < nw + nb) {
    const int k = i - nw;
    float s = 0.f;
    for (int b = 0; b < nblk; ++b) s += partb[(size_t)b * nb + k];
    gb[k] = s;
  }
}

// packed BF16 weights for k_conv: lane order of the A operand.  flip = 0: the layer
// itself (out Co, in Ci); flip = 1: its adjoint (out Ci, in Co, taps mirrored).
__global__ void k_pack(const float* __restrict__ Wm, int Co, int Ci, int flip, int cin_store, int kb_count,
                       int mb_count, bf16* __restrict__ out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int total = mb_count * kb_count * 64 * 8;
  if (idx >= total) return;
  const int e = idx & 7, lane = (idx >> 3) & 63, kbcb = idx >> 9;
  const int kb = kbcb % kb_count, cb = kbcb / kb_count;
  const int co = cb * 16 + (lane & 15);
  const int k = kb * 32 + 8 * (lane >> 4) + e;
  const int tap = k / cin_store, ci = k % cin_store;
  float v = 0.f;
  if (tap < 9) {
    if (!flip) {
      if (co < Co && ci < Ci) v = Wm[((size_t)co * Ci + ci) * 9 + tap];
    } else {
      if (co < Ci && ci < Co) v = Wm[((size_t)ci * Ci + co) * 9 + (8 - tap)];
    }
  }
  out[idx] = (bf16)v;
}

// network input: channels (log(f/mean f), log(g/mean g), 0 x 6)
// means of f and g per sample: MEAN_BLOCKS partial sums per field (each a contiguous
// chunk, coalesced), then a fixed-order fold, so the result does not depend on timing
constexpr int MEAN_BLOCKS = CNN_MEAN_PARTS;
// sum of chunk blockIdx.x of x[0..total) (256 threads; thread 0 holds the result)
__device__ double chunk_sum(const double* __restrict__ x, size_t total) {
  const size_t chunk = (total + MEAN_BLOCKS - 1) / MEAN_BLOCKS;
  const size_t lo = blockIdx.x * chunk, hi = lo + chunk < total ? lo + chunk : total;
  __shared__ double red[256];
  double a = 0.0;
  for (size_t i = lo + threadIdx.x; i < hi; i += 256) a += x[i];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  return red[0];
}

__global__ void k_mean_partials(const double* __restrict__ f, const double* __restrict__ g, int n,
                                double* __restrict__ part) {
  const int field = blockIdx.y, s = field >> 1;
  const double* x = ((field & 1) ? g : f) + (size_t)s * n * n;
  const double v = chunk_sum(x, (size_t)n * n);
  if (threadIdx.x == 0) part[(size_t)field * MEAN_BLOCKS + blockIdx.x] = v;
}

__global__ void k_mean_fold(const double* __restrict__ part, int nfields, double inv_count,
                            double* __restrict__ means) {
  const int field = blockIdx.x * blockDim.x + threadIdx.x;
  if (field >= nfields) return;
  double a = 0.0;
  for (int b = 0; b < MEAN_BLOCKS; ++b) a += part[(size_t)field * MEAN_BLOCKS + b];
  means[field] = a * inv_count;
}

__global__ void k_input(const double* __restrict__ f, const double* __restrict__ g, const double* __restrict__ means,
                        int batch, int n, bf16x8* __restrict__ out) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t total = (size_t)batch * n * n;
  if (i >= total) return;
  const int s = (int)(i / ((size_t)n * n));
  bf16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
  v[0] = (bf16)(float)log(f[i] / means[2 * s]);
  v[1] = (bf16)(float)log(g[i] / means[2 * s + 1]);
  out[i] = v;
}

// MSE loss: dz = 2 (c - t) / count into channel 0 of an 8-channel BF16 tensor
__global__ void k_mse(const float* __restrict__ c, const float* __restrict__ t, size_t count, float inv_count,
                      bf16x8* __restrict__ dz, float* __restrict__ part) {
  __shared__ float red[256];
  float a = 0.f;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (size_t)gridDim.x * 256) {
    const float d = c[i] - t[i];
    a += d * d;
    bf16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
    v[0] = (bf16)(2.f * d * inv_count);
    dz[i] = v;
  }
  red[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_sum(const float* __restrict__ part, int n, float scale, float* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    float s = 0.f;
    for (int i = 0; i < n; ++i) s += part[i];
    *out = s * scale;
  }
}

// Adam (Kingma and Ba): bias corrections c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t)
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       int count, float lr, float b1, float b2, float c1, float c2, float eps) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// training target: the fourth-order difference Laplacian of FP64 fields u, minus
// log(f / mean f) - log(g / mean g) when f and g are given (the network then learns
// the correction to the linearised equation)
__global__ void k_target(const double* __restrict__ u, const double* __restrict__ f, const double* __restrict__ g,
                         const double* __restrict__ means, int batch, int n, float* __restrict__ out) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)batch * n * n) return;
  const size_t s = i / ((size_t)n * n), base = s * n * n;
  const int r = (int)((i / n) % n), c = (int)(i % n);
  auto U = [&](int a, int b) { return u[base + (size_t)wrap(r + a, n) * n + wrap(c + b, n)]; };
  const double lap = -U(-2, 0) + 16.0 * U(-1, 0) - 60.0 * U(0, 0) + 16.0 * U(1, 0) - U(2, 0) - U(0, -2) +
                     16.0 * U(0, -1) + 16.0 * U(0, 1) - U(0, 2);
  double t = lap * (double)n * n / 12.0;
  if (f) t -= log(f[i] / means[2 * s]) - log(g[i] / means[2 * s + 1]);
  out[i] = (float)t;
}

// The warm start of a batch of pairs, every launch covering all of them
// (blockIdx.y = pair; the pairs' buffers come as device arrays of pointers).

// densities at the network's resolution: copied (n = n_net) or restricted by full
// weighting (n = 2 n_net; fine node 2a maps to coarse node a); blockIdx.z = 0 f, 1 g
__global__ void k_gather_inputs(const double* const* __restrict__ f, const double* const* __restrict__ g, int n,
                                int nr, double* __restrict__ fx, double* __restrict__ gx) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nr * nr) return;
  const int k = blockIdx.y;
  const double* x = (blockIdx.z ? g : f)[k];
  double* y = (blockIdx.z ? gx : fx) + (size_t)k * nr * nr;
  if (n == nr) {
    y[i] = x[i];
    return;
  }
  const int a = i / nr, b = i % nr;
  const double w[3] = {0.25, 0.5, 0.25};
  double s = 0.0;
  for (int p = -1; p <= 1; ++p)
    for (int q = -1; q <= 1; ++q) s += w[p + 1] * w[q + 1] * x[(size_t)wrap(2 * a + p, n) * n + wrap(2 * b + q, n)];
  y[i] = s;
}

// partial sums of the full-resolution densities (folded by k_mean_fold)
__global__ void k_mean_partials_ptr(const double* const* __restrict__ f, const double* const* __restrict__ g, int n,
                                    double* __restrict__ part) {
  const int field = blockIdx.y;
  const double* x = ((field & 1) ? g : f)[field >> 1];
  const double v = chunk_sum(x, (size_t)n * n);
  if (threadIdx.x == 0) part[(size_t)field * MEAN_BLOCKS + blockIdx.x] = v;
}

// the head's input at full resolution: c (prolonged bilinearly, periodic, if n = 2 n_net)
// plus log(f / mean f) - log(g / mean g)
__global__ void k_head_input(const float* __restrict__ c, const double* const* __restrict__ f,
                             const double* const* __restrict__ g, const double* __restrict__ means, int n, int nr,
                             float* __restrict__ out) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)n * n) return;
  const int k = blockIdx.y;
  const float* ck = c + (size_t)k * nr * nr;
  float cv;
  if (n == nr) {
    cv = ck[i];
  } else {
    const int r = (int)(i / n), col = (int)(i % n);
    const int a0 = r >> 1, b0 = col >> 1, a1 = wrap(a0 + (r & 1), nr), b1 = wrap(b0 + (col & 1), nr);
    cv = 0.25f * (ck[a0 * nr + b0] + ck[a1 * nr + b0] + ck[a0 * nr + b1] + ck[a1 * nr + b1]);
  }
  out[(size_t)k * n * n + i] =
      (float)((double)cv + log(f[k][i] / means[2 * k]) - log(g[k][i] / means[2 * k + 1]));
}

// the pairs' potentials (contiguous FP32) into the callers' FP64 outputs
__global__ void k_scatter_double(const float* __restrict__ x, size_t nn, double* const* __restrict__ out) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nn) out[blockIdx.y][i] = (double)x[(size_t)blockIdx.y * nn + i];
}

inline unsigned nblocks(size_t count, int bs) { return (unsigned)((count + bs - 1) / bs); }

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void cnn_conv(int cin, int cout_pad, int mode, const void* in, const void* wp, const float* bias, const void* mask,
              void* out_bf, float* out_f, int batch, int H, int W, int dil, hipStream_t st) {
  dim3 grid((H / 16) * (W / 16), 1, batch), block(256);
  const bf16* i = (const bf16*)in;
  const bf16x8* w = (const bf16x8*)wp;
  const bf16* mk = (const bf16*)mask;
  bf16* ob = (bf16*)out_bf;
  if (cin == 8 && cout_pad == 32 && mode == CV_FWD_RELU)
    hipLaunchKernelGGL((k_conv<8, 32, CV_FWD_RELU>), grid, block, 0, st, i, w, bias, mk, ob, out_f, H, W, dil);
  else if (cin == 32 && cout_pad == 32 && mode == CV_FWD_RELU)
    hipLaunchKernelGGL((k_conv<32, 32, CV_FWD_RELU>), grid, block, 0, st, i, w, bias, mk, ob, out_f, H, W, dil);
  else if (cin == 32 && cout_pad == 16 && mode == CV_FWD_LAST)
    hipLaunchKernelGGL((k_conv<32, 16, CV_FWD_LAST>), grid, block, 0, st, i, w, bias, mk, ob, out_f, H, W, dil);
  else if (cin == 8 && cout_pad == 32 && mode == CV_BWD_DATA)
    hipLaunchKernelGGL((k_conv<8, 32, CV_BWD_DATA>), grid, block, 0, st, i, w, bias, mk, ob, out_f, H, W, dil);
  else if (cin == 32 && cout_pad == 32 && mode == CV_BWD_DATA)
    hipLaunchKernelGGL((k_conv<32, 32, CV_BWD_DATA>), grid, block, 0, st, i, w, bias, mk, ob, out_f, H, W, dil);
}

void cnn_wgrad(int cin, int cout, const void* h, const void* dz, int batch, int H, int W, int dil, int cout_real,
               int cin_real, float* part, float* partb, int nblk, float* gw, float* gb, hipStream_t st) {
  const bf16* hh = (const bf16*)h;
  const bf16* dd = (const bf16*)dz;
  if (cin == 8 && cout == 32)
    hipLaunchKernelGGL((k_conv_wgrad<8, 32>), dim3(nblk), dim3(256), 0, st, hh, dd, batch, H, W, dil, cout_real, cin_real,
                       part, partb);
  else if (cin == 32 && cout == 32)
    hipLaunchKernelGGL((k_conv_wgrad<32, 32>), dim3(nblk), dim3(256), 0, st, hh, dd, batch, H, W, dil, cout_real, cin_real,
                       part, partb);
  else if (cin == 32 && cout == 8)
    hipLaunchKernelGGL((k_conv_wgrad<32, 8>), dim3(nblk), dim3(256), 0, st, hh, dd, batch, H, W, dil, cout_real, cin_real,
                       part, partb);
  const int nw = cout_real * cin_real * 9;
  hipLaunchKernelGGL(k_wgrad_reduce, dim3(nblocks(nw + cout_real, 256)), dim3(256), 0, st, part, partb, nblk, nw,
                     cout_real, gw, gb);
}

void cnn_pack(const float* Wm, int Co, int Ci, int flip, int cin_store, int cout_pad, void* out, hipStream_t st) {
  const int kb = (9 * cin_store + 31) / 32, mb = cout_pad / 16;
  const int total = mb * kb * 64 * 8;
  hipLaunchKernelGGL(k_pack, dim3(nblocks(total, 256)), dim3(256), 0, st, Wm, Co, Ci, flip, cin_store, kb, mb,
                     (bf16*)out);
}

void cnn_means(const double* f, const double* g, int batch, int n, double* part, double* means, hipStream_t st) {
  hipLaunchKernelGGL(k_mean_partials, dim3(MEAN_BLOCKS, 2 * batch), dim3(256), 0, st, f, g, n, part);
  hipLaunchKernelGGL(k_mean_fold, dim3(nblocks(2 * batch, 64)), dim3(64), 0, st, part, 2 * batch,
                     1.0 / ((double)n * n), means);
}

void cnn_input(const double* f, const double* g, int batch, int n, double* part, double* means, void* x,
               hipStream_t st) {
  cnn_means(f, g, batch, n, part, means, st);
  hipLaunchKernelGGL(k_input, dim3(nblocks((size_t)batch * n * n, 256)), dim3(256), 0, st, f, g, means, batch, n,
                     (bf16x8*)x);
}

void cnn_mse(const float* c, const float* t, size_t count, void* dz, float* part, int nblk, float* loss, hipStream_t st) {
  hipLaunchKernelGGL(k_mse, dim3(nblk), dim3(256), 0, st, c, t, count, 1.0f / (float)count, (bf16x8*)dz, part);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(64), 0, st, part, nblk, 1.0f / (float)count, loss);
}

void cnn_adam(float* p, const float* g, float* m, float* v, int count, float lr, float b1, float b2, float c1, float c2,
              float eps, hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3(nblocks(count, 256)), dim3(256), 0, st, p, g, m, v, count, lr, b1, b2, c1, c2, eps);
}

void cnn_target(const double* u, const double* f, const double* g, int batch, int n, double* part, double* means,
                float* out, hipStream_t st) {
  if (f) cnn_means(f, g, batch, n, part, means, st);
  hipLaunchKernelGGL(k_target, dim3(nblocks((size_t)batch * n * n, 256)), dim3(256), 0, st, u, f, g, means, batch, n,
                     out);
}

void cnn_gather_inputs(const double* const* f, const double* const* g, int batch, int n, int nr, double* fx,
                       double* gx, hipStream_t st) {
  hipLaunchKernelGGL(k_gather_inputs, dim3(nblocks((size_t)nr * nr, 256), batch, 2), dim3(256), 0, st, f, g, n, nr,
                     fx, gx);
}

void cnn_full_means(const double* const* f, const double* const* g, int batch, int n, double* part, double* means,
                    hipStream_t st) {
  hipLaunchKernelGGL(k_mean_partials_ptr, dim3(MEAN_BLOCKS, 2 * batch), dim3(256), 0, st, f, g, n, part);
  hipLaunchKernelGGL(k_mean_fold, dim3(nblocks(2 * batch, 64)), dim3(64), 0, st, part, 2 * batch,
                     1.0 / ((double)n * n), means);
}

void cnn_head_input(const float* c, const double* const* f, const double* const* g, const double* means, int batch,
                    int n, int nr, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_head_input, dim3(nblocks((size_t)n * n, 256), batch), dim3(256), 0, st, c, f, g, means, n, nr,
                     out);
}

void cnn_scatter_double(const float* x, int batch, size_t nn, double* const* out, hipStream_t st) {
  hipLaunchKernelGGL(k_scatter_double, dim3(nblocks(nn, 256), batch), dim3(256), 0, st, x, nn, out);
}
