// C ABI of the warm-start network: parameters and Adam state, packed BF16 weights,
// activation buffers, forward, backward, training step and the batched warm start.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "cnn.h"
#include "ma_ot.h"
#include "plan_internal.h"

namespace {

struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
  int ensure(size_t b) {
    if (b <= bytes) return MA_OK;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    if (hipMalloc(&p, b) != hipSuccess) return MA_ENOMEM;
    bytes = b;
    return MA_OK;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
};

constexpr int WGRAD_BLOCKS = 256;

}  // namespace

struct ma_cnn {
  int L = 0, C = 0, n = 0, max_batch = 0;
  std::vector<long> w_off, b_off;  // offsets of W_l and b_l in the flat parameter array
  std::vector<int> cin, cout;      // real channel counts per layer
  std::vector<int> dil;            // dilation of each layer's taps
  long count = 0;
  float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr;
  long step = 0;
  std::vector<Buf> wfwd, wbwd;     // packed BF16 weights per layer
  std::vector<Buf> act;            // h_1 .. h_{L-1}, BF16 32 channels
  Buf c, dz_last, dzA, dzB, part, partb, lpart, loss, means, mpart, fx, gx, cbuf, clin, theta, ptrs;
  ma_plan* head = nullptr;         // fourth-order inverse Laplacian for the warm-start head
  int head_n = 0;
};

namespace {

#define TRY(x)                     \
  do {                             \
    int _e = (x);                  \
    if (_e) return _e;             \
  } while (0)
#define HIPTRY(x)                            \
  do {                                       \
    if ((x) != hipSuccess) return MA_EHIP;   \
  } while (0)

int pack_all(ma_cnn* N, hipStream_t st) {
  for (int l = 0; l < N->L; ++l) {
    const int cin_store = (l == 0) ? 8 : 32;
    const int cout_pad = (l == N->L - 1) ? 16 : 32;
    cnn_pack(N->params + N->w_off[l], N->cout[l], N->cin[l], 0, cin_store, cout_pad, N->wfwd[l].p, st);
    if (l > 0) {  // adjoint: input = this layer's output gradient (8 stored channels for the last layer)
      const int cin_b = (l == N->L - 1) ? 8 : 32;
      cnn_pack(N->params + N->w_off[l], N->cout[l], N->cin[l], 1, cin_b, 32, N->wbwd[l].p, st);
    }
  }
  return hipGetLastError() == hipSuccess ? MA_OK : MA_EHIP;
}

int ensure_batch(ma_cnn* N, int batch) {
  const size_t px = (size_t)batch * N->n * N->n;
  for (auto& a : N->act) TRY(a.ensure(px * 32 * 2));
  TRY(N->c.ensure(px * 4));
  TRY(N->dz_last.ensure(px * 8 * 2));
  TRY(N->dzA.ensure(px * 32 * 2));
  TRY(N->dzB.ensure(px * 32 * 2));
  TRY(N->part.ensure((size_t)WGRAD_BLOCKS * 32 * 32 * 9 * 4));
  TRY(N->partb.ensure((size_t)WGRAD_BLOCKS * 32 * 4));
  TRY(N->lpart.ensure(1024 * 4));
  TRY(N->loss.ensure(64));
  TRY(N->means.ensure((size_t)2 * batch * 8));
  return MA_OK;
}

void forward(ma_cnn* N, const void* x, int batch, hipStream_t st) {
  const int n = N->n;
  for (int l = 0; l < N->L; ++l) {
    const void* in = (l == 0) ? x : N->act[l - 1].p;
    const float* bias = N->params + N->b_off[l];
    if (l < N->L - 1)
      cnn_conv(l == 0 ? 8 : 32, 32, CV_FWD_RELU, in, N->wfwd[l].p, bias, nullptr, N->act[l].p, nullptr, batch, n, n,
               N->dil[l], st);
    else
      cnn_conv(32, 16, CV_FWD_LAST, in, N->wfwd[l].p, bias, nullptr, nullptr, (float*)N->c.p, batch, n, n,
               N->dil[l], st);
  }
}

// gradients of the MSE into N->grads; the loss into N->loss (device)
void backward(ma_cnn* N, const void* x, const float* target, int batch, hipStream_t st) {
  const int n = N->n;
  const size_t count = (size_t)batch * n * n;
  cnn_mse((const float*)N->c.p, target, count, N->dz_last.p, (float*)N->lpart.p, 512, (float*)N->loss.p, st);
  const void* dz = N->dz_last.p;
  Buf* outs[2] = {&N->dzA, &N->dzB};
  for (int l = N->L - 1; l >= 0; --l) {
    const void* h = (l == 0) ? x : N->act[l - 1].p;
    const int cin_store = (l == 0) ? 8 : 32, dz_store = (l == N->L - 1) ? 8 : 32;
    cnn_wgrad(cin_store, dz_store, h, dz, batch, n, n, N->dil[l], N->cout[l], N->cin[l], (float*)N->part.p,
              (float*)N->partb.p, WGRAD_BLOCKS, N->grads + N->w_off[l], N->grads + N->b_off[l], st);
    if (l > 0) {
      void* out = outs[l & 1]->p;
      cnn_conv(dz_store, 32, CV_BWD_DATA, dz, N->wbwd[l].p, nullptr, N->act[l - 1].p, out, nullptr, batch, n, n,
               N->dil[l], st);
      dz = out;
    }
  }
}

}  // namespace

extern "C" {

int ma_cnn_create(int layers, int channels, int n_net, int max_batch, const int* dilations, ma_cnn** out) {
  if (!out) return MA_EINVAL;
  *out = nullptr;
  if (layers < 2 || channels != 32 || n_net < 16 || n_net % 16 || max_batch < 1) return MA_EINVAL;
  for (int l = 0; dilations && l < layers; ++l)
    if (dilations[l] < 1 || n_net % (16 * dilations[l])) return MA_EINVAL;
  ma_cnn* N = new ma_cnn();
  N->dil.assign(layers, 1);
  for (int l = 0; dilations && l < layers; ++l) N->dil[l] = dilations[l];
  N->L = layers;
  N->C = channels;
  N->n = n_net;
  N->max_batch = max_batch;
  long off = 0;
  for (int l = 0; l < layers; ++l) {
    const int ci = (l == 0) ? 2 : channels, co = (l == layers - 1) ? 1 : channels;
    N->cin.push_back(ci);
    N->cout.push_back(co);
    N->w_off.push_back(off);
    off += (long)co * ci * 9;
    N->b_off.push_back(off);
    off += co;
  }
  N->count = off;
  const size_t pb = (size_t)off * 4;
  if (hipMalloc(&N->params, pb) != hipSuccess || hipMalloc(&N->grads, pb) != hipSuccess ||
      hipMalloc(&N->m, pb) != hipSuccess || hipMalloc(&N->v, pb) != hipSuccess) {
    ma_cnn_destroy(N);
    return MA_ENOMEM;
  }
  if (hipMemset(N->params, 0, pb) != hipSuccess || hipMemset(N->m, 0, pb) != hipSuccess ||
      hipMemset(N->v, 0, pb) != hipSuccess) {
    ma_cnn_destroy(N);
    return MA_EHIP;
  }
  N->wfwd.resize(layers);
  N->wbwd.resize(layers);
  N->act.resize(layers - 1);
  for (int l = 0; l < layers; ++l) {
    const int kb = (9 * ((l == 0) ? 8 : 32) + 31) / 32, mb = (l == layers - 1) ? 1 : 2;
    if (N->wfwd[l].ensure((size_t)mb * kb * 64 * 8 * 2)) {
      ma_cnn_destroy(N);
      return MA_ENOMEM;
    }
    if (l > 0) {
      const int kbb = (9 * ((l == layers - 1) ? 8 : 32) + 31) / 32;
      if (N->wbwd[l].ensure((size_t)2 * kbb * 64 * 8 * 2)) {
        ma_cnn_destroy(N);
        return MA_ENOMEM;
      }
    }
  }
  if (ensure_batch(N, max_batch)) {
    ma_cnn_destroy(N);
    return MA_ENOMEM;
  }
  if (pack_all(N, nullptr) || hipDeviceSynchronize() != hipSuccess) {
    ma_cnn_destroy(N);
    return MA_EHIP;
  }
  *out = N;
  return MA_OK;
}

void ma_cnn_destroy(ma_cnn* N) {
  if (!N) return;
  for (float* p : {N->params, N->grads, N->m, N->v})
    if (p) (void)hipFree(p);
  for (auto& b : N->wfwd) b.release();
  for (auto& b : N->wbwd) b.release();
  for (auto& b : N->act) b.release();
  for (Buf* b : {&N->c, &N->dz_last, &N->dzA, &N->dzB, &N->part, &N->partb, &N->lpart, &N->loss, &N->means, &N->mpart, &N->fx,
                 &N->gx, &N->cbuf, &N->clin, &N->theta, &N->ptrs})
    b->release();
  if (N->head) ma_plan_destroy(N->head);
  delete N;
}

long ma_cnn_param_count(const ma_cnn* N) { return N ? N->count : 0; }

int ma_cnn_set_params(ma_cnn* N, const float* host, long count) {
  if (!N || !host || count != N->count) return MA_EINVAL;
  const size_t pb = (size_t)count * 4;
  HIPTRY(hipMemcpy(N->params, host, pb, hipMemcpyHostToDevice));
  HIPTRY(hipMemset(N->m, 0, pb));
  HIPTRY(hipMemset(N->v, 0, pb));
  N->step = 0;
  TRY(pack_all(N, nullptr));
  HIPTRY(hipDeviceSynchronize());
  return MA_OK;
}

int ma_cnn_get_params(const ma_cnn* N, float* host, long count) {
  if (!N || !host || count != N->count) return MA_EINVAL;
  HIPTRY(hipDeviceSynchronize());
  HIPTRY(hipMemcpy(host, N->params, (size_t)count * 4, hipMemcpyDeviceToHost));
  return MA_OK;
}

int ma_cnn_prepare_input(ma_cnn* N, const double* f, const double* g, int batch, void* x, void* stream) {
  if (!N || !f || !g || !x || batch < 1) return MA_EINVAL;
  TRY(N->means.ensure((size_t)2 * batch * 8));
  TRY(N->mpart.ensure((size_t)2 * batch * CNN_MEAN_PARTS * 8));
  cnn_input(f, g, batch, N->n, (double*)N->mpart.p, (double*)N->means.p, x, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? MA_OK : MA_EHIP;
}

int ma_cnn_target(ma_cnn* N, const double* psi, const double* f, const double* g, int batch, int n, float* target,
                  void* stream) {
  if (!N || !psi || !target || batch < 1 || n < 8 || (!f) != (!g)) return MA_EINVAL;
  TRY(N->means.ensure((size_t)2 * batch * 8));
  TRY(N->mpart.ensure((size_t)2 * batch * CNN_MEAN_PARTS * 8));
  cnn_target(psi, f, g, batch, n, (double*)N->mpart.p, (double*)N->means.p, target, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? MA_OK : MA_EHIP;
}

int ma_cnn_forward(ma_cnn* N, const void* x, int batch, float* c, void* stream) {
  if (!N || !x || !c || batch < 1 || batch > N->max_batch) return MA_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  forward(N, x, batch, st);
  HIPTRY(hipMemcpyAsync(c, N->c.p, (size_t)batch * N->n * N->n * 4, hipMemcpyDeviceToDevice, st));
  return hipGetLastError() == hipSuccess ? MA_OK : MA_EHIP;
}

int ma_cnn_gradients(ma_cnn* N, const void* x, const float* target, int batch, float* grads, float* loss,
                     void* stream) {
  if (!N || !x || !target || batch < 1 || batch > N->max_batch) return MA_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  forward(N, x, batch, st);
  backward(N, x, target, batch, st);
  if (grads) HIPTRY(hipMemcpyAsync(grads, N->grads, (size_t)N->count * 4, hipMemcpyDeviceToDevice, st));
  if (loss) HIPTRY(hipMemcpyAsync(loss, N->loss.p, 4, hipMemcpyDeviceToHost, st));
  HIPTRY(hipStreamSynchronize(st));
  return MA_OK;
}

int ma_cnn_train_step(ma_cnn* N, const void* x, const float* target, int batch, float lr, float* loss,
                      void* stream) {
  if (!N || !x || !target || batch < 1 || batch > N->max_batch || !(lr > 0.f)) return MA_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  forward(N, x, batch, st);
  backward(N, x, target, batch, st);
  N->step++;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, (double)N->step)));
  const float c2 = (float)(1.0 / (1.0 - std::pow(0.999, (double)N->step)));
  cnn_adam(N->params, N->grads, N->m, N->v, (int)N->count, lr, b1, b2, c1, c2, 1e-8f, st);
  TRY(pack_all(N, st));
  if (loss) {
    HIPTRY(hipMemcpyAsync(loss, N->loss.p, 4, hipMemcpyDeviceToHost, st));
    HIPTRY(hipStreamSynchronize(st));
  }
  return hipGetLastError() == hipSuccess ? MA_OK : MA_EHIP;
}

int ma_cnn_warm_start(ma_cnn* N, int npairs, int n, const double* const* f, const double* const* g,
                      double* const* psi0, void* stream) {
  if (!N || npairs < 1 || !f || !g || !psi0) return MA_EINVAL;
  const int nr = N->n;
  if (n != nr && n != 2 * nr) return MA_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  if (!N->head || N->head_n != n) {
    if (N->head) ma_plan_destroy(N->head);
    N->head = nullptr;
    ma_options o;
    ma_options_default(&o);
    o.symbol = MA_SYMBOL_FD4;
    o.gmres_m = 1;  // the head applies Lbar^{-1} only: one basis vector of workspace
    TRY(ma_plan_create(n, N->max_batch, &o, &N->head));
    N->head_n = n;
  }
  const int B = N->max_batch;
  const size_t pr = (size_t)nr * nr, pn = (size_t)n * n;
  const int nbatch = (npairs + B - 1) / B;
  TRY(N->fx.ensure((size_t)B * pr * 8));
  TRY(N->gx.ensure((size_t)B * pr * 8));
  TRY(N->cbuf.ensure((size_t)B * pr * 2 * 8));  // network input (8 BF16 channels = 16 bytes per pixel)
  TRY(N->clin.ensure((size_t)B * pn * 4));
  TRY(N->theta.ensure((size_t)B * pn * 4));
  TRY(N->means.ensure((size_t)2 * B * 8));
  TRY(N->mpart.ensure((size_t)2 * B * CNN_MEAN_PARTS * 8));
  TRY(N->ptrs.ensure((size_t)nbatch * 3 * B * sizeof(void*)));  // one region per batch: no reuse in a call
  const double lap[5] = {1.0, 0.0, 1.0, 0.0, 0.0};  // averaged operator = the Laplacian
  std::vector<const void*> hp((size_t)nbatch * 3 * B, nullptr);
  for (int q = 0; q < npairs; ++q) {
    const size_t base = (size_t)(q / B) * 3 * B, k = q % B;
    hp[base + k] = f[q];
    hp[base + B + k] = g[q];
    hp[base + 2 * B + k] = psi0[q];
  }
  HIPTRY(hipMemcpyAsync(N->ptrs.p, hp.data(), hp.size() * sizeof(void*), hipMemcpyHostToDevice, st));
  std::vector<const float*> sig(B);
  std::vector<float*> th(B);
  for (int q0 = 0; q0 < npairs; q0 += B) {
    const int b = (npairs - q0 < B) ? npairs - q0 : B;
    const void* const* pb = (const void* const*)N->ptrs.p + (size_t)(q0 / B) * 3 * B;
    const double* const* fp = (const double* const*)pb;
    const double* const* gp = (const double* const*)(pb + B);
    double* const* op = (double* const*)(pb + 2 * B);
    cnn_gather_inputs(fp, gp, b, n, nr, (double*)N->fx.p, (double*)N->gx.p, st);
    TRY(ma_cnn_prepare_input(N, (const double*)N->fx.p, (const double*)N->gx.p, b, N->cbuf.p, stream));
    forward(N, N->cbuf.p, b, st);
    cnn_full_means(fp, gp, b, n, (double*)N->mpart.p, (double*)N->means.p, st);
    cnn_head_input((const float*)N->c.p, fp, gp, (const double*)N->means.p, b, n, nr, (float*)N->clin.p, st);
    for (int k = 0; k < b; ++k) {
      sig[k] = (const float*)N->clin.p + (size_t)k * pn;
      th[k] = (float*)N->theta.p + (size_t)k * pn;
    }
    TRY(plan_lbar_inverse_many(N->head, n, b, sig.data(), lap, th.data(), st));
    cnn_scatter_double((const float*)N->theta.p, b, pn, op, st);
  }
  return hipGetLastError() == hipSuccess ? MA_OK : MA_EHIP;
}

}  // extern "C"
