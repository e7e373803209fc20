// Launchers of the warm-start network kernels (k_cnn.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

enum : int { CV_FWD_RELU = 0, CV_FWD_LAST = 1, CV_BWD_DATA = 2 };

// dil: dilation of the 3x3 taps (H and W multiples of 16 * dil)
void cnn_conv(int cin, int cout_pad, int mode, const void* in, const void* wp, const float* bias, const void* mask,
              void* out_bf, float* out_f, int batch, int H, int W, int dil, hipStream_t st);
void cnn_wgrad(int cin, int cout, const void* h, const void* dz, int batch, int H, int W, int dil, int cout_real,
               int cin_real, float* part, float* partb, int nblk, float* gw, float* gb, hipStream_t st);
void cnn_pack(const float* Wm, int Co, int Ci, int flip, int cin_store, int cout_pad, void* out, hipStream_t st);
constexpr int CNN_MEAN_PARTS = 64;  // partial sums per field in the mean reductions
void cnn_means(const double* f, const double* g, int batch, int n, double* part, double* means, hipStream_t st);
void cnn_input(const double* f, const double* g, int batch, int n, double* part, double* means, void* x,
               hipStream_t st);
void cnn_mse(const float* c, const float* t, size_t count, void* dz, float* part, int nblk, float* loss, hipStream_t st);
void cnn_adam(float* p, const float* g, float* m, float* v, int count, float lr, float b1, float b2, float c1, float c2,
              float eps, hipStream_t st);
void cnn_target(const double* u, const double* f, const double* g, int batch, int n, double* part, double* means,
                float* out, hipStream_t st);
// warm start of a batch: f, g, out are device arrays of the pairs' device pointers
void cnn_gather_inputs(const double* const* f, const double* const* g, int batch, int n, int nr, double* fx,
                       double* gx, hipStream_t st);
void cnn_full_means(const double* const* f, const double* const* g, int batch, int n, double* part, double* means,
                    hipStream_t st);
void cnn_head_input(const float* c, const double* const* f, const double* const* g, const double* means, int batch,
                    int n, int nr, float* out, hipStream_t st);
void cnn_scatter_double(const float* x, int batch, size_t nn, double* const* out, hipStream_t st);
