// The damped Newton method in three dimensions: device structures and launchers.
//
// One pair on an N x N x N grid, u[i][j][k] with k contiguous (axis a is the coordinate
// x_{a+1}).  The residual and the Newton update run in FP64, Strain's operator in FP32
// (three forward line transforms, the averaged symbol, nine derived inverse transforms
// folded into 3 + 6 + 5 complex line transforms), the Arnoldi bookkeeping in FP64 on
// the device.  The host drives the Newton steps and the GMRES cycles and reads one small
// summary per Newton step or cycle.
#pragma once
#include <hip/hip_runtime.h>

#define MA3_MMAX 30          // largest GMRES restart length
#define MA3_NPART 20         // partial sums per residual block
#define MA3_BLOCK 256

// coefficient planes: a11, a22, a33, a12, a13, a23, b1, b2, b3
struct Desc3 {
  int n, pad;
  const double* f_in;
  const double* g_in;
  double* u;      // n^3 iterate
  double* f;      // n^3 f scaled to mean one
  double* g;      // n^3 g scaled to mean one
  float4* gg;     // n^3 fourth-order gradient of g (x, y, z; w unused)
  float* coef;    // 9 n^3
  float* r;       // n^3 f - f_n (the translation constant is added by its readers)
  double* theta;  // n^3 last correction
  float* x;       // n^3 GMRES solution accumulated over restarts
  float* V;       // (m + 1) n^3 Krylov vectors, unnormalised (v_l = vscale[l] V[l])
  float2* S;      // n^3 complex: forward transforms
  float2* T;      // 3 n^3 complex: after the inverse transform along x1
  float2* U;      // 6 n^3 complex: after the inverse transforms along x2
  double* part;   // per-block partial sums
  const float2* tw;  // tw[m] = exp(-2 pi i m / n)
  const float2* mt;  // per wavenumber index: (Im of the first-derivative multiplier, second-derivative multiplier)
};

struct State3 {
  int gm_running, gm_restart, gm_cycle, gm_k, gmres_iters, m, max_restarts, pad;
  double bnorm, gm_target, gmres_tol, mass_c, tau;
  double abar[9];
  double vscale[MA3_MMAX + 1];
  double Hm[(MA3_MMAX + 1) * MA3_MMAX];  // column-major: Hm[j * (MMAX + 1) + i]
  double cs[MA3_MMAX], sn[MA3_MMAX], gv[MA3_MMAX + 1], y[MA3_MMAX + 1], q[MA3_MMAX + 1];
  // residual summary: sum f_n, sum r, sum r^2, Simpson sums of the 9 coefficients,
  // sum |grad u|^2 f, sum u, min det, min M11, min of the 2 x 2 leading minor, max r,
  // min r, count of non-finite values
  double sums[MA3_NPART];
  double mean_f, mean_g;
};

// operator passes (launch dispatch over the compiled grid sizes)
enum : int {
  P3_MATVEC = 0,  // Krylov product: nine derived transforms, combination, inner products
  P3_THETA = 1,   // theta = Lbar^{-1} x: one derived transform, u += theta
  P3_STEP = 2,    // single-step use: Lbar^{-1} of an input into x
};
enum : int { V3_INIT = 0, V3_ARNOLDI = 1, V3_RECOVER = 2 };

bool n3_supported(int n);
int k3_blocks(int n);      // blocks of the elementwise / stencil kernels
int k3_dot_blocks(int n);  // blocks of the last operator pass (its inner-product partials)
// scaled f, g (by the means the state holds, or those the kernels compute first when
// `scale`), the gradient of g, u = 0
void k3_setup(const Desc3& d, State3* s, bool scale, hipStream_t st);
void k3_residual(const Desc3& d, State3* s, int op_mode, hipStream_t st);
void k3_update(const Desc3& d, double a, hipStream_t st);
void k3_outputs(const Desc3& d, const State3* s, double* psi, double* map, hipStream_t st);
// Krylov vector build (mode V3_*): V[0] from r (init, then its norm), V[jn] from w minus
// the projections (Arnoldi, then ||V[jn]|| and the rotations), or x + sum y V (recovery,
// into the x plane)
void k3_vector(const Desc3& d, State3* s, int mode, int jn, hipStream_t st);
// the operator passes (mode P3_*): P1 on V[j] (matvec) or x, then P2, then P3..P5
void k3_first_pass(const Desc3& d, State3* s, int mode, int j, hipStream_t st);
void k3_forward_rest(const Desc3& d, State3* s, int mode, hipStream_t st);
void k3_inverse(const Desc3& d, State3* s, int mode, int j, hipStream_t st);
// x += sum y V and V[0] = the cycle's residual; the next cycle begins
void k3_restart(const Desc3& d, State3* s, hipStream_t st);
