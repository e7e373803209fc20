/*
 * ma_ot.h -- C ABI of the MI355X damped-Newton Monge-Ampere optimal-transport solver.
 *
 * Method: Saumier, Agueh, Khouider, "An efficient numerical algorithm for the L2
 * optimal transport problem with applications to image processing" (2010).
 * For 1-periodic probability densities f, g on the unit torus the library solves
 * the Monge-Ampere equation g(x + grad u) det(I + D^2 u) = f  (Section 3.1, eq. ma2)
 * for the mean-zero periodic potential u with |x|^2/2 + u convex, by the damped
 * Newton iteration of eq. (linma), each linear step solved by Strain's FFT method
 * with restarted GMRES(m) (Section 4.2) or, as an option, by the finite-difference
 * system of Section 4.1 with BiCG.  The optimal map is x + grad u
 * (Theorem CE1 and Section 5.2).
 *
 * Conventions shared by every entry point
 *   - Grids are N x N, h = 1/N, node (i, j) at (x1, x2) = (i h, j h)  (Section 4).
 *     Arrays are row-major [i][j]: i indexes x1, j (contiguous) indexes x2.
 *   - Field pointers are DEVICE pointers (HIP global memory) unless marked host.
 *     The caller owns every pointer it passes; the library never frees them and
 *     never writes to inputs.  Outputs are written on return codes >= 0.
 *   - `stream` is a hipStream_t cast to void* (NULL = the default stream).  Calls
 *     are stream-ordered; the solve entry points synchronise `stream` before they
 *     return because their Newton loop reads per-pair status on the host.
 *   - Supported N: even, 16 <= N <= 2048, N a multiple of 16, N = 2^a 3^b.
 *   - Return codes: MA_OK (0); soft failures > 0 with the best iterate written;
 *     hard failures < 0 with nothing written.  ma_strerror() names each code.
 *   - One plan serves one stream at a time; plans are not thread-safe.
 */
#ifndef MA_OT_H
#define MA_OT_H

#ifdef __cplusplus
extern "C" {
#endif

#define MA_OT_ABI_VERSION 12

/* return / status codes */
#define MA_OK 0           /* converged: rms residual <= tol                           */
#define MA_ENOCONV 1      /* max Newton iterations, or step halving exhausted         */
#define MA_ENONCONVEX 2   /* det(I + D^2 u) <= 0 or trace <= 0 at an iterate (Sec. 3.3) */
#define MA_ENAN 3         /* a non-finite residual                                    */
#define MA_EINVAL (-1)    /* bad argument: N, tau < 1, tol <= 0, density <= 0 or NaN  */
#define MA_ENOMEM (-2)    /* device allocation failed                                 */
#define MA_EHIP (-3)      /* a HIP runtime call failed                                */

/* interpolation of g and grad g at x + grad u (Section 4) */
#define MA_INTERP_BILINEAR 0
#define MA_INTERP_NEAREST 1
/* linear operator: full eq. (linearmaeq), or without the grad g term (Remarks, Sec. 3.3) */
#define MA_OP_FULL 0
#define MA_OP_NO_DRIFT 1
/* damping: fixed tau (eq. linma); or halve the step (double tau) while the trial
 * iterate is non-convex or does not lower the residual, relaxing tau back towards
 * the caller's value after each accepted step.  Both keep tau >= 1. */
#define MA_DAMP_FIXED 0
#define MA_DAMP_BACKTRACK 1
/* multipliers of the derivatives in the linear solve: the paper's 2 pi i k and
 * -(2 pi k)^2 (Section 4.2), or the symbols of the fourth-order differences used for
 * the residual (an option: the linear solve then uses the Jacobian of the discrete
 * residual; the fixed point is unchanged) */
#define MA_SYMBOL_SPECTRAL 0
#define MA_SYMBOL_FD4 1
/* GMRES on L Lbar^{-1} sigma = h as in Section 4.2, or (an option) on the system
 * scaled on the left by D(x) = (a11 + a22)(x) / (abar11 + abar22), the trace of the
 * coefficient matrix relative to the averaged operator's: the same direction when
 * solved exactly, fewer iterations at a loose tolerance; the fixed point is unchanged */
#define MA_PRECOND_NONE 0
#define MA_PRECOND_DIAG 1
/* GMRES tolerance of each Newton direction: gmres_tol throughout (the paper), or (an
 * option, with MA_DAMP_BACKTRACK) per pair: after a step other than the first that had
 * to be halved twice or more, the next direction is solved 4x tighter (down to
 * min(gmres_tol, 1e-3)), after a full step 4x looser again (up to gmres_tol) */
#define MA_FORCING_FIXED 0
#define MA_FORCING_ADAPTIVE 1
/* The linear step of each Newton iteration: Strain's FFT method with GMRES(m)
 * (Section 4.2), or the finite-difference system of Section 4.1: second-order centred
 * differences for theta (a nine-point stencil), made nonsingular by the row of ones
 * that its Lemma adds to every row (tilde A = A + 1 1^T), solved by BiCG without a
 * preconditioner from a zero start with shadow residual r~0 = r0, until
 * ||r_k||_2 <= gmres_tol ||b||_2 or bicg_max_iters iterations.  Vectors and
 * reductions in FP64, coefficients in FP32.  Requires MA_PRECOND_NONE; gmres_m,
 * gmres_max_restarts and symbol are not used. */
#define MA_LINEAR_STRAIN_GMRES 0
#define MA_LINEAR_FD_BICG 1

typedef struct ma_options {
  int max_newton;          /* Newton iterations before MA_ENOCONV (100)              */
  int gmres_m;             /* GMRES restart length m, 1..30 (10, Section 5.1)       */
  int gmres_max_restarts;  /* restarts per linear solve (20)                         */
  double gmres_tol;        /* relative residual of the linear solve (1e-4, Sec. 5.1) */
  int interp;              /* MA_INTERP_*                                            */
  int op_mode;             /* MA_OP_*                                                */
  int damping_policy;      /* MA_DAMP_*                                              */
  int max_backtrack;       /* step halvings per Newton step before failing (12)      */
  int symbol;              /* MA_SYMBOL_* (MA_SYMBOL_SPECTRAL)                       */
  int precond;             /* MA_PRECOND_* (MA_PRECOND_NONE)                         */
  double boundary_frac;    /* MA_DAMP_BACKTRACK: a step is also halved while min det  */
                           /* (I + D^2 u) would fall below this fraction of its       */
                           /* current value, 0 <= . < 1 (0.1; 0 = off)                */
  int forcing;             /* MA_FORCING_* (MA_FORCING_FIXED)                        */
  double wait_limit_s;     /* longest host wait for one device summary, in seconds  */
                           /* (> 0; 600).  A solve whose device work does not reach  */
                           /* the summary within it returns MA_EHIP; the work        */
                           /* already queued on the stream still runs to its end,    */
                           /* so the caller synchronises the stream before reusing   */
                           /* its buffers or the plan                                */
  int max_active;          /* ma_solve_batched: at most this many pairs in flight; a  */
                           /* finished pair's slot takes the next pending pair of its */
                           /* size within the same call (0: every pair at once)       */
  int linear_solver;       /* MA_LINEAR_* (MA_LINEAR_STRAIN_GMRES)                    */
  int bicg_max_iters;      /* MA_LINEAR_FD_BICG: iterations per Newton step (1000,    */
                           /* Section 5.1), >= 1                                      */
} ma_options;

typedef struct ma_report {
  int status;              /* MA_OK or a soft failure code                           */
  int newton_iters;        /* Newton directions computed                             */
  int gmres_iters;         /* inner iterations of the linear steps: GMRES operator  */
                           /* applications, or BiCG iterations (one product with    */
                           /* tilde A and one with its transpose each)               */
  int backtracks;          /* rejected trial steps (MA_DAMP_BACKTRACK)               */
  double res_rms;          /* sqrt(mean (f - f~_n)^2) at the returned iterate        */
  double res_max;          /* max |f - f~_n|                                         */
  double res0_rms;         /* residual at the initial iterate                        */
  double mass_defect;      /* mean(f_n) - 1 before the translation of eq. translation */
  double min_det;          /* min det(I + D^2 u) at the returned iterate             */
  double w2sq;             /* mean(|grad u|^2 f): the transport distance (Sec. 5.2)  */
  double tau_final;        /* damping in force at exit                               */
  double time_ms;          /* wall time of the call that produced this report        */
  int warm_steps;          /* 1 if a given initial potential (possibly halved) was kept */
  int pad;
} ma_report;

typedef struct ma_plan ma_plan;

/* ABI version compiled into the library (MA_OT_ABI_VERSION). */
int ma_abi_version(void);

/* Fills *opt with the defaults listed above. */
void ma_options_default(ma_options* opt);

/* Static string naming a return/status code. */
const char* ma_strerror(int code);

/* Creates a plan holding all device workspace for up to `batch_capacity` pairs of
 * size up to `n_max` (workspace grows on demand past that).  `opt` may be NULL
 * (defaults).  Returns MA_OK, MA_EINVAL or MA_ENOMEM; *out is NULL on failure. */
int ma_plan_create(int n_max, int batch_capacity, const ma_options* opt, ma_plan** out);

/* Releases the plan and its device memory.  NULL is allowed. */
void ma_plan_destroy(ma_plan* plan);

/* Replaces the plan's options (validated; MA_EINVAL leaves them unchanged). */
int ma_plan_set_options(ma_plan* plan, const ma_options* opt);

/* Solves one pair (Section 3.1 algorithm, Section 4.2 linear solver).
 *   f, g    N*N FP64 densities, positive and finite; each is scaled to grid mean one.
 *   damping tau >= 1 of eq. (linma).  tol > 0: stop when sqrt(mean r^2) <= tol.
 *   psi0    N*N FP64 initial potential or NULL for u0 = 0.  Given one, the solve
 *           starts from u = 0 and tries psi0 - mean(psi0) as its first step: the step
 *           is kept if the iterate is convex and the residual drops, halved
 *           otherwise, and abandoned for u = 0 after max_backtrack halvings (an
 *           addition: it makes any initial guess safe to offer).
 *   psi     N*N FP64 out: the mean-zero potential u.
 *   map     2*N*N FP64 out: [0] = x1 + d1 u, [1] = x2 + d2 u (unwrapped, fourth-order
 *           differences), or NULL.
 *   rep     host out (may be NULL). */
int ma_solve(ma_plan* plan, const double* f, const double* g, int n, double damping,
             double tol, const double* psi0, double* psi, double* map, ma_report* rep,
             void* stream);

/* Solves `npairs` independent pairs, possibly of different sizes, together: every
 * kernel launch serves all pairs of one grid size and each pair follows its own
 * Newton / GMRES / step-halving state on the device.  All arrays of pointers are
 * HOST arrays of `npairs` device pointers (psi0 may be NULL, or hold NULL entries;
 * map may be NULL or hold NULL entries); n is a host array of sizes; reps a host
 * array of npairs reports (may be NULL).  Returns the largest per-pair status
 * (hard errors first). */
int ma_solve_batched(ma_plan* plan, int npairs, const int* n, const double* const* f,
                     const double* const* g, const double* const* psi0, double damping,
                     double tol, double* const* psi, double* const* map, ma_report* reps,
                     void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): ma_solve for one pair
 * without a plan and without any allocation.  The options are passed directly
 * (ma_options_default fills the defaults).  Every device buffer the solve needs
 * (the pair's workspace, descriptor, state, transform tables, the host-loop
 * summary) is carved from a fixed 48 MiB device array that the library holds on
 * each GPU it runs on until the process ends; no hipMalloc, hipFree or other
 * allocating routine is called.  Limit: n <= 512 and the pair's workspace within
 * that array (at n = 512: gmres_m <= 24); larger requests return MA_EINVAL.  Every
 * call on one GPU shares that GPU's array and leaves its contents there: calls
 * that overlap on one GPU (two streams, two host threads) race and must be
 * serialised by the caller.  The GMRES cycles are not cut short by the host (no
 * mapped summary), so the launch sequence differs from ma_solve; the arithmetic
 * and the result do not.  Arguments, outputs and return codes as ma_solve with the
 * launch geometry of a plan that has not been autotuned; the default wait limit
 * applies to each host wait. */
int ma_solve_noalloc(const ma_options* opt, const double* f, const double* g, int n,
                     double damping, double tol, const double* psi0, double* psi, double* map,
                     ma_report* rep, void* stream);

/* ---------------------------------------------------------------------------
 * Timing hook for one kernel class, used by the benchmark to report a roofline.
 * While enabled, every `every`-th launch of that class inside ma_solve /
 * ma_solve_batched (counting from the first after the call) is bracketed by HIP
 * events on the caller's stream, and adds the algorithmic bytes of the pairs it
 * actually serves (inputs read once, outputs written once; pairs that skip the
 * launch add nothing) to a device counter.  Events cost a few microseconds of
 * queue time around each timed launch: a stride above 1 keeps that overhead out of
 * the surrounding throughput while the average stays a live measurement.
 * ------------------------------------------------------------------------- */
#define MA_PROF_NONE 0
#define MA_PROF_RESIDUAL 1   /* fused residual / coefficient kernel             */
#define MA_PROF_ROW_A 2      /* row pass A: Krylov vector build + forward rows  */
#define MA_PROF_COLUMN 3     /* column pass B with the spectral multiply        */
#define MA_PROF_ROW_C 4      /* row pass C: inverse rows + combine + dots       */
#define MA_PROF_BICG_MATVEC 5  /* BiCG: the products with tilde A and tilde A^T   */

/* Selects the class to time (MA_PROF_NONE disables) and the sampling stride
 * (every >= 1; 1 = every launch), and clears the counters.  MA_EINVAL for an
 * unknown class or every < 1. */
int ma_plan_profile(ma_plan* plan, int kernel_class, int every);

/* Totals since ma_plan_profile: over the timed launches, summed event time (ms),
 * their number and their algorithmic bytes; over all launches of the class, their
 * number and algorithmic bytes.  Any pointer may be NULL.  Synchronises nothing (counters are final once
 * the solve call has returned). */
int ma_plan_profile_read(ma_plan* plan, double* ms, long long* launches, double* bytes,
                         long long* all_launches, double* all_bytes);

/* ---------------------------------------------------------------------------
 * Single steps of the hot path, for verification and profiling.  They run the
 * same kernels as the solver on one pair, using the plan's workspace, and are
 * stream-ordered (no host synchronisation unless a host output is requested).
 * They apply the operator of Section 4.2 whatever the plan's `precond` option.
 * ------------------------------------------------------------------------- */

/* Section 4 + eq. (ma2), (translation), (linearmaeq): fourth-order derivatives of u,
 * g and the grid gradient of g interpolated at x + grad u, f_n, the translated
 * residual and the operator coefficients.
 *   u, f, g   N*N FP64; f and g are used as given (no rescaling).
 *   r         N*N FP32 out: r = f - f~_n.
 *   coef      5*N*N FP32 out: planes a11, a12, a22, b1, b2 (op_mode applies).
 *   scalars   host out, 12 doubles: res_rms, res_max, mass_defect, min_det,
 *             min_trace, abar11, abar12, abar22, bbar1, bbar2 (Simpson means,
 *             Section 4.2), w2 = mean(|grad u|^2 f), mean(u).  Synchronises. */
int ma_step_residual(ma_plan* plan, int n, const double* u, const double* f,
                     const double* g, float* r, float* coef, double* scalars, void* stream);

/* Forward 2-D DFT of a real N*N FP32 field (the row and column FFT passes):
 * spec is N*(N/2) complex FP32 (interleaved re, im).  For 1 <= s < N/2,
 * spec[k1][s] = sum_{i,j} v[i][j] exp(-2 pi i (k1 i + s j)/N).  Slot s = 0 holds
 * the column transform of the packed real row coefficients:
 * spec[k1][0] = sum_i (X_i[0] + i X_i[N/2]) exp(-2 pi i k1 i/N), where
 * X_i[k] = sum_j v[i][j] exp(-2 pi i k j/N). */
int ma_step_fft2(ma_plan* plan, int n, const float* v, float* spec, void* stream);

/* Strain's operator (Section 4.2): w = L Lbar^{-1} v with coefficient planes `coef`
 * (5*N*N FP32, order a11, a12, a22, b1, b2) and host averages abar[5]. */
int ma_step_strain_apply(ma_plan* plan, int n, const float* v, const float* coef,
                         const double* abar, float* w, void* stream);

/* theta = Lbar^{-1} sigma (Section 4.2): the mean-zero solution of the averaged
 * operator, via rhobar(k). */
int ma_step_lbar_inverse(ma_plan* plan, int n, const float* sigma, const double* abar,
                         float* theta, void* stream);

/* Restarted GMRES(m) on L Lbar^{-1} sigma = h (Section 4.2), zero start, stopping
 * at ||h - A sigma|| <= tol ||h|| (estimated by the Givens rotations), followed by
 * theta = Lbar^{-1} sigma: the linear step of one Newton iteration.  h, theta N*N
 * FP32; coef 5*N*N FP32; abar host[5]; iters host out (operator applications).
 * Synchronises. */
int ma_step_gmres(ma_plan* plan, int n, const float* h, const float* coef,
                  const double* abar, int m, double tol, int max_restarts, float* theta,
                  int* iters, void* stream);

/* Spectral radius of the inverse of the linearised operator by the power method
 * (Section 5.1, stability paragraph after Table 1): from b_0 (N*N FP32 device, not
 * written) with its mean removed and normalised, `iters` steps b_{k+1} = A^{-1} b_k /
 * ||A^{-1} b_k||_2, each product A^{-1} b_k computed by Section 4.2's method (GMRES(m)
 * on L Lbar^{-1} sigma = b_k to gmres_tol, then theta = Lbar^{-1} sigma) for the
 * operator with coefficients coef (5*N*N FP32 device: a11, a12, a22, b1, b2) and
 * averages abar (host[5]).  rho (host[iters]) receives ||A^{-1} b_k||_2 (for the unit
 * b_k), gmres_iters (host[iters], may be NULL) the GMRES iterations of each product.
 * Uses the plan's workspace and synchronises the stream; MA_EINVAL for bad sizes. */
int ma_power_inverse(ma_plan* plan, int n, const float* coef, const double* abar,
                     const float* b0, int iters, double gmres_tol, int gmres_m,
                     int max_restarts, double* rho, int* gmres_iters, void* stream);

/* The finite-difference operator of Section 4.1 and its transpose:
 *   q  = tilde A p  = L_h p + (sum p) 1,
 *   qt = tilde A^T pt = L_h^T pt + (sum pt) 1,
 * with L_h p = a11 D11 p + 2 a12 D12 p + a22 D22 p + b1 D1 p + b2 D2 p (second-order
 * centred periodic differences, D12 on the four diagonal neighbours over 4h^2) and
 * L_h^T y = D11(a11 y) + 2 D12(a12 y) + D22(a22 y) - D1(b1 y) - D2(b2 y).
 * p, pt, q, qt N*N FP64; coef 5*N*N FP32 (a11, a12, a22, b1, b2).  The sums are taken
 * on the host in FP64 (this entry point copies p and pt there).  Synchronises. */
int ma_step_fd_apply(ma_plan* plan, int n, const double* p, const double* pt, const float* coef,
                     double* q, double* qt, void* stream);

/* BiCG on tilde A x = h (Section 4.1): zero start, shadow residual r~0 = r0, stop at
 * ||h - tilde A x||_2 <= tol ||h||_2 (the recurrence residual) or after max_iters
 * iterations, or at a breakdown (a zero denominator).  h N*N FP32, coef 5*N*N FP32,
 * x N*N FP64 out; iters host out (iterations done).  Synchronises. */
int ma_step_bicg(ma_plan* plan, int n, const float* h, const float* coef, double tol, int max_iters,
                 double* x, int* iters, void* stream);

/* ---------------------------------------------------------------------------
 * Three dimensions.  The method is stated for any dimension d (eq. (linearmaeq) with
 * the cofactor matrix of the d x d matrix I + D^2 u; Section 4.2 counts d(d+1) inverse
 * transforms per product).  One pair on an N x N x N grid, h = 1/N, arrays [i][j][k]
 * row-major with k contiguous (i <-> x1, j <-> x2, k <-> x3), N in {16, 32, 48, 64,
 * 96, 128, 192, 256}.  g and grad g are interpolated trilinearly at x + grad u; the
 * iterate must keep the leading minors of I + D^2 u positive (else MA_ENONCONVEX).
 * The linear step is Strain's method with nine derived transforms (alpha_ab, six, and
 * beta_a, three) and GMRES(m).  Options as for the 2-D solver, except that nearest
 * interpolation, MA_PRECOND_DIAG, MA_FORCING_ADAPTIVE and MA_LINEAR_FD_BICG are not
 * available (MA_EINVAL).  Each call synchronises `stream`.
 * ------------------------------------------------------------------------- */
typedef struct ma3_plan ma3_plan;

/* Plan for grids up to n_max (a supported N); opt may be NULL (defaults).  The device
 * workspace (about (172 + 4 (gmres_m + 1)) bytes per point) is allocated by the first
 * call that needs it and kept. */
int ma3_plan_create(int n_max, const ma_options* opt, ma3_plan** out);
void ma3_plan_destroy(ma3_plan* plan);

/* Damped Newton (eq. linma) in 3-D from u = 0: f, g N^3 FP64 positive densities
 * (scaled to mean one inside), damping tau >= 1, tol > 0 on the rms residual.
 * psi N^3 FP64 out (mean zero); map 3 N^3 FP64 out (x_a + D_a u, planes a = 1, 2, 3)
 * or NULL; rep host out or NULL.  Return codes as ma_solve; MA_EINVAL for an
 * unsupported N, N > n_max, or a density that is not positive and finite. */
int ma3_solve(ma3_plan* plan, const double* f, const double* g, int n, double damping, double tol,
              double* psi, double* map, ma_report* rep, void* stream);

/* One residual evaluation at a given iterate: u, f, g N^3 FP64 (f and g used as
 * given); r N^3 FP32 out (f - f_n); coef 9 N^3 FP32 out (a11, a22, a33, a12, a13, a23,
 * b1, b2, b3; op_mode applies); scalars host out, 17 doubles: res_rms, res_max,
 * mass_defect, min det, min (I + D^2 u)_11, min of the leading 2 x 2 minor, the nine
 * Simpson averages in coefficient order, mean(|grad u|^2 f), mean(u). */
int ma3_step_residual(ma3_plan* plan, int n, const double* u, const double* f, const double* g, float* r,
                      float* coef, double* scalars, void* stream);

/* Strain's operator in 3-D: w = L Lbar^{-1} v, v and w N^3 FP32, coef 9 N^3 FP32,
 * abar host[9] (the averages Lbar uses). */
int ma3_step_strain_apply(ma3_plan* plan, int n, const float* v, const float* coef, const double* abar,
                          float* w, void* stream);

/* theta = Lbar^{-1} sigma in 3-D (mean zero), sigma and theta N^3 FP32, abar host[9]. */
int ma3_step_lbar_inverse(ma3_plan* plan, int n, const float* sigma, const double* abar, float* theta,
                          void* stream);

/* ---------------------------------------------------------------------------
 * Autotuner (not in the paper): launch geometry per grid size.  Each of the four
 * bandwidth-bound kernel classes (row pass A, column pass B, row pass C, residual
 * stencil) has MA_TUNE_VARIANTS compiled geometries: 0 the default, 1 half as many
 * rows / columns per workgroup (residual: half the tile width), 2 twice as many
 * (residual: a quarter of the tile width), 3 the default tile with half the threads
 * (residual: the streaming kernel, where n is a multiple of 64: a wave walks down
 * 64 columns with the stencil rows in registers and no LDS tile); 4..7 the
 * wave-owned transforms, where each wavefront runs whole transforms in a padded LDS
 * region of its own with wave-level synchronisation only (row pass C: one or two row
 * pairs per block, n >= 128; its variants 6 and 7 are instead the block geometries 0
 * and 3 with the coefficient loads issued before the transforms and the twiddles read
 * from LDS); 8..11 the FFT radix plans of the three transform passes: 8 and 10 radix 4
 * throughout (a factor 3 first, a last 8 or 2), 9 and 11 radix 16 where it saves a
 * stage (512 = 16 8 4, 256 = 16 16, 384 = 3 16 8), at the default geometry (8, 9) or
 * at geometry 2 (passes A, B) / 3 (pass C) (10, 11); the default plan takes a factor 3
 * first, then eights (512 = 8 8 8, 384 = 3 8 4 4).  A variant that coincides with a
 * smaller index is skipped; its geometry query returns that index.
 * ------------------------------------------------------------------------- */
#define MA_TUNE_VARIANTS 12
#define MA_TUNE_SLOTS 12  /* room for the per-variant times below */

typedef struct ma_tuning {
  int n;               /* grid side */
  int npairs;          /* pairs per launch used for the timing */
  int variant[4];      /* pass A, pass B, pass C, residual; 0 = default geometry */
  int from_cache;      /* 1: read from the cache file, nothing timed */
  int rejected;        /* variants whose output differed from the default's */
  double us[4];        /* per-launch time of the chosen variants, microseconds (0 from the cache) */
  double us_default[4];/* per-launch time of the default geometry */
  double us_variant[4][MA_TUNE_SLOTS]; /* per-launch time of every variant timed, -1 where a
                                          variant was skipped (duplicate, rejected, absent);
                                          zeros when read from the cache */
  int npairs_part;     /* pairs of the partial-batch timing: npairs / 16, at least 1 */
  double us_part_variant[4][MA_TUNE_SLOTS]; /* per-launch time of every variant on the
                                          first npairs_part pairs (0 where npairs_part equals
                                          npairs); -1 and zeros as in us_variant.  A variant's
                                          score is us_variant + us_part_variant * npairs /
                                          npairs_part; the choice is the lowest score, an
                                          earlier variant kept unless beaten by 2% */
} ma_tuning;

/* Times every distinct variant of each kernel class on `npairs` synthetic pairs of
 * side n (smooth densities, coefficients near the Laplacian's, pseudo-random Krylov
 * vectors), rejects a variant whose output differs from the default geometry's by
 * more than FP32 reordering (fields 1e-6, folded partial sums 1e-5 of their
 * magnitude), times each on all npairs and on the first npairs / 16 (a solve's launches
 * shrink as pairs finish), and makes the best score (ma_tuning) the plan's choice for n.  If cache_path is not
 * NULL and holds an entry for this device, library build, n, npairs and the plan's
 * gmres_m, that entry is used instead; otherwise the result is added to the file
 * (a small JSON document, one entry per line).  Uses the plan's workspace (any
 * earlier solve's buffers are overwritten) and synchronises the stream. */
int ma_plan_autotune(ma_plan* plan, int n, int npairs, const char* cache_path, ma_tuning* out,
                     void* stream);
/* Sets the plan's variants for t->n (t->variant[0..3]); MA_EINVAL if out of range. */
int ma_plan_set_tuning(ma_plan* plan, const ma_tuning* t);
/* The plan's variants for n (zeros if never tuned). */
int ma_plan_get_tuning(const ma_plan* plan, int n, ma_tuning* out);
/* Geometry of a variant: pass 0..3 (A, B, C, residual); per_block = row pairs (A, C),
 * columns (B) or tile width (residual); threads per workgroup.  Returns the canonical
 * variant index (smaller if a duplicate), or -1 for an unsupported n or variant.
 * Host-only, no GPU needed. */
int ma_tune_geometry(int pass, int n, int variant, int* per_block, int* threads);

/* ---------------------------------------------------------------------------
 * Learned warm start (not in the paper): a periodic-padded 3x3 convolutional
 * network, BF16 on MFMA with FP32 accumulation, trained on pairs the solver
 * produces.  Linearising the equation about psi = 0 (Section 2) gives
 * Laplacian(psi) = log f - log g to first order for mean-one densities; the network
 * maps (log f, log g) at resolution n_net to c, its estimate of the remainder of the
 * fourth-order difference Laplacian of the potential, and the initial guess is
 * psi0 = (that Laplacian)^{-1} (c + log f - log g), mean zero.  The solver takes
 * psi0 as a checked start (ma_solve), so zero-init Newton stays the fallback.
 *
 * Parameters are FP32 masters in the order W_0, b_0, W_1, b_1, ... with
 * W_l[co][ci][3][3], 2 input channels, `channels` hidden, 1 output channel.  Layer l
 * computes z(x) = b + sum W[co][ci][a][c] h[ci](x + d_l (a - 1, c - 1)), periodic.
 * Network inputs are BF16 tensors [batch][n_net][n_net][8] (channels 0 and 1 are
 * log(f/mean f) and log(g/mean g), the rest zero), made by ma_cnn_prepare_input.
 * ------------------------------------------------------------------------- */
typedef struct ma_cnn ma_cnn;

/* layers >= 2, channels == 32, max_batch >= 1; dilations: host array of `layers`
 * dilation factors d_l >= 1 (the 3x3 taps of layer l are d_l pixels apart), or NULL
 * for all 1; n_net must be a multiple of 16 d_l for every layer. */
int ma_cnn_create(int layers, int channels, int n_net, int max_batch, const int* dilations, ma_cnn** out);
void ma_cnn_destroy(ma_cnn* net);
long ma_cnn_param_count(const ma_cnn* net);
/* host FP32 arrays of ma_cnn_param_count values; set also resets the Adam state */
int ma_cnn_set_params(ma_cnn* net, const float* host_params, long count);
int ma_cnn_get_params(const ma_cnn* net, float* host_params, long count);

/* f, g: device FP64 [batch][n_net][n_net]; x: device BF16 [batch][n_net][n_net][8]. */
int ma_cnn_prepare_input(ma_cnn* net, const double* f, const double* g, int batch, void* x, void* stream);
/* Training target, device FP64 in, FP32 out, all [batch][n][n]: the fourth-order
 * difference Laplacian of psi minus log(f / mean f) - log(g / mean g).  f and g may
 * both be NULL (then the plain Laplacian); one NULL without the other is MA_EINVAL. */
int ma_cnn_target(ma_cnn* net, const double* psi, const double* f, const double* g, int batch, int n,
                  float* target, void* stream);
/* c: device FP32 [batch][n_net][n_net]. */
int ma_cnn_forward(ma_cnn* net, const void* x, int batch, float* c, void* stream);
/* forward, MSE against target, backward: gradients (device FP32, parameter order)
 * and the loss (host) without updating.  Synchronises. */
int ma_cnn_gradients(ma_cnn* net, const void* x, const float* target, int batch, float* grads, float* loss,
                     void* stream);
/* one Adam step (beta 0.9, 0.999, eps 1e-8) on the MSE loss; loss (host) may be NULL
 * (then no synchronisation). */
int ma_cnn_train_step(ma_cnn* net, const void* x, const float* target, int batch, float lr, float* loss,
                      void* stream);
/* psi0 for npairs pairs of size n (n == n_net, or n == 2 n_net: the densities are
 * restricted by full weighting for the network and c is prolonged bilinearly; the log
 * ratio is taken at full resolution).
 * Arrays of pointers are host arrays of device pointers. */
int ma_cnn_warm_start(ma_cnn* net, int npairs, int n, const double* const* f, const double* const* g,
                      double* const* psi0, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MA_OT_H */
