"""Damped Newton for the periodic Monge-Ampere equation, Strain's FFT operator, GMRES(m).

TEST INFRASTRUCTURE ONLY (see the package header).  FP64 throughout, NumPy FFTs.

What the paper fixes, and where:

* Section 3.1, eq. (ma2): with Psi = |x|^2/2 + u and u 1-periodic, solve
  M(u) = g(x + grad u) det(I + D^2 u) = f for u with |x|^2/2 + u convex.
* Section 3.1, eq. (linearmaeq): the derivative of M in direction theta is
  g(x + grad u) Tr(Adj(I + D^2 u) D^2 theta) + det(I + D^2 u) grad g(x + grad u) . grad theta,
  Adj(A) = det(A) A^{-1}.  In 2-D, Adj(I + H) = [[1 + u22, -u12], [-u12, 1 + u11]],
  so L theta = a11 theta_11 + 2 a12 theta_12 + a22 theta_22 + b1 theta_1 + b2 theta_2 with
  a11 = g(y)(1 + u22), a22 = g(y)(1 + u11), a12 = -g(y) u12, b_i = det * d_i g(y).
* Section 3.1, eq. (linma): f_n = g(x + grad u_n) det(I + D^2 u_n); solve
  D_{u_n}M theta_n = (f - f_n)/tau; u_{n+1} = u_n + theta_n; theta_n of mean zero.
  The Remarks of Section 3.3 allow dropping the b term (op_mode=1).
* Section 4: fourth-order differences for the derivatives of u_n (oracle.fd),
  interpolation of g (oracle.interp), and the normalisation of eq. (translation)
  f~_n = f_n - mean(f_n) + 1.
* Option precond = "diag" (not in the paper): GMRES on the system scaled on the left
  by D(x) = trace of the coefficient matrix over that of the averaged one; the same
  Newton direction when GMRES is run to convergence, fewer iterations at a loose
  tolerance.  Pins: identical to the plain solve when D = 1, the same direction
  at a tight GMRES tolerance, the same converged potential.
* Section 4.2: Strain's method.  Solve L Lbar^{-1} sigma = h by GMRES(m), then
  theta = Lbar^{-1} sigma, where Lbar has the Simpson averages of the coefficients,
  rhobar(k) = 1 / (sum abar_ij (2 pi i k_i)(2 pi i k_j) + sum bbar_i 2 pi i k_i), zero where
  that sum vanishes, and the Fourier sums run over |k_i| <= N/2.

Readings taken where the paper is silent (each listed with its pin in the design
notes): inputs scaled to mean one (P1); grid nodes (i h, j h) (P2); the five-point
formulas (P3); bilinear interpolation of g and of the grid gradient of g (P4, P5);
the grid-normalised l2 norm sqrt(mean r^2) as the stopping measure (P6); periodic
Simpson weights (P7); FFT wavenumbers -N/2..N/2-1 with the first-derivative
multiplier zero at -N/2 and the second-derivative multiplier -(2 pi k)^2 for
every k (P8); GMRES(m) with relative residual test and zero start (P9).

The optional step-halving policy ``damping_policy="backtrack"`` is not in the
paper; it only chooses tau per step (tau >= 1 as the paper requires) and leaves
the fixed point unchanged.

Pins: tests/test_oracle_ma.py (dense spectral-collocation matrices in closed
form; dense least squares for GMRES; spectral Poisson for the first step;
discrete-exact manufactured solution; fourth-order grid convergence against
the analytic solution; f = g; mass and gauge; the W2 closed form; the Nyquist
decay rate the paper reports).
"""

import math
import time

import numpy as np

from . import fd
from . import fd_bicg
from . import interp as _interp

OK, ENOCONV, ENONCONVEX, ENAN = 0, 1, 2, 3
EINVAL = -1
STATUS_NAMES = {OK: "ok", ENOCONV: "no convergence", ENONCONVEX: "lost convexity",
                ENAN: "non-finite value", EINVAL: "invalid argument"}


# ---------------------------------------------------------------------------
# Problem set-up
# ---------------------------------------------------------------------------

def check_inputs(f, g, tau, tol):
    """Argument checks shared by every entry point; raises ValueError."""
    f = np.asarray(f)
    g = np.asarray(g)
    if f.ndim != 2 or f.shape[0] != f.shape[1] or g.shape != f.shape:
        raise ValueError("f and g must be equal square N x N arrays")
    N = f.shape[0]
    if N < 8 or N % 2:
        raise ValueError("N must be even and at least 8")
    if not (tau >= 1.0):
        raise ValueError("the damping tau must be >= 1")
    if not (tol > 0.0):
        raise ValueError("tol must be positive")
    if not (np.all(np.isfinite(f)) and np.all(np.isfinite(g))):
        raise ValueError("densities must be finite")
    if not (np.all(f > 0) and np.all(g > 0)):
        raise ValueError("densities must be positive")
    return N


class Problem:
    """Normalised densities, grid, and the grid gradient of g (readings P1, P5)."""

    def __init__(self, f, g, interp="bilinear", g_analytic=None):
        N = f.shape[0]
        self.N = N
        self.h = 1.0 / N
        self.f = np.asarray(f, dtype=np.float64) / np.mean(f)
        self.g = np.asarray(g, dtype=np.float64) / np.mean(g)
        self.Gg1 = fd.d1(self.g, 0, self.h)
        self.Gg2 = fd.d1(self.g, 1, self.h)
        x = np.arange(N) * self.h
        self.X1, self.X2 = np.meshgrid(x, x, indexing="ij")
        if interp not in ("bilinear", "nearest"):
            raise ValueError("interp must be 'bilinear' or 'nearest'")
        self.interp = interp
        # g_analytic(y1, y2) -> (g, dg/dy1, dg/dy2); used instead of the grid g
        self.g_analytic = g_analytic

    def g_at(self, y1, y2):
        """g and grad g at the displaced points (Section 4)."""
        if self.g_analytic is not None:
            return self.g_analytic(y1, y2)
        I = _interp.bilinear if self.interp == "bilinear" else _interp.nearest
        return I(self.g, y1, y2), I(self.Gg1, y1, y2), I(self.Gg2, y1, y2)


class Evaluation:
    """Everything one Newton iteration computes from u_n before the linear solve."""


def evaluate(u, prob):
    """f_n, the normalised residual r = f - f~_n and its norms (eq. ma2, eq. translation)."""
    ev = Evaluation()
    h = prob.h
    u1, u2, u11, u22, u12 = fd.derivatives(u, h)
    y1 = prob.X1 + u1
    y2 = prob.X2 + u2
    gy, gy1, gy2 = prob.g_at(y1, y2)
    det = (1.0 + u11) * (1.0 + u22) - u12 * u12
    fn = gy * det
    mean_fn = float(np.mean(fn))
    ft = fn - mean_fn + 1.0
    r = prob.f - ft
    ev.u1, ev.u2, ev.u11, ev.u22, ev.u12 = u1, u2, u11, u22, u12
    ev.gy, ev.gy1, ev.gy2 = gy, gy1, gy2
    ev.det, ev.fn, ev.ft, ev.r = det, fn, ft, r
    ev.mass_defect = mean_fn - 1.0
    ev.res_rms = float(np.sqrt(np.mean(r * r)))
    ev.res_max = float(np.max(np.abs(r)))
    ev.min_det = float(np.min(det))
    ev.min_trace = float(np.min(2.0 + u11 + u22))
    ev.finite = bool(np.all(np.isfinite(r)))
    # the iterate must stay uniformly convex (Section 3.3): det > 0 and trace > 0
    ev.convex = ev.finite and ev.min_det > 0.0 and ev.min_trace > 0.0
    return ev


def coefficients(ev, op_mode=0):
    """Coefficients of L_n (eq. linearmaeq in 2-D); op_mode=1 drops the b term."""
    a11 = ev.gy * (1.0 + ev.u22)
    a22 = ev.gy * (1.0 + ev.u11)
    a12 = -ev.gy * ev.u12
    if op_mode == 1:
        b1 = np.zeros_like(a11)
        b2 = np.zeros_like(a11)
    else:
        b1 = ev.det * ev.gy1
        b2 = ev.det * ev.gy2
    return a11, a12, a22, b1, b2


def averaged(coef):
    """Simpson averages (abar11, abar12, abar22, bbar1, bbar2) over the torus (Section 4.2)."""
    return tuple(fd.simpson_mean(c) for c in coef)


# ---------------------------------------------------------------------------
# Strain's FFT operator (Section 4.2)
# ---------------------------------------------------------------------------

def multipliers(N, symbol="spectral"):
    """Multipliers of d/dx and d^2/dx^2 in FFT order.

    "spectral" (the paper, Section 4.2): 2 pi i k and -(2 pi k)^2, reading P8 at -N/2.
    "fd4" (an option, not the paper): the symbols of the fourth-order differences of
    Section 4, i (8 sin t - sin 2t)/(6h) and (32 cos t - 2 cos 2t - 30)/(12 h^2), t = 2 pi k h,
    so that the linear solve uses the Jacobian of the discrete residual.
    """
    k = np.fft.fftfreq(N, d=1.0 / N)
    if symbol == "fd4":
        h = 1.0 / N
        t = 2.0 * np.pi * k * h
        m1 = 1j * (8.0 * np.sin(t) - np.sin(2.0 * t)) / (6.0 * h)
        m1[k == -N // 2] = 0.0
        m2 = (32.0 * np.cos(t) - 2.0 * np.cos(2.0 * t) - 30.0) / (12.0 * h * h)
        return m1, m2
    if symbol != "spectral":
        raise ValueError("symbol must be 'spectral' or 'fd4'")
    m1 = 2j * np.pi * k
    m1[k == -N // 2] = 0.0
    m2 = -(2.0 * np.pi * k) ** 2
    return m1, m2


def symbol(abar, N, symbol="spectral"):
    """rhobar(k): the inverse symbol of the averaged operator, zero where the symbol is 0."""
    a11, a12, a22, b1, b2 = abar
    m1, m2 = multipliers(N, symbol)
    K1 = m1[:, None]
    K2 = m1[None, :]
    S = (a11 * m2[:, None] + 2.0 * a12 * (K1 * K2) + a22 * m2[None, :]
         + b1 * K1 + b2 * K2)
    S = np.broadcast_to(S, (N, N)).astype(np.complex128)
    rho = np.zeros((N, N), dtype=np.complex128)
    nz = S != 0
    nz[0, 0] = False  # the constant mode: the symbol is exactly zero there
    rho[nz] = 1.0 / S[nz]
    return rho


def strain_apply(v, coef, rho, symbol="spectral"):
    """A v = L Lbar^{-1} v = sum a_ij alpha_ij + sum b_i beta_i (Section 4.2)."""
    N = v.shape[0]
    m1, m2 = multipliers(N, symbol)
    a11, a12, a22, b1, b2 = coef
    s = rho * np.fft.fft2(v)
    alpha11 = np.fft.ifft2(m2[:, None] * s).real
    alpha22 = np.fft.ifft2(m2[None, :] * s).real
    alpha12 = np.fft.ifft2((m1[:, None] * m1[None, :]) * s).real
    beta1 = np.fft.ifft2(m1[:, None] * s).real
    beta2 = np.fft.ifft2(m1[None, :] * s).real
    return a11 * alpha11 + 2.0 * a12 * alpha12 + a22 * alpha22 + b1 * beta1 + b2 * beta2


def lbar_inverse(sigma, rho):
    """theta = Lbar^{-1} sigma = sum rhobar(k) sigmahat(k) e^{2 pi i k.x} (Section 4.2)."""
    return np.fft.ifft2(rho * np.fft.fft2(sigma)).real


# ---------------------------------------------------------------------------
# Restarted GMRES(m) (Section 4.2; Saad's textbook algorithm with Givens rotations)
# ---------------------------------------------------------------------------

def gmres(apply, b, m=10, tol=1e-4, max_restarts=20):
    """Solve apply(x) = b from x0 = 0 until ||b - A x|| <= tol ||b||.

    Modified Gram-Schmidt Arnoldi, Givens rotations on the Hessenberg matrix,
    restart every m inner iterations.  Returns (x, inner_iterations, converged).
    """
    x = np.zeros_like(b)
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        return x, 0, True
    target = tol * bnorm
    total = 0
    r = b.copy()
    for cycle in range(max_restarts + 1):
        if cycle > 0:
            r = b - apply(x)
        beta = float(np.linalg.norm(r))
        if beta <= target:
            return x, total, True
        V = [r / beta]
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        gv = np.zeros(m + 1)
        gv[0] = beta
        k = 0
        for j in range(m):
            w = apply(V[j])
            total += 1
            for i in range(j + 1):
                H[i, j] = float(np.vdot(V[i], w))
                w = w - H[i, j] * V[i]
            H[j + 1, j] = float(np.linalg.norm(w))
            hnext = H[j + 1, j]
            for i in range(j):  # earlier rotations act on the new column
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = math.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            gv[j + 1] = -sn[j] * gv[j]
            gv[j] = cs[j] * gv[j]
            k = j + 1
            if abs(gv[j + 1]) <= target or hnext == 0.0:
                break
            V.append(w / hnext)
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):  # back substitution on the rotated H
            y[i] = (gv[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        for i in range(k):
            x = x + y[i] * V[i]
        if abs(gv[k]) <= target:
            return x, total, True
    return x, total, False


# ---------------------------------------------------------------------------
# The damped Newton loop (eq. linma)
# ---------------------------------------------------------------------------

class Report(dict):
    """Per-solve report; the keys mirror the GPU library's report struct."""

    __getattr__ = dict.__getitem__


# adaptive forcing: halvings that trigger a tighter next direction (the first Newton
# direction exempt), the tightening factor, and the relaxation factor after a full step
_FORCING_HALVINGS = 2
_FORCING_TIGHTEN = 4.0
_FORCING_RELAX = 4.0


def diag_scale(coef, abar):
    """D(x) = (a11 + a22)(x) / (abar11 + abar22): the operator's trace relative to that
    of the averaged operator (positive wherever the iterate is convex)."""
    return (coef[0] + coef[2]) / (abar[0] + abar[2])


def newton_direction(ev, prob, rhs_scale, op_mode, gmres_m, gmres_tol, gmres_max_restarts,
                     symbol_kind="spectral", precond="none"):
    """theta solving D M theta = r * rhs_scale by Strain's method; returns (theta, its).

    precond = "diag" (not in the paper) runs GMRES on the left-scaled system
    D^{-1} L Lbar^{-1} sigma = D^{-1} h with D from diag_scale: the same sigma when
    solved exactly, a different Krylov space and stopping norm otherwise."""
    coef = coefficients(ev, op_mode)
    abar = averaged(coef)
    rho = symbol(abar, prob.N, symbol_kind)
    rhs = ev.r * rhs_scale
    if precond == "diag":
        D = diag_scale(coef, abar)
        op = lambda v: strain_apply(v, coef, rho, symbol_kind) / D  # noqa: E731
        rhs = rhs / D
    elif precond == "none":
        op = lambda v: strain_apply(v, coef, rho, symbol_kind)  # noqa: E731
    else:
        raise ValueError("precond must be 'none' or 'diag'")
    sigma, its, _ = gmres(op, rhs, m=gmres_m, tol=gmres_tol, max_restarts=gmres_max_restarts)
    return lbar_inverse(sigma, rho), its


def solve(f, g, tau=1.0, tol=1e-6, psi0=None, max_newton=100, gmres_m=10,
          gmres_tol=1e-4, gmres_max_restarts=20, interp="bilinear", op_mode=0,
          damping_policy="fixed", max_backtrack=12, g_analytic=None, history=False,
          symbol="spectral", precond="none", boundary_frac=0.1, forcing="fixed",
          linear="strain", bicg_max_iters=1000):
    """Damped Newton (eq. linma) with Strain's linear solver (Section 4.2), or with
    linear="fd_bicg" the finite-difference system of Section 4.1 solved by BiCG
    (oracle.fd_bicg) to the tolerance gmres_tol and at most bicg_max_iters iterations
    per Newton step; the report's gmres_iters then counts BiCG iterations.

    psi0, if given, is tried as a first step from u = 0 (accepted if convex and the
    residual drops, halved otherwise, abandoned after max_backtrack halvings).

    With damping_policy "backtrack" a Newton step is accepted only if the iterate
    stays convex, the residual drops, and min det(I + D^2 u) does not fall below
    boundary_frac times its current value (a fraction-to-the-boundary rule: without
    it an iterate can land next to the boundary of convexity, where every later
    direction leaves it and the halving stalls).

    Returns (psi, map, report): psi is the mean-zero potential u on the grid, map is
    x + D_h u as a (2, N, N) array (unwrapped: the additive map of Theorem CE1),
    report holds status, iteration counts and residual measures.
    """
    t0 = time.perf_counter()
    check_inputs(f, g, tau, tol)
    prob = Problem(np.asarray(f, np.float64), np.asarray(g, np.float64), interp, g_analytic)
    N = prob.N
    u = np.zeros((N, N))
    ev = evaluate(u, prob)
    res0 = ev.res_rms
    hist = [ev.res_rms]
    n = 0
    gm_total = 0
    backtracks = 0
    warm_steps = 0
    tau_cur = float(tau)
    status = None
    if forcing not in ("fixed", "adaptive"):
        raise ValueError("forcing must be 'fixed' or 'adaptive'")
    if linear not in ("strain", "fd_bicg"):
        raise ValueError("linear must be 'strain' or 'fd_bicg'")
    if linear == "fd_bicg" and precond != "none":
        raise ValueError("the BiCG step has no preconditioner (Section 4.1)")
    eta, eta_min = gmres_tol, min(gmres_tol, 1e-3)  # GMRES tolerance of the next direction
    if psi0 is not None and ev.finite and ev.res_rms > tol:
        # checked start (not in the paper): psi0 is tried as a first step from u = 0 and
        # halved while the trial is non-convex or does not lower the residual; after
        # max_backtrack halvings the solve continues from u = 0
        step = np.asarray(psi0, dtype=np.float64) - np.mean(psi0)
        for k in range(max_backtrack + 1):
            ev_try = evaluate(step, prob)
            if ev_try.convex and ev_try.res_rms < ev.res_rms:
                u, ev = step, ev_try
                warm_steps = 1
                hist.append(ev.res_rms)
                break
            step = 0.5 * step
    while True:
        if not ev.finite:
            status = ENAN
            break
        if not ev.convex:
            status = ENONCONVEX
            break
        if ev.res_rms <= tol:
            status = OK
            break
        if n >= max_newton:
            status = ENOCONV
            break
        if linear == "fd_bicg":
            theta, its = fd_bicg.newton_direction(coefficients(ev, op_mode), ev.r, 1.0 / tau_cur,
                                                  eta, bicg_max_iters)
        else:
            theta, its = newton_direction(ev, prob, 1.0 / tau_cur, op_mode, gmres_m,
                                          eta, gmres_max_restarts, symbol, precond)
        gm_total += its
        n += 1
        if damping_policy == "fixed":
            u = u + theta
            ev = evaluate(u, prob)
        elif damping_policy == "backtrack":
            tau_solve = tau_cur
            accepted = False
            halvings = 0
            for _ in range(max_backtrack + 1):
                u_try = u + theta * (tau_solve / tau_cur)
                ev_try = evaluate(u_try, prob)
                if (ev_try.convex and ev_try.res_rms < ev.res_rms
                        and ev_try.min_det >= boundary_frac * ev.min_det):
                    accepted = True
                    break
                tau_cur *= 2.0
                backtracks += 1
                halvings += 1
            if not accepted:
                status = ENOCONV
                break
            u, ev = u_try, ev_try
            tau_cur = max(float(tau), tau_cur / 2.0)
            if forcing == "adaptive":
                # a step (after the first) that had to be halved twice or more came from a
                # direction solved too loosely for the distance to the solution: solve the
                # next one more tightly; relax again after a full step.  The first direction
                # is exempt: from u = 0 it is halved for its linearisation, not its accuracy
                if halvings >= _FORCING_HALVINGS and n > 1:
                    eta = max(eta / _FORCING_TIGHTEN, eta_min)
                elif halvings == 0:
                    eta = min(gmres_tol, _FORCING_RELAX * eta)
        else:
            raise ValueError("damping_policy must be 'fixed' or 'backtrack'")
        hist.append(ev.res_rms)
    # u is fixed up to a constant (Section 4.1 fixes it by a zero integral): the mean-zero
    # representative is returned; the Strain step keeps u at mean zero by itself, the BiCG
    # step moves the mean whenever the right-hand side is not in the range of A (F4)
    psi = u - np.mean(u)
    mp = np.stack([prob.X1 + ev.u1, prob.X2 + ev.u2])
    rep = Report(status=status, newton_iters=n, gmres_iters=gm_total, res_rms=ev.res_rms,
                 res_max=ev.res_max, res0_rms=res0, mass_defect=ev.mass_defect,
                 min_det=ev.min_det, w2sq=float(np.mean((ev.u1 ** 2 + ev.u2 ** 2) * prob.f)),
                 time_ms=1e3 * (time.perf_counter() - t0), backtracks=backtracks,
                 tau_final=tau_cur, warm_steps=warm_steps)
    if history:
        rep["history"] = hist
    return psi, mp, rep
