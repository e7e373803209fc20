"""Damped Newton for the 3-D periodic Monge-Ampere equation.

TEST INFRASTRUCTURE ONLY (see the package header).  FP64 throughout, NumPy FFTs.

The paper states its method in any dimension d (Section 3: Adj(I + D^2 u) is the
cofactor matrix of a d x d matrix; Section 4.2: a product with Strain's operator takes
one forward and d(d+1) inverse transforms; the concluding remarks: the method holds in
higher dimensions).  Here d = 3, on the N x N x N grid x_ijk = (i h, j h, k h), h = 1/N,
array u[i, j, k] with axis a the coordinate x_{a+1}:

* eq. (ma2): M(u) = g(x + grad u) det(I + D^2 u) = f;
* eq. (linearmaeq): L theta = g(y) Tr(Adj(I + D^2 u) D^2 theta) + det(I + D^2 u) grad g(y) . grad theta,
  Adj(A) the cofactor matrix (Adj(A) = det(A) A^{-1}), so with M = I + D^2 u
  a_aa = g(y) (M_bb M_cc - M_bc^2), a_ab = g(y) (M_ac M_bc - M_ab M_cc)  ({a, b, c} = {1, 2, 3}),
  b_a = det(M) d_a g(y), and L theta = sum_a a_aa theta_aa + 2 sum_{a<b} a_ab theta_ab + b . grad theta;
* eq. (linma) with the translation of eq. (translation), the fourth-order differences of
  Section 4 along each axis (mixed derivatives as the first-derivative formula along one
  axis applied to the one along the other), g and grad g interpolated trilinearly at
  x + grad u (the 3-D form of reading P4), Simpson averages as the tensor product of the
  periodic 1-D weights (reading P7);
* Section 4.2 in 3-D: rhobar(k) = 1 / (sum abar_ab (2 pi i k_a)(2 pi i k_b) + sum bbar_a 2 pi i k_a),
  zero where the sum vanishes, alpha_ab = d_ab Lbar^{-1} sigma (six) and
  beta_a = d_a Lbar^{-1} sigma (three): nine distinct inverse transforms, the paper's
  d(d+1) = 12 counted without the symmetry alpha_ab = alpha_ba.

The wavenumber convention (reading P8), the residual norm (P6), the GMRES details (P9)
and the step-halving policy (P12, P22) are those of oracle.ma, whose multipliers and
GMRES this module calls.

Pins: tests/test_oracle_ma3d.py (cofactors against det(A) A^{-1}; data constant along x3
reduce to the 2-D solver's computation and solution; Strain's operator against the dense
Kronecker collocation matrices; the linearisation as the derivative of M; a discrete-exact
manufactured solution; fourth-order grid convergence against an analytic solution; the
W2 closed form; f = g gives no step).
"""

import time

import numpy as np

from . import fd
from . import interp as _interp
from . import ma

OK, ENOCONV, ENONCONVEX, ENAN = ma.OK, ma.ENOCONV, ma.ENONCONVEX, ma.ENAN

# index pairs of the six distinct second derivatives, in the coefficient order used
# throughout: a11, a22, a33, a12, a13, a23, then b1, b2, b3
PAIRS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))


def simpson_mean3(a):
    """Simpson approximation of the integral over the unit 3-torus (tensor weights)."""
    N = a.shape[0]
    w = fd.simpson_weights_1d(N)
    return float(np.einsum("i,j,k,ijk->", w, w, w, a))


def derivatives3(u, h):
    """(u1, u2, u3) and the six second derivatives (u11, u22, u33, u12, u13, u23)."""
    g = tuple(fd.d1(u, a, h) for a in range(3))
    sec = []
    for a, b in PAIRS:
        sec.append(fd.d2(u, a, h) if a == b else fd.d1(fd.d1(u, b, h), a, h))
    return g, tuple(sec)


def cofactors(M):
    """Cofactor matrix entries (c11, c22, c33, c12, c13, c23) and det of the symmetric
    3 x 3 field M = (m11, m22, m33, m12, m13, m23)."""
    m11, m22, m33, m12, m13, m23 = M
    c11 = m22 * m33 - m23 * m23
    c22 = m11 * m33 - m13 * m13
    c33 = m11 * m22 - m12 * m12
    c12 = m13 * m23 - m12 * m33
    c13 = m12 * m23 - m13 * m22
    c23 = m12 * m13 - m11 * m23
    det = m11 * c11 + m12 * c12 + m13 * c13
    return (c11, c22, c33, c12, c13, c23), det


class Problem3:
    """Normalised densities, the grid, and the grid gradient of g (readings P1, P5)."""

    def __init__(self, f, g, g_analytic=None):
        N = f.shape[0]
        if f.shape != (N, N, N) or g.shape != (N, N, N):
            raise ValueError("f and g must be N x N x N")
        self.N = N
        self.h = 1.0 / N
        self.f = np.asarray(f, dtype=np.float64) / np.mean(f)
        self.g = np.asarray(g, dtype=np.float64) / np.mean(g)
        self.Gg = tuple(fd.d1(self.g, a, self.h) for a in range(3))
        x = np.arange(N) * self.h
        self.X = np.meshgrid(x, x, x, indexing="ij")
        # g_analytic(y1, y2, y3) -> (g, dg/dy1, dg/dy2, dg/dy3), used instead of the grid g
        self.g_analytic = g_analytic

    def g_at(self, y):
        if self.g_analytic is not None:
            return self.g_analytic(*y)
        return (_interp.trilinear(self.g, *y),) + tuple(_interp.trilinear(G, *y) for G in self.Gg)


class Evaluation3:
    """Everything one Newton iteration computes from u_n before the linear solve."""


def evaluate3(u, prob):
    """f_n, the normalised residual r = f - f~_n and its norms (eq. ma2, eq. translation)."""
    ev = Evaluation3()
    grad, sec = derivatives3(u, prob.h)
    y = tuple(prob.X[a] + grad[a] for a in range(3))
    gy = prob.g_at(y)
    M = tuple((1.0 if a == b else 0.0) + s for (a, b), s in zip(PAIRS, sec))
    cof, det = cofactors(M)
    fn = gy[0] * det
    mean_fn = float(np.mean(fn))
    r = prob.f - (fn - mean_fn + 1.0)
    ev.grad, ev.sec, ev.gy, ev.cof, ev.det, ev.fn, ev.r = grad, sec, gy, cof, det, fn, r
    ev.mass_defect = mean_fn - 1.0
    ev.res_rms = float(np.sqrt(np.mean(r * r)))
    ev.res_max = float(np.max(np.abs(r)))
    ev.min_det = float(np.min(det))
    ev.min_trace = float(np.min(M[0] + M[1] + M[2]))
    ev.finite = bool(np.all(np.isfinite(r)))
    # uniform convexity of |x|^2/2 + u: the leading minors of I + D^2 u stay positive
    minor2 = M[0] * M[1] - M[3] * M[3]
    ev.convex = ev.finite and float(np.min(M[0])) > 0.0 and float(np.min(minor2)) > 0.0 and ev.min_det > 0.0
    return ev


def coefficients3(ev, op_mode=0):
    """(a11, a22, a33, a12, a13, a23, b1, b2, b3) of L_n (eq. linearmaeq in 3-D);
    op_mode = 1 drops the b term (Remarks of Section 3.3)."""
    a = tuple(ev.gy[0] * c for c in ev.cof)
    if op_mode == 1:
        b = tuple(np.zeros_like(ev.det) for _ in range(3))
    else:
        b = tuple(ev.det * ev.gy[1 + k] for k in range(3))
    return a + b


def averaged3(coef):
    return tuple(simpson_mean3(c) for c in coef)


def _mult(N, symbol):
    m1, m2 = ma.multipliers(N, symbol)
    return m1, m2


def _axes(v, a):
    """Broadcast a 1-D multiplier along axis a of an N x N x N array."""
    shape = [1, 1, 1]
    shape[a] = -1
    return v.reshape(shape)


def derivative_multiplier(N, a, b=None, symbol="spectral"):
    """Fourier multiplier of d_a (b None) or d_ab on the N^3 grid, FFT order (reading P8:
    the first-derivative multiplier vanishes at -N/2, the second-derivative one does not)."""
    m1, m2 = _mult(N, symbol)
    if b is None:
        return _axes(m1, a)
    if a == b:
        return _axes(m2, a)
    return _axes(m1, a) * _axes(m1, b)


def symbol3(abar, N, symbol="spectral"):
    """rhobar(k): the inverse symbol of the averaged operator, zero where it vanishes."""
    S = np.zeros((N, N, N), dtype=np.complex128)
    for w, (a, b) in zip(abar[:6], PAIRS):
        S = S + (1.0 if a == b else 2.0) * w * derivative_multiplier(N, a, b, symbol)
    for k in range(3):
        S = S + abar[6 + k] * derivative_multiplier(N, k, None, symbol)
    rho = np.zeros((N, N, N), dtype=np.complex128)
    nz = S != 0
    nz[0, 0, 0] = False
    rho[nz] = 1.0 / S[nz]
    return rho


def strain_apply3(v, coef, rho, symbol="spectral"):
    """A v = L Lbar^{-1} v = sum a_ab alpha_ab + sum b_a beta_a (Section 4.2 in 3-D)."""
    N = v.shape[0]
    s = rho * np.fft.fftn(v)
    out = np.zeros((N, N, N))
    for w, (a, b) in zip(coef[:6], PAIRS):
        alpha = np.fft.ifftn(derivative_multiplier(N, a, b, symbol) * s).real
        out += (1.0 if a == b else 2.0) * w * alpha
    for k in range(3):
        beta = np.fft.ifftn(derivative_multiplier(N, k, None, symbol) * s).real
        out += coef[6 + k] * beta
    return out


def lbar_inverse3(sigma, rho):
    return np.fft.ifftn(rho * np.fft.fftn(sigma)).real


def newton_direction3(ev, rhs_scale, op_mode, gmres_m, gmres_tol, gmres_max_restarts, symbol="spectral"):
    """theta solving D M theta = r * rhs_scale by Strain's method; returns (theta, its)."""
    coef = coefficients3(ev, op_mode)
    rho = symbol3(averaged3(coef), ev.r.shape[0], symbol)
    sigma, its, _ = ma.gmres(lambda v: strain_apply3(v.reshape(ev.r.shape), coef, rho, symbol).ravel(),
                             (ev.r * rhs_scale).ravel(), m=gmres_m, tol=gmres_tol,
                             max_restarts=gmres_max_restarts)
    return lbar_inverse3(sigma.reshape(ev.r.shape), rho), its


def solve3(f, g, tau=1.0, tol=1e-6, max_newton=100, gmres_m=10, gmres_tol=1e-4, gmres_max_restarts=20,
           op_mode=0, damping_policy="fixed", max_backtrack=12, boundary_frac=0.1, symbol="spectral",
           history=False, g_analytic=None):
    """Damped Newton (eq. linma) in 3-D with Strain's linear solver; the same control as
    oracle.ma.solve (fixed step 1/tau, or step halving with the boundary rule).

    Returns (psi, map, report): psi the mean-zero potential, map = x + D_h u as a
    (3, N, N, N) array, report as in oracle.ma."""
    t0 = time.perf_counter()
    f = np.asarray(f, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    N = f.shape[0]
    if N < 8 or N % 2 or not (tau >= 1.0) or not (tol > 0.0) or np.any(~np.isfinite(f)) or \
            np.any(~np.isfinite(g)) or np.min(f) <= 0 or np.min(g) <= 0:
        raise ValueError("invalid arguments")
    prob = Problem3(f, g, g_analytic)
    u = np.zeros((N, N, N))
    ev = evaluate3(u, prob)
    res0 = ev.res_rms
    hist = [ev.res_rms]
    n = gm = bt = 0
    tau_cur = float(tau)
    status = None
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
        theta, its = newton_direction3(ev, 1.0 / tau_cur, op_mode, gmres_m, gmres_tol, gmres_max_restarts, symbol)
        gm += its
        n += 1
        if damping_policy == "fixed":
            u = u + theta
            ev = evaluate3(u, prob)
        elif damping_policy == "backtrack":
            tau_solve = tau_cur
            accepted = False
            for _ in range(max_backtrack + 1):
                u_try = u + theta * (tau_solve / tau_cur)
                ev_try = evaluate3(u_try, prob)
                if (ev_try.convex and ev_try.res_rms < ev.res_rms
                        and ev_try.min_det >= boundary_frac * ev.min_det):
                    accepted = True
                    break
                tau_cur *= 2.0
                bt += 1
            if not accepted:
                status = ENOCONV
                break
            u, ev = u_try, ev_try
            tau_cur = max(float(tau), tau_cur / 2.0)
        else:
            raise ValueError("damping_policy must be 'fixed' or 'backtrack'")
        hist.append(ev.res_rms)
    psi = u - np.mean(u)
    mp = np.stack([prob.X[a] + ev.grad[a] for a in range(3)])
    w2 = float(np.mean((ev.grad[0] ** 2 + ev.grad[1] ** 2 + ev.grad[2] ** 2) * prob.f))
    rep = ma.Report(status=status, newton_iters=n, gmres_iters=gm, res_rms=ev.res_rms, res_max=ev.res_max,
                    res0_rms=res0, mass_defect=ev.mass_defect, min_det=ev.min_det, w2sq=w2,
                    time_ms=1e3 * (time.perf_counter() - t0), backtracks=bt, tau_final=tau_cur, warm_steps=0)
    if history:
        rep["history"] = hist
    return psi, mp, rep
