"""Pins for oracle.ma: Strain's operator, GMRES, and the damped Newton loop.

Each test checks the oracle against something other than itself: closed-form
spectral collocation matrices (Trefethen, Spectral Methods in MATLAB, ch. 3),
dense linear algebra, analytic solutions, or numbers the paper prints.
"""

import math
import os

import numpy as np
import pytest

from oracle import fd, ma
from paper_1009_6039_amd import workloads as W


# ---------------------------------------------------------------- dense references

def trefethen_d1(N):
    """Closed-form Fourier first-derivative matrix on [0,1) with N (even) nodes."""
    h = 2 * math.pi / N
    D = np.zeros((N, N))
    for j in range(N):
        for l in range(N):
            if j != l:
                D[j, l] = 0.5 * (-1) ** (j - l) / math.tan((j - l) * h / 2)
    return 2 * math.pi * D


def trefethen_d2(N):
    """Closed-form Fourier second-derivative matrix on [0,1) (not the square of D1)."""
    h = 2 * math.pi / N
    D = np.zeros((N, N))
    for j in range(N):
        for l in range(N):
            if j == l:
                D[j, l] = -math.pi ** 2 / (3 * h * h) - 1.0 / 6.0
            else:
                D[j, l] = -((-1) ** (j - l)) / (2 * math.sin((j - l) * h / 2) ** 2)
    return 4 * math.pi ** 2 * D


def dense_operator(coef, N):
    """L = a11 D11 + 2 a12 D12 + a22 D22 + b1 D1 + b2 D2 on row-major vec(u), u[i,j], i <-> x1."""
    D1, D2, I = trefethen_d1(N), trefethen_d2(N), np.eye(N)
    a11, a12, a22, b1, b2 = [np.broadcast_to(c, (N, N)).ravel() for c in coef]
    return (a11[:, None] * np.kron(D2, I) + 2 * a12[:, None] * np.kron(D1, D1)
            + a22[:, None] * np.kron(I, D2) + b1[:, None] * np.kron(D1, I)
            + b2[:, None] * np.kron(I, D1))


def random_coefficients(N, seed):
    rng = np.random.default_rng(seed)
    x = np.arange(N) / N
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    gy = 1 + 0.4 * np.cos(2 * np.pi * X1 + rng.uniform()) * np.sin(2 * np.pi * X2)
    u11 = 0.3 * np.sin(2 * np.pi * (X1 + X2))
    u22 = 0.2 * np.cos(4 * np.pi * X2)
    u12 = 0.15 + 0.1 * np.sin(2 * np.pi * X1)  # nonzero mean: abar12 != 0
    a11, a22, a12 = gy * (1 + u22), gy * (1 + u11), -gy * u12
    b1 = 0.5 * rng.standard_normal((N, N))
    b2 = 0.5 * rng.standard_normal((N, N))
    return a11, a12, a22, b1, b2


# ---------------------------------------------------------------- Strain operator

def test_trefethen_matrices_are_the_fourier_multipliers():
    # independent check that the closed forms encode reading P8 (D1 kills Nyquist, D2 keeps it)
    N = 8
    x = np.arange(N) / N
    for k in range(-N // 2, N // 2):
        e = np.exp(2j * np.pi * k * x)
        m1 = 0.0 if k == -N // 2 else 2j * np.pi * k
        if k == -N // 2:  # the Nyquist mode is real on the grid: derivative of cos(pi N x) is 0
            e = e.real
        assert np.allclose(trefethen_d1(N) @ e, m1 * e, atol=1e-9)
        assert np.allclose(trefethen_d2(N) @ e, -(2 * np.pi * k) ** 2 * e, atol=1e-8)


@pytest.mark.parametrize("N", [8, 12])
def test_strain_matvec_equals_dense_collocation_product(N):
    coef = random_coefficients(N, N)
    abar = ma.averaged(coef)
    rho = ma.symbol(abar, N)
    L = dense_operator(coef, N)
    Lbar = dense_operator(abar, N)
    A = L @ np.linalg.pinv(Lbar, rcond=1e-12)
    v = np.random.default_rng(7).standard_normal((N, N))
    assert np.allclose(ma.strain_apply(v, coef, rho).ravel(), A @ v.ravel(), rtol=1e-9, atol=1e-9)
    theta = ma.lbar_inverse(v, rho)
    assert np.allclose(theta.ravel(), np.linalg.pinv(Lbar, rcond=1e-12) @ v.ravel(), atol=1e-10)


def test_symbol_is_hermitian_and_zero_only_at_the_constant_mode():
    N = 16
    abar = (1.3, -0.2, 0.9, 0.4, -0.7)
    rho = ma.symbol(abar, N)
    idx = (-np.arange(N)) % N
    assert np.allclose(rho[idx][:, idx], np.conj(rho), rtol=1e-14, atol=0)
    assert rho[0, 0] == 0
    assert np.count_nonzero(rho == 0) == 1
    # the averaged operator is elliptic: Re S(k) < 0 for k != 0
    S = 1.0 / rho[rho != 0]
    assert np.all(S.real < 0)


def test_strain_operator_outputs_are_real():
    N = 16
    coef = random_coefficients(N, 3)
    rho = ma.symbol(ma.averaged(coef), N)
    s = rho * np.fft.fft2(np.random.default_rng(1).standard_normal((N, N)))
    m1, m2 = ma.multipliers(N)
    for mult in (m2[:, None], m2[None, :], m1[:, None] * m1[None, :], m1[:, None], m1[None, :],
                 np.ones((1, 1))):
        z = np.fft.ifft2(mult * s)
        assert np.max(np.abs(z.imag)) < 1e-12 * max(1.0, np.max(np.abs(z.real)))


# ---------------------------------------------------------------- GMRES

def test_gmres_matches_dense_solution():
    N = 8
    coef = random_coefficients(N, 11)
    rho = ma.symbol(ma.averaged(coef), N)
    A = np.stack([ma.strain_apply(e.reshape(N, N), coef, rho).ravel()
                  for e in np.eye(N * N)], axis=1)
    h = (A @ np.random.default_rng(5).standard_normal(N * N)).reshape(N, N)
    sig, its, conv = ma.gmres(lambda v: ma.strain_apply(v, coef, rho), h, m=N * N, tol=1e-12)
    assert conv
    ref = np.linalg.lstsq(A, h.ravel(), rcond=None)[0].reshape(N, N)
    # sigma is defined up to the kernel of A (constants); theta = Lbar^{-1} sigma is unique
    assert np.allclose(ma.lbar_inverse(sig, rho), ma.lbar_inverse(ref, rho), atol=1e-10)


def test_restarted_gmres_reaches_tolerance_and_counts_iterations():
    N = 16
    coef = random_coefficients(N, 2)
    rho = ma.symbol(ma.averaged(coef), N)
    op = lambda v: ma.strain_apply(v, coef, rho)  # noqa: E731
    h = op(np.random.default_rng(9).standard_normal((N, N)))
    sig, its, conv = ma.gmres(op, h, m=3, tol=1e-8, max_restarts=200)
    assert conv and its > 3
    assert np.linalg.norm(h - op(sig)) <= 1.01e-8 * np.linalg.norm(h)


def test_gmres_identity_converges_in_one_iteration():
    b = np.random.default_rng(0).standard_normal((8, 8))
    x, its, conv = ma.gmres(lambda v: 2.0 * v, b, m=10, tol=1e-12)
    assert conv and its == 1 and np.allclose(x, b / 2)


# ---------------------------------------------------------------- Newton loop

def test_first_step_with_uniform_target_is_a_spectral_poisson_solve():
    # g = 1, u0 = 0: L = Lbar = Laplacian, A = I on mean-zero fields, theta0 = Lap^{-1}(f - 1)/tau
    N = 16
    f, g, _ = W.manufactured(N, A=0.02)
    prob = ma.Problem(f, g)
    ev = ma.evaluate(np.zeros((N, N)), prob)
    tau = 3.0
    coef = ma.coefficients(ev)
    rho = ma.symbol(ma.averaged(coef), N)
    sig, its, _ = ma.gmres(lambda v: ma.strain_apply(v, coef, rho), ev.r / tau, tol=1e-12)
    assert its == 1
    theta = ma.lbar_inverse(sig, rho)
    D2, I = trefethen_d2(N), np.eye(N)
    lap = np.kron(D2, I) + np.kron(I, D2)
    ref = np.linalg.pinv(lap, rcond=1e-12) @ ((prob.f - 1.0) / tau).ravel()
    assert np.allclose(theta.ravel(), ref, atol=1e-12)


def test_discrete_exact_manufactured_solution_is_recovered():
    # f := det(I + D_h^2 psi*) translated to mean 1, g = 1: the discrete fixed point is psi* itself
    N = 32
    _, g, ps = W.manufactured(N, A=0.01)
    u1, u2, u11, u22, u12 = fd.derivatives(ps, 1.0 / N)
    fdisc = (1 + u11) * (1 + u22) - u12 ** 2
    fdisc = fdisc - fdisc.mean() + 1.0
    psi, _, rep = ma.solve(fdisc, g, tau=1.0, tol=1e-13)
    assert rep.status == ma.OK
    assert np.max(np.abs(psi - ps)) < 1e-10


def golden(name):
    """Rows of a fixture in tests/golden/ (values printed in the paper, cited there)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)
    with open(path) as fh:
        return [line.split() for line in fh if line.strip() and not line.startswith("#")]


def test_fourth_order_grid_convergence_on_the_manufactured_example():
    # Section 5.1 prints the observed orders for grids 16..256 (tests/golden/)
    paper = [float(r[2]) for r in golden("sec5_1_observed_orders.txt")]
    errs = []
    for N in (16, 32, 64):
        f, g, ps = W.manufactured(N)
        psi, _, rep = ma.solve(f, g, tau=1.0, tol=1e-11)
        assert rep.status == ma.OK
        errs.append(math.sqrt(np.mean((psi - ps) ** 2)))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert abs(orders[-1] - paper[-1]) < 0.05  # the asymptotic order
    assert all(min(paper) - 0.1 < o < max(paper) + 0.05 for o in orders)


def test_equal_densities_give_zero_potential_without_iterating():
    N = 32
    f, _ = W.blobs(N, 5)
    psi, mp, rep = ma.solve(f, f.copy(), tau=1.0, tol=1e-12)
    assert rep.status == ma.OK and rep.newton_iters == 0
    assert np.all(psi == 0)
    x = np.arange(N) / N
    assert np.allclose(mp[0], x[:, None]) and np.allclose(mp[1], x[None, :])


def test_mass_and_gauge_are_preserved():
    N = 32
    f, g = W.blobs(N, 8)
    prob = ma.Problem(f, g)
    u = 0.002 * np.random.default_rng(0).standard_normal((N, N))
    u -= u.mean()
    ev = ma.evaluate(u, prob)
    assert abs(np.mean(ev.ft) - 1.0) < 1e-14
    assert abs(np.mean(ev.r)) < 1e-14
    psi, _, rep = ma.solve(f, g, tau=1.0, tol=1e-8, damping_policy="backtrack", gmres_tol=0.1)
    assert rep.status == ma.OK
    assert abs(np.mean(psi)) < 1e-15 * max(1, rep.newton_iters) * 100


def test_w2_closed_form():
    # g = 1, psi* = A sin sin: d(f,g) = int |grad psi*|^2 f = 2 pi^2 A^2 (Section 5.2 distance)
    A = 0.01
    f, g, _ = W.manufactured(64, A=A)
    _, _, rep = ma.solve(f, g, tau=1.0, tol=1e-11)
    assert rep.w2sq == pytest.approx(2 * math.pi ** 2 * A ** 2, rel=1e-5)


def test_nyquist_mode_decays_at_the_rate_the_paper_reports():
    # Section 5.1: the residual of the FFT implementation decays by "about 0.45" per iteration.
    # For a Nyquist-mode error the fourth-order and spectral second-derivative symbols differ
    # by the factor (64/12)/pi^2, so one tau=1 step leaves 1 - 64/(12 pi^2) = 0.4596 of it.
    N = 32
    f = np.ones((N, N))
    u0 = 1e-7 * (-1.0) ** np.arange(N)[:, None] * np.ones((1, N))
    prob = ma.Problem(f, f)
    ev0 = ma.evaluate(u0, prob)
    theta, _ = ma.newton_direction(ev0, prob, 1.0, 0, 10, 1e-12, 20)
    ev1 = ma.evaluate(u0 + theta, prob)
    rate = ev1.res_rms / ev0.res_rms
    assert rate == pytest.approx(1 - 64 / (12 * math.pi ** 2), abs=2e-4)
    paper = {r[0]: float(r[1]) for r in golden("sec5_1_residual_ratio.txt")}
    assert abs(rate - paper["fft"]) < 0.015


def test_larger_damping_converges_more_slowly():
    # Figure error_diff_tau: bigger tau, slower convergence; rate bound 1 - 1/(2 tau) (Section 3.3)
    f, g, _ = W.manufactured(32, A=0.01)
    iters = []
    for tau in (1.0, 2.0, 4.0):
        _, _, rep = ma.solve(f, g, tau=tau, tol=1e-9, history=True)
        assert rep.status == ma.OK
        iters.append(rep.newton_iters)
        h = rep.history
        tail = h[-1] / h[-2]
        if tau > 1:
            assert tail <= 1 - 1 / (2 * tau) + 1e-3
    assert iters[0] < iters[1] < iters[2]


def test_iterates_stay_convex_on_blob_pairs():
    N = 64
    f, g = W.blobs(N, W.seed_for(1, 0))
    psi, _, rep = ma.solve(f, g, tau=1.0, tol=1e-6, damping_policy="backtrack", gmres_tol=0.1)
    assert rep.status == ma.OK and rep.min_det > 0 and rep.res_rms <= 1e-6


def test_fixed_full_step_on_blob_pair_loses_convexity():
    f, g = W.blobs(64, W.seed_for(1, 0))
    _, _, rep = ma.solve(f, g, tau=1.0, tol=1e-6, gmres_tol=0.1)
    assert rep.status == ma.ENONCONVEX


@pytest.mark.parametrize("bad", ["odd", "small", "tau", "tol", "neg", "nan"])
def test_invalid_arguments_are_rejected(bad):
    f = np.ones((16, 16))
    g = np.ones((16, 16))
    kw = dict(tau=1.0, tol=1e-6)
    if bad == "odd":
        f = g = np.ones((15, 15))
    elif bad == "small":
        f = g = np.ones((6, 6))
    elif bad == "tau":
        kw["tau"] = 0.5
    elif bad == "tol":
        kw["tol"] = 0.0
    elif bad == "neg":
        f = f.copy()
        f[3, 3] = -1
    elif bad == "nan":
        g = g.copy()
        g[0, 0] = np.nan
    with pytest.raises(ValueError):
        ma.solve(f, g, **kw)


def test_linearisation_is_the_derivative_of_M():
    # eq. (linearmaeq) is the directional derivative of M(u) = g(x + grad u) det(I + D^2 u).
    # With an analytic g (the Section 5.1 form) and smooth u, theta, the central difference
    # of f_n along theta must match L theta evaluated with the oracle's coefficients.
    N = 64
    al = 0.3

    def g_an(y1, y2):
        c1, c2 = np.cos(2 * np.pi * y1), np.cos(2 * np.pi * y2)
        s1, s2 = np.sin(2 * np.pi * y1), np.sin(2 * np.pi * y2)
        return 1 + al * c1 * c2, -2 * np.pi * al * s1 * c2, -2 * np.pi * al * c1 * s2

    x = np.arange(N) / N
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    prob = ma.Problem(np.ones((N, N)), np.ones((N, N)), g_analytic=g_an)
    u = 0.01 * np.cos(2 * np.pi * X1) * np.sin(2 * np.pi * X2) + 0.004 * np.sin(2 * np.pi * (X1 - X2))
    theta = np.sin(2 * np.pi * X1 + 0.3) * np.cos(2 * np.pi * X2) + 0.5 * np.sin(4 * np.pi * X2)
    eps = 1e-6
    dfn = (ma.evaluate(u + eps * theta, prob).fn - ma.evaluate(u - eps * theta, prob).fn) / (2 * eps)
    ev = ma.evaluate(u, prob)
    a11, a12, a22, b1, b2 = ma.coefficients(ev)
    h = 1.0 / N
    t1, t2, t11, t22, t12 = fd.derivatives(theta, h)
    Ltheta = a11 * t11 + 2 * a12 * t12 + a22 * t22 + b1 * t1 + b2 * t2
    assert np.max(np.abs(dfn - Ltheta)) < 1e-7 * np.max(np.abs(Ltheta))


def test_fd4_symbol_option_is_the_difference_operator():
    # the "fd4" multipliers are exactly the fourth-order difference operators of oracle.fd
    N = 16
    rng = np.random.default_rng(3)
    u = rng.standard_normal((N, N))
    m1, m2 = ma.multipliers(N, "fd4")
    U = np.fft.fft2(u)
    h = 1.0 / N
    # the first-derivative symbol is zero at -N/2 in both conventions; remove that mode
    nyq = np.cos(np.pi * np.arange(N))
    u0 = u - np.outer(nyq, np.ones(N)) * (nyq @ u.sum(axis=1)) / (N * N)
    assert np.allclose(np.fft.ifft2(m2[:, None] * U).real, fd.d2(u, 0, h), atol=1e-9)
    assert np.allclose(np.fft.ifft2(m2[None, :] * U).real, fd.d2(u, 1, h), atol=1e-9)
    assert np.allclose(np.fft.ifft2(m1[:, None] * np.fft.fft2(u0)).real, fd.d1(u0, 0, h), atol=1e-9)


def test_fd4_symbol_newton_converges_to_the_same_fixed_point_faster():
    N = 64
    f, g = W.blobs(N, W.seed_for(1, 1))
    a, _, ra = ma.solve(f, g, tol=1e-10, damping_policy="backtrack", gmres_tol=0.1, max_newton=300)
    b, _, rb = ma.solve(f, g, tol=1e-10, damping_policy="backtrack", gmres_tol=0.1, max_newton=300,
                        symbol="fd4")
    assert ra.status == rb.status == ma.OK
    assert np.max(np.abs(a - b)) < 1e-9 * max(1.0, np.max(np.abs(a))) * 10
    assert rb.newton_iters < ra.newton_iters


def test_checked_start_accepts_a_good_guess_and_survives_a_bad_one():
    N = 32
    f, g, ps = W.manufactured(N, A=0.01)
    ref, _, r0 = ma.solve(f, g, tol=1e-10)
    # a good guess is taken at full step and saves Newton iterations
    good, _, rg = ma.solve(f, g, tol=1e-10, psi0=ps)
    assert rg.warm_steps == 1 and rg.newton_iters < r0.newton_iters
    assert np.max(np.abs(good - ref)) < 1e-9
    # a guess that makes I + D^2 psi indefinite is halved until it helps, or dropped
    bad = 3.0 * np.sin(2 * np.pi * np.arange(N) / N)[:, None] * np.ones((1, N))
    out, _, rb = ma.solve(f, g, tol=1e-10, psi0=bad)
    assert rb.status == ma.OK and np.max(np.abs(out - ref)) < 1e-9


# --- option precond = "diag": left scaling by the relative trace of the coefficients ---

def _blob_eval(N, seed):
    from paper_1009_6039_amd import workloads as W
    f, g = W.blobs(N, W.seed_for(1, seed))
    prob = ma.Problem(f, g)
    x = np.arange(N) / N
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    u = 0.004 * np.sin(2 * np.pi * X1 + 0.3) * np.cos(2 * np.pi * X2)
    return prob, ma.evaluate(u, prob)


def test_diag_scale_is_one_for_the_laplacian():
    N = 16
    prob = ma.Problem(np.ones((N, N)) + 0.1 * np.cos(2 * np.pi * np.arange(N) / N)[:, None], np.ones((N, N)))
    ev = ma.evaluate(np.zeros((N, N)), prob)
    coef = ma.coefficients(ev, 0)
    assert np.allclose(ma.diag_scale(coef, ma.averaged(coef)), 1.0, atol=1e-14)
    t1, i1 = ma.newton_direction(ev, prob, 1.0, 0, 10, 1e-8, 20, "spectral", "none")
    t2, i2 = ma.newton_direction(ev, prob, 1.0, 0, 10, 1e-8, 20, "spectral", "diag")
    assert i1 == i2 and np.allclose(t1, t2, atol=1e-12 * np.max(np.abs(t1)))


@pytest.mark.parametrize("symbol", ["spectral", "fd4"])
def test_diag_scaled_direction_equals_plain_direction_when_solved_exactly(symbol):
    # D^{-1} A sigma = D^{-1} h has the solution of A sigma = h: scaling only one side
    # (or using a different D on the two sides) breaks this.  The right-hand side is
    # taken in the range of A (h = A v), where both systems are solvable exactly.
    import copy
    prob, ev = _blob_eval(32, 2)
    coef = ma.coefficients(ev, 0)
    rho = ma.symbol(ma.averaged(coef), 32, symbol)
    v = np.random.default_rng(7).standard_normal((32, 32))
    ev2 = copy.copy(ev)
    ev2.r = ma.strain_apply(v, coef, rho, symbol)
    expect = ma.lbar_inverse(v, rho)
    for pc in ("none", "diag"):
        t, _ = ma.newton_direction(ev2, prob, 1.0, 0, 40, 1e-11, 40, symbol, pc)
        assert np.max(np.abs(t - expect)) <= 1e-8 * np.max(np.abs(expect)), pc


def test_diag_scaled_solve_reaches_the_same_potential_with_fewer_iterations():
    from paper_1009_6039_amd import workloads as W
    f, g = W.blobs(64, W.seed_for(1, 4))
    kw = dict(tol=1e-10, damping_policy="backtrack", gmres_tol=0.1, max_newton=300, symbol="fd4")
    p1, _, r1 = ma.solve(f, g, **kw)
    p2, _, r2 = ma.solve(f, g, precond="diag", **kw)
    assert r1.status == ma.OK and r2.status == ma.OK
    assert np.max(np.abs(p1 - p2)) <= 1e-8 * np.max(np.abs(p1))
    assert r2.gmres_iters < 0.8 * r1.gmres_iters, (r1.gmres_iters, r2.gmres_iters)
    with pytest.raises(ValueError):
        ma.solve(f, g, precond="jacobi")


def test_boundary_fraction_keeps_the_fixed_point():
    # the fraction-to-the-boundary rule only changes which steps are accepted: a strict
    # fraction halves more often and reaches the same potential; 0 is the plain rule
    from paper_1009_6039_amd import workloads as W
    f, g = W.blobs(64, W.seed_for(1, 6))
    kw = dict(tol=1e-10, damping_policy="backtrack", gmres_tol=0.1, max_newton=300, symbol="fd4")
    results = [ma.solve(f, g, boundary_frac=b, **kw) for b in (0.0, 0.1, 0.8)]
    assert all(r.status == ma.OK for _, _, r in results)
    ref = results[0][0]
    for psi, _, _ in results[1:]:
        assert np.max(np.abs(psi - ref)) <= 1e-8 * np.max(np.abs(ref))
    assert results[2][2].backtracks >= results[0][2].backtracks


def test_adaptive_forcing_keeps_the_fixed_point():
    # adaptive forcing only changes how accurately each direction is solved
    from paper_1009_6039_amd import workloads as W
    f, g = W.blobs(64, W.seed_for(1, 7))
    kw = dict(tol=1e-10, damping_policy="backtrack", gmres_tol=0.2, max_newton=300, symbol="fd4", precond="diag")
    p1, _, r1 = ma.solve(f, g, **kw)
    p2, _, r2 = ma.solve(f, g, forcing="adaptive", **kw)
    assert r1.status == ma.OK and r2.status == ma.OK
    assert np.max(np.abs(p1 - p2)) <= 1e-8 * np.max(np.abs(p1))
    with pytest.raises(ValueError):
        ma.solve(f, g, forcing="ew", **kw)


# --- orientation of the map: an asymmetric potential (Section 5.2 distance, Theorem CE1) ---

def asymmetric_manufactured(N, A=0.004, B=0.003):
    """psi* = A sin(2 pi x1) sin(4 pi x2) + B cos(2 pi x1), g = 1, f = det(I + D^2 psi*) in
    closed form (mean exactly one: det(I + H) - 1 - tr H is a divergence).  Returns the
    grid, psi*, its analytic gradient and f; d1 psi* and d2 psi* differ, so a map with
    its components exchanged (or built from the wrong axis) is far off."""
    x = np.arange(N) / N
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    s1, c1 = np.sin(2 * np.pi * X1), np.cos(2 * np.pi * X1)
    s4, c4 = np.sin(4 * np.pi * X2), np.cos(4 * np.pi * X2)
    ps = A * s1 * s4 + B * c1
    p1 = 2 * np.pi * A * c1 * s4 - 2 * np.pi * B * s1
    p2 = 4 * np.pi * A * s1 * c4
    p11 = -4 * np.pi ** 2 * A * s1 * s4 - 4 * np.pi ** 2 * B * c1
    p22 = -16 * np.pi ** 2 * A * s1 * s4
    p12 = 8 * np.pi ** 2 * A * c1 * c4
    f = (1 + p11) * (1 + p22) - p12 ** 2
    return X1, X2, ps, p1, p2, f


def test_map_components_follow_the_axes_for_an_asymmetric_potential():
    # T(x) = x + grad psi (Theorem CE1; Section 5.2): map[0] is x1 + d psi / d x1 and map[1]
    # is x2 + d psi / d x2, each to fourth order in h against the analytic gradient
    errs = []
    for N in (32, 64):
        X1, X2, ps, p1, p2, f = asymmetric_manufactured(N)
        psi, mp, rep = ma.solve(f, np.ones((N, N)), tau=1.0, tol=1e-11)
        assert rep.status == ma.OK
        e0 = np.max(np.abs(mp[0] - (X1 + p1)))
        e1 = np.max(np.abs(mp[1] - (X2 + p2)))
        errs.append(max(e0, e1))
        # exchanged components are off by the size of the gradient difference
        assert np.max(np.abs(mp[0] - (X1 + p2))) > 0.05 and np.max(np.abs(mp[1] - (X2 + p1))) > 0.05
        assert np.max(np.abs(mp[0] - (X2 + p1))) > 0.5  # wrong base coordinate
    assert errs[1] < 5e-6
    assert errs[0] / errs[1] > 12.0  # fourth order: 16 per halving of h


def test_w2_of_an_asymmetric_potential_against_quadrature():
    # d(f, g) = int |grad psi*|^2 f (Section 5.2) by the trapezoid rule on a fine grid (spectrally
    # accurate for smooth periodic integrands), independent of the solver's differences
    _, _, _, q1, q2, ff = asymmetric_manufactured(512)
    w2 = float(np.mean((q1 ** 2 + q2 ** 2) * ff))
    _, _, _, _, _, f = asymmetric_manufactured(64)
    _, _, rep = ma.solve(f, np.ones((64, 64)), tau=1.0, tol=1e-11)
    assert rep.w2sq == pytest.approx(w2, rel=1e-4)


# --- the simplified operator without the b . grad theta term (Remarks of Section 3.3) ---

def _nodrift_setup(N):
    x = np.arange(N) / N
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    f = 1 + 0.3 * np.cos(2 * np.pi * X1) * np.sin(2 * np.pi * X2)
    g = 1 + 0.4 * np.sin(2 * np.pi * (X1 + 0.2)) + 0.2 * np.cos(2 * np.pi * X2)  # grad g != 0: b != 0
    prob = ma.Problem(f, g)
    u = 0.01 * np.cos(2 * np.pi * X1) * np.sin(2 * np.pi * X2) + 0.004 * np.sin(2 * np.pi * (X1 - X2))
    return prob, ma.evaluate(u, prob), X1, X2


def test_no_drift_coefficients_drop_only_b():
    prob, ev, _, _ = _nodrift_setup(16)
    full = ma.coefficients(ev, 0)
    nd = ma.coefficients(ev, 1)
    for k in range(3):
        assert np.array_equal(full[k], nd[k])
    assert np.all(nd[3] == 0) and np.all(nd[4] == 0)
    assert np.max(np.abs(full[3])) > 0.1 and np.max(np.abs(full[4])) > 0.1


def test_no_drift_direction_solves_the_dense_operator_without_b():
    # op_mode 1: the Newton direction theta solves g Tr(Adj(I + D^2 u) D^2 theta) = h (no b term).
    # Dense spectral collocation (Trefethen's closed-form matrices) gives that operator
    # independently; h is taken in its range, h = L_nd theta_true with theta_true of mean zero.
    import copy
    N = 12
    prob, ev, X1, X2 = _nodrift_setup(N)
    a11, a12, a22, _, _ = ma.coefficients(ev, 1)
    Lnd = dense_operator((a11, a12, a22, 0.0, 0.0), N)
    theta_true = np.sin(2 * np.pi * X1 + 0.4) * np.cos(4 * np.pi * X2) + 0.3 * np.cos(2 * np.pi * X2)
    theta_true -= theta_true.mean()
    ev2 = copy.copy(ev)
    ev2.r = (Lnd @ theta_true.ravel()).reshape(N, N)
    th, its = ma.newton_direction(ev2, prob, 1.0, 1, N * N, 1e-12, 5)
    assert np.max(np.abs(th - theta_true)) < 1e-9 * np.max(np.abs(theta_true))
    # the full operator (with b . grad theta) gives another direction on the same h
    th_full, _ = ma.newton_direction(ev2, prob, 1.0, 0, N * N, 1e-12, 5)
    assert np.max(np.abs(th_full - theta_true)) > 1e-2 * np.max(np.abs(theta_true))


def test_no_drift_newton_reaches_the_same_fixed_point():
    # the simplified operator changes the path, not the discrete solution F(u) = 0.  The
    # paper only says it gives good results in practice; on a mild-contrast pair it does
    # (on the high-contrast blob pairs, density ratio about 20, its directions stall)
    N = 32
    prob, _, X1, X2 = _nodrift_setup(N)
    f = 1 + 0.3 * np.cos(2 * np.pi * X1) * np.sin(2 * np.pi * X2) + 0.1 * np.sin(4 * np.pi * X1)
    g = prob.g
    a, _, ra = ma.solve(f, g, tau=1.0, tol=1e-11)
    b, _, rb = ma.solve(f, g, tau=1.0, tol=1e-11, op_mode=1)
    assert ra.status == ma.OK and rb.status == ma.OK
    assert np.max(np.abs(a - b)) <= 1e-9 * np.max(np.abs(a))
    assert rb.gmres_iters > ra.gmres_iters  # the dropped term makes each direction cruder
