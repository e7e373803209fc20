"""Pins for oracle.fd_bicg: the second-order stencil, the Lemma's augmented system,
BiCG, and the finite-difference Newton step (Section 4.1).

Each test checks the oracle against something other than itself: closed-form symbols
of the stencil on Fourier modes, grid convergence against analytic derivatives, the
Lemma's row construction done by hand, the Petrov-Galerkin conditions that define the
BiCG iterates (solved densely), and numbers the paper prints.
"""

import math
import os

import numpy as np
import pytest

from oracle import fd_bicg as fb
from oracle import ma
from paper_1009_6039_amd import workloads as W


def golden(name):
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)
    with open(path) as fh:
        return [line.split() for line in fh if line.strip() and not line.startswith("#")]


def const_coef(N, a11, a12, a22, b1, b2):
    return tuple(np.full((N, N), v) for v in (a11, a12, a22, b1, b2))


@pytest.mark.parametrize("k1,k2", [(1, 0), (0, 3), (2, -5), (4, 4), (8, 3), (-8, 8)])
def test_stencil_symbol_on_fourier_modes(k1, k2):
    # constant coefficients: A e_k = lambda(k) e_k with the symbol of the centred formulas
    # (t = 2 pi k h): a11 (2 cos t1 - 2)/h^2 - 2 a12 sin t1 sin t2 / h^2 + a22 (2 cos t2 - 2)/h^2
    # + i b1 sin t1 / h + i b2 sin t2 / h
    N = 16
    h = 1.0 / N
    c = (1.3, -0.4, 0.9, 2.5, -1.7)
    A = fb.fd2_matrix(const_coef(N, *c), N)
    x = np.arange(N) * h
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    e = np.exp(2j * math.pi * (k1 * X1 + k2 * X2)).ravel()
    t1, t2 = 2 * math.pi * k1 * h, 2 * math.pi * k2 * h
    lam = (c[0] * (2 * math.cos(t1) - 2) / h ** 2 - 2 * c[1] * math.sin(t1) * math.sin(t2) / h ** 2
           + c[2] * (2 * math.cos(t2) - 2) / h ** 2 + 1j * c[3] * math.sin(t1) / h
           + 1j * c[4] * math.sin(t2) / h)
    Ae = A @ e.real + 1j * (A @ e.imag)
    assert np.max(np.abs(Ae - lam * e)) <= 1e-10 * max(1.0, abs(lam))


def test_stencil_is_second_order_with_variable_coefficients():
    # L theta for theta = sin(2 pi x1) cos(4 pi x2) and smooth coefficients, against the
    # analytic derivatives: the max error falls by 4 per doubling of N
    errs = []
    for N in (32, 64, 128):
        h = 1.0 / N
        x = np.arange(N) * h
        X1, X2 = np.meshgrid(x, x, indexing="ij")
        s, c = np.sin, np.cos
        tw = 2 * math.pi
        coef = (1.0 + 0.3 * s(tw * X1) * c(tw * X2), 0.2 * c(tw * (X1 + X2)), 1.2 + 0.1 * s(tw * X2),
                0.5 * c(tw * X1), -0.7 * s(tw * X2) * s(tw * X1))
        th = s(tw * X1) * c(2 * tw * X2)
        t1 = tw * c(tw * X1) * c(2 * tw * X2)
        t2 = -2 * tw * s(tw * X1) * s(2 * tw * X2)
        t11 = -tw ** 2 * th
        t22 = -(2 * tw) ** 2 * th
        t12 = -2 * tw ** 2 * c(tw * X1) * s(2 * tw * X2)
        exact = coef[0] * t11 + 2 * coef[1] * t12 + coef[2] * t22 + coef[3] * t1 + coef[4] * t2
        A = fb.fd2_matrix(coef, N)
        errs.append(np.max(np.abs((A @ th.ravel()).reshape(N, N) - exact)))
    orders = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert all(abs(o - 2.0) < 0.05 for o in orders), orders


def test_lemma_construction_row_by_row():
    # hat A: the row sum x_k = 0 first, then A; that row added to every other row and
    # removed.  Every row of tilde A is the row of A plus a row of ones
    rng = np.random.default_rng(3)
    N = 4
    coef = tuple(rng.uniform(0.5, 1.5, (N, N)) for _ in range(5))
    A = fb.fd2_matrix(coef, N)
    At = fb.augmented_dense(A)
    Ad = A.toarray()
    P = N * N
    assert At.shape == (P, P)
    for k in range(P):
        assert np.array_equal(At[k], Ad[k] + 1.0)
    x = rng.standard_normal(P)
    assert np.allclose(fb.augmented_apply(A, x), At @ x, rtol=1e-13, atol=1e-10)
    assert np.allclose(fb.augmented_apply_t(A, x), At.T @ x, rtol=1e-13, atol=1e-10)


def test_lemma_solution_has_zero_sum_and_solves_a():
    # for b = A z with sum z = 0 the augmented system is nonsingular and returns z: the
    # zero-integral solution of A x = b that Section 4.1 selects
    rng = np.random.default_rng(4)
    N = 8
    h = 1.0 / N
    x = np.arange(N) * h
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    coef = (1.0 + 0.2 * np.sin(2 * np.pi * X1), 0.1 * np.cos(2 * np.pi * X2), 1.0 + 0.3 * np.cos(2 * np.pi * X1),
            0.4 * np.sin(2 * np.pi * X2), -0.3 * np.cos(2 * np.pi * X1))
    A = fb.fd2_matrix(coef, N)
    At = fb.augmented_dense(A)
    assert np.linalg.matrix_rank(A.toarray()) == N * N - 1
    assert np.linalg.matrix_rank(At) == N * N
    z = rng.standard_normal(N * N)
    z -= z.mean()
    sol = np.linalg.solve(At, A @ z)
    assert np.allclose(sol, z, atol=1e-9)
    assert abs(sol.sum()) < 1e-9


def krylov_basis(M, v, k):
    K = np.empty((v.size, k))
    w = v.copy()
    for j in range(k):
        K[:, j] = w
        w = M @ w
    Q, _ = np.linalg.qr(K)
    return Q


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bicg_iterates_are_the_petrov_galerkin_solutions(seed):
    # x_k lies in K_k(A, b) and b - A x_k is orthogonal to K_k(A^T, b) (shadow residual
    # r~_0 = b): solving that k x k projected system densely gives the same x_k
    rng = np.random.default_rng(seed)
    P = 30
    M = np.eye(P) * 4 + rng.standard_normal((P, P)) * 0.5
    b = rng.standard_normal(P)
    _, its, conv, hist = fb.bicg(lambda v: M @ v, lambda v: M.T @ v, b, tol=1e-12, maxit=200, history=True)
    assert conv
    for k in range(1, 7):
        V = krylov_basis(M, b, k)
        Wt = krylov_basis(M.T, b, k)
        y = np.linalg.solve(Wt.T @ M @ V, Wt.T @ b)
        xk = V @ y
        assert np.max(np.abs(hist[k - 1] - xk)) <= 1e-9 * np.max(np.abs(xk))
    assert np.allclose(hist[-1], np.linalg.solve(M, b), atol=1e-10)


def test_bicg_terminates_within_the_dimension():
    # in exact arithmetic at most P steps; a well-conditioned P = 12 system in FP64 too
    rng = np.random.default_rng(7)
    P = 12
    M = np.eye(P) * 3 + rng.standard_normal((P, P))
    b = rng.standard_normal(P)
    x, its, conv = fb.bicg(lambda v: M @ v, lambda v: M.T @ v, b, tol=1e-10, maxit=100)
    assert conv and its <= P
    assert np.allclose(M @ x, b, atol=1e-8)


def test_bicg_zero_rhs_and_breakdown():
    x, its, conv = fb.bicg(lambda v: v, lambda v: v, np.zeros(5))
    assert conv and its == 0 and not np.any(x)
    # A = [[0, 1], [1, 0]], b = e_1: p^T A p = 0 at once, the iteration stops with x = 0
    M = np.array([[0.0, 1.0], [1.0, 0.0]])
    x, its, conv = fb.bicg(lambda v: M @ v, lambda v: M.T @ v, np.array([1.0, 0.0]))
    assert not conv and its == 0 and not np.any(x)


def test_bicg_respects_the_iteration_cap():
    N = 32
    f, g, _ = W.e1_example(N)
    prob = ma.Problem(f, g)
    ev = ma.evaluate(np.zeros((N, N)), prob)
    _, its = fb.newton_direction(ma.coefficients(ev), ev.r, 1.0, 1e-12, 7)
    assert its == 7


def test_nyquist_mode_decays_at_the_rate_the_paper_reports():
    # Section 5.1: the residual of the finite-difference implementation decays by "about
    # 0.33" per iteration.  For a Nyquist-mode error (-1)^i the fourth-order residual's
    # symbol is -64/(12 h^2) and the second-order step's -4/h^2, so one tau = 1 step leaves
    # 1 - 64/48 = -1/3 of it
    N = 32
    f = np.ones((N, N))
    u0 = 1e-7 * (-1.0) ** np.arange(N)[:, None] * np.ones((1, N))
    prob = ma.Problem(f, f)
    ev0 = ma.evaluate(u0, prob)
    theta, _ = fb.newton_direction(ma.coefficients(ev0), ev0.r, 1.0, 1e-12, 1000)
    ev1 = ma.evaluate(u0 + theta, prob)
    rate = ev1.res_rms / ev0.res_rms
    assert rate == pytest.approx(1.0 / 3.0, abs=2e-4)
    assert np.allclose(ev1.r, -ev0.r / 3.0, atol=1e-4 * np.max(np.abs(ev0.r)))
    paper = {r[0]: float(r[1]) for r in golden("sec5_1_residual_ratio.txt")}
    assert abs(rate - paper["finite_differences"]) < 0.01


@pytest.mark.parametrize("gt", [1e-1, 1e-4])
def test_same_fixed_point_as_the_strain_implementation(gt):
    # both linear steps solve for the same residual equation: the converged potentials
    # agree to the residual tolerance (tau = 1 suffices for both, Section 5.1)
    N = 32
    f, g, _ = W.e1_example(N)
    p1, m1, r1 = ma.solve(f, g, tau=1.0, tol=1e-10, gmres_tol=gt, linear="fd_bicg", max_newton=200)
    p2, m2, r2 = ma.solve(f, g, tau=1.0, tol=1e-10, gmres_tol=gt, max_newton=200)
    assert r1.status == ma.OK and r2.status == ma.OK
    assert abs(np.mean(p1)) < 1e-15 and abs(np.mean(p2)) < 1e-15
    assert np.max(np.abs(p1 - p2)) <= 1e-7 * np.max(np.abs(p2))
    assert np.max(np.abs(m1 - m2)) <= 1e-7


def test_bicg_iterations_grow_with_n_as_table_1_reports():
    # Table 1: BiCG iterations per Newton step roughly double with N from N = 32 on
    # (17.79, 31.11, 63.32, 134.63), while GMRES's stay nearly constant.  The example's
    # constants are not given, so the trend is checked, not the values: each doubling
    # of N multiplies the oracle's count by a factor within 30% of the paper's
    rows = {int(r[0]): (float(r[1]), float(r[2])) for r in golden("sec5_1_table1_iterations.txt")}
    per = {}
    for N in (32, 64, 128):
        f, g, _ = W.e1_example(N)
        _, _, r = ma.solve(f, g, tau=1.0, tol=1e-9, gmres_tol=1e-1, linear="fd_bicg", max_newton=100)
        assert r.status == ma.OK
        per[N] = r.gmres_iters / r.newton_iters
    for N in (32, 64):
        ours = per[2 * N] / per[N]
        paper = rows[2 * N][1] / rows[N][1]
        assert abs(ours / paper - 1.0) < 0.3, (N, ours, paper)


def test_bicg_with_preconditioner_is_rejected():
    f = np.ones((16, 16))
    with pytest.raises(ValueError):
        ma.solve(f, f, linear="fd_bicg", precond="diag")
    with pytest.raises(ValueError):
        ma.solve(f, f, linear="cg")
