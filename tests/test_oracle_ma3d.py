"""Pins for oracle.ma3d: the 3-D residual, linearisation, Strain operator and Newton loop.

Each test checks the 3-D oracle against something other than itself: a library
determinant and inverse, the pinned 2-D oracle on data that do not depend on x3, dense
Kronecker products of the closed-form spectral collocation matrices, a central
difference of the discrete residual, manufactured solutions (discrete-exact and
analytic), and a fine-grid quadrature.
"""

import math

import numpy as np
import pytest

from oracle import fd, ma, ma3d
from paper_1009_6039_amd import workloads as W


def trefethen_d1(N):
    """Closed-form Fourier first-derivative matrix on [0, 1) with N (even) nodes."""
    h = 2 * math.pi / N
    D = np.zeros((N, N))
    for j in range(N):
        for l in range(N):
            if j != l:
                D[j, l] = 0.5 * (-1) ** (j - l) / math.tan((j - l) * h / 2)
    return 2 * math.pi * D


def trefethen_d2(N):
    """Closed-form Fourier second-derivative matrix on [0, 1) (not the square of D1)."""
    h = 2 * math.pi / N
    D = np.zeros((N, N))
    for j in range(N):
        for l in range(N):
            if j == l:
                D[j, l] = -math.pi ** 2 / (3 * h * h) - 1.0 / 6.0
            else:
                D[j, l] = -((-1) ** (j - l)) / (2 * math.sin((j - l) * h / 2) ** 2)
    return 4 * math.pi ** 2 * D


def along(D, a, N):
    """The 1-D matrix D acting along axis a of an N x N x N array (C order)."""
    I = np.eye(N)
    mats = [I, I, I]
    mats[a] = D
    return np.kron(np.kron(mats[0], mats[1]), mats[2])


def asymmetric3(N, A=0.004):
    """psi* with different dependence on each axis, its gradient and the f it gives with
    g = 1 (f = det(I + D^2 psi*) in closed form)."""
    X1, X2, X3 = W.grid3(N)
    t = 2 * np.pi
    s, c = np.sin, np.cos
    psi = A * (s(t * X1) * s(2 * t * X2) * c(t * X3) + 0.5 * c(t * X1) + 0.3 * s(t * X3) * c(t * X2))
    p1 = A * (t * c(t * X1) * s(2 * t * X2) * c(t * X3) - 0.5 * t * s(t * X1))
    p2 = A * (2 * t * s(t * X1) * c(2 * t * X2) * c(t * X3) - 0.3 * t * s(t * X3) * s(t * X2))
    p3 = A * (-t * s(t * X1) * s(2 * t * X2) * s(t * X3) + 0.3 * t * c(t * X3) * c(t * X2))
    p11 = A * (-t * t * s(t * X1) * s(2 * t * X2) * c(t * X3) - 0.5 * t * t * c(t * X1))
    p22 = A * (-4 * t * t * s(t * X1) * s(2 * t * X2) * c(t * X3) - 0.3 * t * t * s(t * X3) * c(t * X2))
    p33 = A * (-t * t * s(t * X1) * s(2 * t * X2) * c(t * X3) - 0.3 * t * t * s(t * X3) * c(t * X2))
    p12 = A * (2 * t * t * c(t * X1) * c(2 * t * X2) * c(t * X3))
    p13 = A * (-t * t * c(t * X1) * s(2 * t * X2) * s(t * X3))
    p23 = A * (-2 * t * t * s(t * X1) * c(2 * t * X2) * s(t * X3) - 0.3 * t * t * c(t * X3) * s(t * X2))
    M = np.array([[1 + p11, p12, p13], [p12, 1 + p22, p23], [p13, p23, 1 + p33]])
    f = np.linalg.det(np.moveaxis(M, (0, 1), (-2, -1)))
    return (X1, X2, X3), psi, (p1, p2, p3), f


def test_cofactors_are_det_times_inverse():
    rng = np.random.default_rng(0)
    B = rng.standard_normal((7, 3, 3))
    S = np.eye(3) * 3 + 0.5 * (B + np.transpose(B, (0, 2, 1)))
    M = (S[:, 0, 0], S[:, 1, 1], S[:, 2, 2], S[:, 0, 1], S[:, 0, 2], S[:, 1, 2])
    cof, det = ma3d.cofactors(M)
    assert np.allclose(det, np.linalg.det(S), rtol=1e-13)
    adj = np.linalg.det(S)[:, None, None] * np.linalg.inv(S)
    for (a, b), cv in zip(ma3d.PAIRS, cof):
        assert np.allclose(cv, adj[:, a, b], rtol=1e-12, atol=1e-12)


def test_x3_independent_data_reduce_to_the_2d_solver():
    # with f, g constant along x3, u stays constant along x3: M = diag(2-D block, 1), the
    # cofactors a11, a22, a12 and b1, b2 are the 2-D coefficients, a13 = a23 = b3 = 0, and
    # the trilinear interpolation at nodes along x3 is the bilinear one
    N = 16
    f2, g2 = W.blobs(N, W.seed_for(0, 7))
    f2 = 0.8 + 0.2 * f2  # milder contrast: fixed tau = 1 converges
    g2 = 0.8 + 0.2 * g2
    f3 = np.repeat(f2[:, :, None], N, axis=2)
    g3 = np.repeat(g2[:, :, None], N, axis=2)
    p2, m2, r2 = ma.solve(f2, g2, tau=1.0, tol=1e-10, gmres_tol=1e-6)
    p3, m3, r3 = ma3d.solve3(f3, g3, tau=1.0, tol=1e-10, gmres_tol=1e-6)
    assert r2.status == ma.OK and r3.status == ma.OK
    assert r3.newton_iters == r2.newton_iters
    for k in range(N):
        assert np.max(np.abs(p3[:, :, k] - p2)) <= 1e-10 * np.max(np.abs(p2))
        assert np.max(np.abs(m3[0][:, :, k] - m2[0])) <= 1e-10
        assert np.max(np.abs(m3[1][:, :, k] - m2[1])) <= 1e-10
    X3 = W.grid3(N)[2]
    assert np.max(np.abs(m3[2] - X3)) <= 1e-12
    assert r3.w2sq == pytest.approx(r2.w2sq, rel=1e-10)


def test_strain_operator_matches_dense_collocation():
    # A v = L Lbar^+ v with L = sum c_ab D_ab + sum b_a D_a built from Kronecker products of
    # the closed-form collocation matrices (D_aa the second-derivative matrix, D_ab = D_a D_b)
    N = 8
    rng = np.random.default_rng(1)
    d1, d2 = trefethen_d1(N), trefethen_d2(N)
    Da = [along(d1, a, N) for a in range(3)]
    Daa = [along(d2, a, N) for a in range(3)]
    coef = tuple(1.0 + 0.3 * rng.standard_normal((N, N, N)) if k < 3 else 0.2 * rng.standard_normal((N, N, N))
                 for k in range(9))
    abar = ma3d.averaged3(coef)

    def op(cs):
        L = 0
        for w, (a, b) in zip(cs[:6], ma3d.PAIRS):
            Dab = Daa[a] if a == b else Da[a] @ Da[b]
            L = L + (1.0 if a == b else 2.0) * (np.diag(np.ravel(w)) if np.ndim(w) else w * np.eye(N ** 3)) @ Dab
        for k in range(3):
            w = cs[6 + k]
            L = L + (np.diag(np.ravel(w)) if np.ndim(w) else w * np.eye(N ** 3)) @ Da[k]
        return L

    Lbar_pinv = np.linalg.pinv(op(abar), rcond=1e-10)
    A = op(coef) @ Lbar_pinv
    rho = ma3d.symbol3(abar, N)
    for _ in range(3):
        v = rng.standard_normal((N, N, N))
        got = ma3d.strain_apply3(v, coef, rho)
        want = (A @ v.ravel()).reshape(N, N, N)
        assert np.max(np.abs(got - want)) <= 1e-9 * np.max(np.abs(want))
        th = ma3d.lbar_inverse3(v, rho)
        assert np.max(np.abs(th.ravel() - Lbar_pinv @ v.ravel())) <= 1e-9 * np.max(np.abs(th))


def g_analytic3(alpha=0.3, rho=1):
    t = 2 * np.pi * rho

    def g(y1, y2, y3):
        c1, c2, c3 = np.cos(t * y1), np.cos(t * y2), np.cos(t * y3)
        s1, s2, s3 = np.sin(t * y1), np.sin(t * y2), np.sin(t * y3)
        return (1 + alpha * c1 * c2 * c3, -alpha * t * s1 * c2 * c3, -alpha * t * c1 * s2 * c3,
                -alpha * t * c1 * c2 * s3)
    return g


def test_linearisation_is_the_derivative_of_the_discrete_residual():
    # (M(u + eps theta) - M(u - eps theta)) / (2 eps) = sum_a a_aa theta_aa + 2 sum a_ab theta_ab
    # + b . grad theta with the same differences (eq. linearmaeq), analytic g
    N = 12
    X1, X2, X3 = W.grid3(N)
    t = 2 * np.pi
    u = 0.004 * np.sin(t * X1) * np.cos(t * X2 + 0.3) * np.sin(t * X3 + 0.7) + 0.002 * np.cos(t * (X1 - X3))
    th = np.cos(t * X1 + 0.2) * np.sin(t * X2) * np.cos(2 * t * X3) + 0.5 * np.sin(t * (X2 + X3))
    f = np.ones((N, N, N))
    prob = ma3d.Problem3(f, f, g_analytic=g_analytic3())
    # det is cubic in eps: the central difference is off by eps^2 det(D_h^2 theta) ~ 1e-12 * 150^3
    eps = 1e-6
    fp = ma3d.evaluate3(u + eps * th, prob).fn
    fm = ma3d.evaluate3(u - eps * th, prob).fn
    deriv = (fp - fm) / (2 * eps)
    ev = ma3d.evaluate3(u, prob)
    coef = ma3d.coefficients3(ev)
    grad, sec = ma3d.derivatives3(th, prob.h)
    lin = sum((1.0 if a == b else 2.0) * c * s for c, s, (a, b) in zip(coef[:6], sec, ma3d.PAIRS))
    lin = lin + sum(coef[6 + k] * grad[k] for k in range(3))
    assert np.max(np.abs(deriv - lin)) <= 1e-7 * np.max(np.abs(lin))


def test_discrete_exact_manufactured_solution():
    # f := det(I + D_h^2 psi*) translated to mean one, g = 1: the oracle returns psi*
    N = 12
    _, psi, _, _ = asymmetric3(N)
    _, sec = ma3d.derivatives3(psi, 1.0 / N)
    M = tuple((1.0 if a == b else 0.0) + s for (a, b), s in zip(ma3d.PAIRS, sec))
    _, det = ma3d.cofactors(M)
    f = det - det.mean() + 1.0
    out, _, rep = ma3d.solve3(f, np.ones((N, N, N)), tau=1.0, tol=1e-12, gmres_tol=1e-8)
    assert rep.status == ma3d.OK
    assert np.max(np.abs(out - (psi - psi.mean()))) <= 1e-10 * np.max(np.abs(psi))


def test_fourth_order_convergence_with_analytic_g():
    # the Section 5.1 construction in 3-D with g known in closed form: the error against
    # u* falls as h^4 (the paper's observed orders in 2-D are 4.0)
    errs = []
    for N in (8, 16, 32):
        f, g, us = W.e1_example3(N)
        psi, _, rep = ma3d.solve3(f, g, tau=1.0, tol=1e-12, gmres_tol=1e-8, g_analytic=g_analytic3())
        assert rep.status == ma3d.OK
        e = psi - (us - us.mean())
        errs.append(float(np.sqrt(np.mean(e * e))))
    orders = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert 3.6 < orders[1] < 4.4, orders


def test_map_components_and_w2_for_an_asymmetric_potential():
    # map[a] = x_a + d_a psi (fourth order), exchanged components fail; W2 = int |grad psi|^2 f
    # against a trapezoid quadrature on a fine grid (spectrally accurate for periodic data)
    _, _, gf, ff = asymmetric3(48)
    w2 = float(np.mean((gf[0] ** 2 + gf[1] ** 2 + gf[2] ** 2) * ff))
    errs, w2err = [], []
    for N in (12, 24):
        X, psi, grad, f = asymmetric3(N)
        _, mp, rep = ma3d.solve3(f, np.ones((N, N, N)), tau=1.0, tol=1e-12, gmres_tol=1e-8)
        assert rep.status == ma3d.OK
        errs.append(max(float(np.max(np.abs(mp[a] - (X[a] + grad[a])))) for a in range(3)))
        w2err.append(abs(rep.w2sq - w2) / w2)
        assert np.max(np.abs(mp[0] - (X[0] + grad[1]))) > 0.02
        assert np.max(np.abs(mp[2] - (X[2] + grad[0]))) > 0.02
    # fourth order in both: 16 per halving of h
    assert errs[0] / errs[1] > 12.0
    assert w2err[0] / w2err[1] > 12.0 and w2err[1] < 5e-3, w2err


def test_equal_densities_take_no_step_and_no_drift_reaches_the_same_point():
    N = 8
    f, _, _ = W.e1_example3(N)
    psi, _, rep = ma3d.solve3(f, f.copy(), tol=1e-10)
    assert rep.status == ma3d.OK and rep.newton_iters == 0 and not np.any(psi)
    f, g, _ = W.e1_example3(12)
    a, _, ra = ma3d.solve3(f, g, tol=1e-11, gmres_tol=1e-6)
    b, _, rb = ma3d.solve3(f, g, tol=1e-11, gmres_tol=1e-6, op_mode=1)
    assert ra.status == ma3d.OK and rb.status == ma3d.OK
    assert np.max(np.abs(a - b)) <= 1e-8 * np.max(np.abs(a))
    ev = ma3d.evaluate3(a, ma3d.Problem3(f, g))
    c0, c1 = ma3d.coefficients3(ev, 0), ma3d.coefficients3(ev, 1)
    assert all(np.array_equal(x, y) for x, y in zip(c0[:6], c1[:6]))
    assert not any(np.any(c) for c in c1[6:]) and any(np.any(c) for c in c0[6:])


def test_invalid_arguments_are_rejected():
    f = np.ones((8, 8, 8))
    for bad in (dict(f=np.ones((7, 7, 7)), g=np.ones((7, 7, 7))), dict(tau=0.5), dict(tol=0.0)):
        kw = dict(f=f, g=f, tau=1.0, tol=1e-6)
        kw.update(bad)
        with pytest.raises(ValueError):
            ma3d.solve3(kw.pop("f"), kw.pop("g"), **kw)
    neg = f.copy()
    neg[1, 2, 3] = -1.0
    with pytest.raises(ValueError):
        ma3d.solve3(neg, f)


def test_simpson_mean3_is_the_tensor_rule():
    # the periodic composite Simpson rule in each direction (reading P7): a product of 1-D
    # fields integrates to the product of scipy's Simpson integrals on the closed grid, and
    # the Nyquist mode along one axis gets the weight -1/3 (the plain mean would give 0)
    from scipy.integrate import simpson
    N = 10
    rng = np.random.default_rng(3)
    vs = [rng.standard_normal(N) for _ in range(3)]
    field = np.einsum("i,j,k->ijk", *vs)
    x = np.arange(N + 1) / N
    want = np.prod([simpson(np.append(v, v[0]), x=x) for v in vs])
    assert ma3d.simpson_mean3(field) == pytest.approx(want, rel=1e-12)
    nyq = np.broadcast_to(((-1.0) ** np.arange(N))[:, None, None], (N, N, N))
    assert ma3d.simpson_mean3(nyq) == pytest.approx(-1.0 / 3.0, rel=1e-12)
