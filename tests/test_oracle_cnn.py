"""Pins for oracle.cnn: convolution, gradients, BF16 rounding, Adam."""

import numpy as np
import pytest

from oracle import cnn


def brute_conv(x, W, b):
    C_out, C_in = W.shape[:2]
    H, Wd = x.shape[1:]
    out = np.zeros((C_out, H, Wd))
    for co in range(C_out):
        for i in range(H):
            for j in range(Wd):
                s = b[co]
                for ci in range(C_in):
                    for a in range(3):
                        for c in range(3):
                            s += W[co, ci, a, c] * x[ci, (i + a - 1) % H, (j + c - 1) % Wd]
                out[co, i, j] = s
    return out


def test_convolution_matches_brute_force():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 5, 6))
    W = rng.standard_normal((2, 3, 3, 3))
    b = rng.standard_normal(2)
    assert np.allclose(cnn.conv3x3(x, W, b), brute_conv(x, W, b), atol=1e-12)


def test_convolution_commutes_with_periodic_shifts():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((4, 8, 8))
    W = rng.standard_normal((3, 4, 3, 3))
    b = rng.standard_normal(3)
    sh = lambda v: np.roll(np.roll(v, 3, axis=1), -2, axis=2)  # noqa: E731
    assert np.allclose(cnn.conv3x3(sh(x), W, b), sh(cnn.conv3x3(x, W, b)), atol=1e-12)


def _loss(params, x, t):
    c, _ = cnn.forward(x, params)
    return cnn.mse(c, t)


def test_gradients_match_central_differences():
    rng = np.random.default_rng(2)
    params = cnn.init_params(channels=4, layers=3, c_in=2, c_out=1, seed=3)
    params = [(W, rng.standard_normal(b.shape) * 0.1) for W, b in params]
    x = rng.standard_normal((2, 8, 8))
    t = rng.standard_normal((1, 8, 8))
    c, cache = cnn.forward(x, params)
    grads = cnn.backward(c, t, cache, params)
    eps = 1e-6
    for l in range(len(params)):
        W, b = params[l]
        for idx in [tuple(rng.integers(0, s) for s in W.shape) for _ in range(6)]:
            Wp, Wm = W.copy(), W.copy()
            Wp[idx] += eps
            Wm[idx] -= eps
            pp = list(params)
            pp[l] = (Wp, b)
            lp = _loss(pp, x, t)
            pp[l] = (Wm, b)
            lm = _loss(pp, x, t)
            fdv = (lp - lm) / (2 * eps)
            assert grads[l][0][idx] == pytest.approx(fdv, rel=1e-5, abs=1e-9)
        for k in range(b.shape[0]):
            bp, bm = b.copy(), b.copy()
            bp[k] += eps
            bm[k] -= eps
            pp = list(params)
            pp[l] = (W, bp)
            lp = _loss(pp, x, t)
            pp[l] = (W, bm)
            lm = _loss(pp, x, t)
            assert grads[l][1][k] == pytest.approx((lp - lm) / (2 * eps), rel=1e-5, abs=1e-9)


def test_input_gradient_matches_central_differences():
    rng = np.random.default_rng(4)
    x = rng.standard_normal((3, 6, 7))
    W = rng.standard_normal((2, 3, 3, 3))
    b = np.zeros(2)
    dz = rng.standard_normal((2, 6, 7))
    dx = cnn.conv3x3_input_grad(dz, W)
    eps = 1e-6
    for idx in [(0, 0, 0), (1, 5, 6), (2, 3, 2), (0, 2, 5)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += eps
        xm[idx] -= eps
        fdv = (np.sum(dz * cnn.conv3x3(xp, W, b)) - np.sum(dz * cnn.conv3x3(xm, W, b))) / (2 * eps)
        assert dx[idx] == pytest.approx(fdv, rel=1e-6)


@pytest.mark.parametrize("value,expected", [
    (1.0, 1.0),
    (1.0 + 2.0 ** -8, 1.0),                      # tie: mantissa of 1.0 is even
    (1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -6),      # tie between odd and even: to even
    (1.0 + 2.0 ** -8 + 2.0 ** -20, 1.0 + 2.0 ** -7),
    (3.14159265, 3.140625),
    (-3.14159265, -3.140625),
    (2.0 ** -130, 2.0 ** -130),                  # a subnormal that fits exactly
    (0.0, 0.0),
])
def test_bf16_rounding(value, expected):
    assert cnn.bf16_round(np.array([value]))[0] == expected


def test_adam_first_step_moves_by_the_learning_rate():
    # with bias correction the first step is lr * g / (|g| + eps)
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 0.0])
    p1, m, v = cnn.adam_step(p, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), atol=1e-15)
    assert p1[2] == p[2]


def test_training_reduces_the_loss():
    rng = np.random.default_rng(5)
    params = cnn.init_params(channels=4, layers=2, seed=6)
    x = rng.standard_normal((2, 8, 8))
    t = 0.5 * x[:1] - 0.3 * x[1:]
    ms = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
    vs = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
    c, _ = cnn.forward(x, params)
    l0 = cnn.mse(c, t)
    for step in range(1, 60):
        c, cache = cnn.forward(x, params)
        grads = cnn.backward(c, t, cache, params)
        new = []
        for l, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
            W, mW, vW = cnn.adam_step(W, gW, ms[l][0], vs[l][0], step, 0.01)
            b, mb, vb = cnn.adam_step(b, gb, ms[l][1], vs[l][1], step, 0.01)
            ms[l], vs[l] = (mW, mb), (vW, vb)
            new.append((W, b))
        params = new
    c, _ = cnn.forward(x, params)
    assert cnn.mse(c, t) < 0.2 * l0


def test_laplacian_target_and_head_invert_each_other():
    rng = np.random.default_rng(8)
    u = rng.standard_normal((16, 16))
    u -= u.mean()
    assert np.allclose(cnn.inverse_laplacian_fd4(cnn.laplacian_fd4(u)), u, atol=1e-10)
    # on a Fourier mode the target is the fourth-order symbol times the mode
    N = 32
    x = np.arange(N) / N
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    e = np.cos(2 * np.pi * 3 * X1)
    t = 2 * np.pi * 3 / N
    sym = (32 * np.cos(t) - 2 * np.cos(2 * t) - 30) * N * N / 12
    assert np.allclose(cnn.laplacian_fd4(e), sym * e, atol=1e-8)


def test_restriction_and_prolongation():
    N = 32
    x = np.arange(2 * N) / (2 * N)
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    assert np.allclose(cnn.restrict_full_weighting(np.full((2 * N, 2 * N), 3.0)), 3.0)
    # full weighting of a mode multiplies it by cos^2(pi k h) in each direction
    k = 3
    e = np.cos(2 * np.pi * k * X1)
    damp = np.cos(np.pi * k / (2 * N)) ** 2
    assert np.allclose(cnn.restrict_full_weighting(e), damp * e[::2, ::2], atol=1e-12)
    # bilinear prolongation reproduces coarse values at even nodes and averages between
    c = np.random.default_rng(9).standard_normal((8, 8))
    y = cnn.prolong_bilinear(c)
    assert np.array_equal(y[::2, ::2], c)
    assert np.allclose(y[1, 2], 0.5 * (c[0, 1] + c[1, 1]))
    assert np.allclose(y[15, 15], 0.25 * (c[7, 7] + c[0, 7] + c[7, 0] + c[0, 0]))


def test_batched_gradient_normalisation():
    rng = np.random.default_rng(10)
    params = cnn.init_params(channels=4, layers=2, seed=1)
    xs = [rng.standard_normal((2, 8, 8)) for _ in range(2)]
    ts = [rng.standard_normal((1, 8, 8)) for _ in range(2)]
    # the batch loss is the mean over all samples and pixels: per-sample gradients with
    # count = total elements add up to the gradient of the batch loss
    tot = None
    for x, t in zip(xs, ts):
        c, cache = cnn.forward(x, params)
        g = cnn.backward(c, t, cache, params, count=2 * 64)
        tot = g if tot is None else [(a[0] + b[0], a[1] + b[1]) for a, b in zip(tot, g)]
    l_batch = np.mean([cnn.mse(cnn.forward(x, params)[0], t) for x, t in zip(xs, ts)])
    eps = 1e-6
    W, b = params[0]
    Wp = W.copy()
    Wp[1, 0, 1, 2] += eps
    pp = [(Wp, b), params[1]]
    l_p = np.mean([cnn.mse(cnn.forward(x, pp)[0], t) for x, t in zip(xs, ts)])
    assert tot[0][0][1, 0, 1, 2] == pytest.approx((l_p - l_batch) / eps, rel=1e-4)


def test_zero_network_gives_the_linearised_solution():
    # For f = 1 + eps h, g = 1 the solution of the discrete equation satisfies
    # Laplacian_h(psi) = log f + O(eps^2), so a network that outputs zero must give a
    # start within O(eps^2) of the solver's answer; a wrong sign or a missing log ratio
    # leaves an O(eps) error.
    from oracle import ma
    N = 32
    x = np.arange(N) / N
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    h = np.cos(2 * np.pi * X1) * np.sin(4 * np.pi * X2) + 0.5 * np.sin(2 * np.pi * (X1 + X2))
    zero = [(np.zeros_like(W), np.zeros_like(b)) for W, b in cnn.init_params(channels=4, layers=2, seed=0)]
    errs = []
    for eps in (1e-2, 5e-3):
        f, g = 1.0 + eps * h, np.ones((N, N))
        psi, _, rep = ma.solve(f, g, tol=1e-13, max_newton=50)
        assert rep.status == ma.OK
        start = cnn.warm_start(f, g, zero, N, bf16=False)
        errs.append(np.max(np.abs(start - psi)))
        assert errs[-1] < 0.05 * np.max(np.abs(psi))
    assert 3.5 < errs[0] / errs[1] < 4.5  # second order in eps


def test_training_target_subtracts_the_log_ratio():
    rng = np.random.default_rng(11)
    psi = rng.standard_normal((16, 16)) * 1e-3
    f = 1.0 + 0.3 * rng.random((16, 16))
    g = 2.0 + rng.random((16, 16))
    t = cnn.training_target(psi, f, g)
    assert np.allclose(t, cnn.laplacian_fd4(psi) - np.log(f / f.mean()) + np.log(g / g.mean()), atol=1e-12)
    assert np.array_equal(cnn.training_target(psi), cnn.laplacian_fd4(psi))


def test_unflatten_inverts_the_flat_order():
    params = cnn.init_params(channels=4, layers=3, seed=2)
    flat = np.concatenate([np.concatenate([W.ravel(), b + 0.5]) for W, b in params])
    back = cnn.unflatten_params(flat, 3, 4)
    for (W, b), (W2, b2) in zip(params, back):
        assert np.array_equal(W, W2) and np.array_equal(b + 0.5, b2)
    with pytest.raises(ValueError):
        cnn.unflatten_params(flat[:-1], 3, 4)


def brute_conv_dilated(x, W, b, d):
    C_out, C_in = W.shape[:2]
    H, Wd = x.shape[1:]
    out = np.zeros((C_out, H, Wd))
    for co in range(C_out):
        for i in range(H):
            for j in range(Wd):
                s = b[co]
                for ci in range(C_in):
                    for a in range(3):
                        for c in range(3):
                            s += W[co, ci, a, c] * x[ci, (i + d * (a - 1)) % H, (j + d * (c - 1)) % Wd]
                out[co, i, j] = s
    return out


@pytest.mark.parametrize("d", [2, 3])
def test_dilated_convolution_matches_brute_force(d):
    rng = np.random.default_rng(20 + d)
    x = rng.standard_normal((2, 6, 9))
    W = rng.standard_normal((3, 2, 3, 3))
    b = rng.standard_normal(3)
    assert np.allclose(cnn.conv3x3(x, W, b, d), brute_conv_dilated(x, W, b, d), atol=1e-12)


def test_dilated_convolution_acts_on_interleaved_subgrids():
    # dilation d on an n x n grid = the undilated convolution on each of the d^2
    # subgrids of pixels with equal residues mod d (what the GPU tiles rely on)
    rng = np.random.default_rng(30)
    x = rng.standard_normal((2, 12, 12))
    W = rng.standard_normal((2, 2, 3, 3))
    b = rng.standard_normal(2)
    full = cnn.conv3x3(x, W, b, 3)
    for ry in range(3):
        for rx in range(3):
            assert np.allclose(full[:, ry::3, rx::3], cnn.conv3x3(x[:, ry::3, rx::3], W, b), atol=1e-12)


def test_dilated_gradients_match_central_differences():
    rng = np.random.default_rng(31)
    params = cnn.init_params(channels=4, layers=3, c_in=2, c_out=1, seed=5)
    params = [(W, rng.standard_normal(b.shape) * 0.1) for W, b in params]
    dil = [1, 2, 4]
    x = rng.standard_normal((2, 8, 8))
    t = rng.standard_normal((1, 8, 8))
    c, cache = cnn.forward(x, params, dilations=dil)
    grads = cnn.backward(c, t, cache, params, dilations=dil)
    eps = 1e-6
    for l in range(3):
        W, b = params[l]
        for idx in [tuple(rng.integers(0, s) for s in W.shape) for _ in range(4)]:
            Wp, Wm = W.copy(), W.copy()
            Wp[idx] += eps
            Wm[idx] -= eps
            pp = list(params)
            pp[l] = (Wp, b)
            lp = cnn.mse(cnn.forward(x, pp, dilations=dil)[0], t)
            pp[l] = (Wm, b)
            lm = cnn.mse(cnn.forward(x, pp, dilations=dil)[0], t)
            assert grads[l][0][idx] == pytest.approx((lp - lm) / (2 * eps), rel=1e-5, abs=1e-9)
