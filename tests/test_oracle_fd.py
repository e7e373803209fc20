"""Pins for oracle.fd: difference weights and Simpson weights (Section 4, Section 4.2)."""

import math

import numpy as np
import pytest
from scipy import integrate

from oracle import fd


@pytest.mark.parametrize("p", range(0, 7))
def test_first_derivative_weights_on_monomials(p):
    # d/dx x^p at 0 with h = 1 is 1 for p = 1 and 0 otherwise; fourth order => exact to p = 4
    s = sum(w * (o ** p) for o, w in fd.W1.items())
    exact = 1.0 if p == 1 else 0.0
    if p <= 4:
        assert s == pytest.approx(exact, abs=1e-14)
    elif p == 5:
        assert abs(s - exact) > 1.0  # the leading error term appears at degree 5


@pytest.mark.parametrize("p", range(0, 8))
def test_second_derivative_weights_on_monomials(p):
    s = sum(w * (o ** p) for o, w in fd.W2.items())
    exact = 2.0 if p == 2 else 0.0
    if p <= 5:
        assert s == pytest.approx(exact, abs=1e-13)
    elif p == 6:
        assert abs(s - exact) > 1.0


@pytest.mark.parametrize("N,k", [(16, 1), (16, 5), (32, 7), (32, 16), (24, 12)])
def test_symbols_on_fourier_modes(N, k):
    # on e^{2 pi i k x} the schemes multiply by their symbols, derived by hand:
    #   D1 -> i (8 sin t - sin 2t) / (6 h),  D11 -> (32 cos t - 2 cos 2t - 30) / (12 h^2),  t = 2 pi k h
    h = 1.0 / N
    t = 2 * math.pi * k * h
    x = np.arange(N) * h
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    e = np.exp(2j * math.pi * k * X1)
    s1 = 1j * (8 * math.sin(t) - math.sin(2 * t)) / (6 * h)
    s2 = (32 * math.cos(t) - 2 * math.cos(2 * t) - 30) / (12 * h * h)
    assert np.allclose(fd.d1(e, 0, h), s1 * e, atol=1e-9 * abs(s2) + 1e-12)
    assert np.allclose(fd.d2(e, 0, h), s2 * e, atol=1e-9 * abs(s2) + 1e-12)
    e2 = np.exp(2j * math.pi * k * (X1 + X2))
    assert np.allclose(fd.d12(e2, h), s1 * s1 * e2, atol=1e-9 * abs(s2) + 1e-12)
    e3 = np.exp(2j * math.pi * k * X2)
    assert np.allclose(fd.d1(e3, 1, h), s1 * e3, atol=1e-9 * abs(s2) + 1e-12)


def test_fourth_order_convergence_on_smooth_function():
    errs = []
    for N in (32, 64, 128):
        h = 1.0 / N
        x = np.arange(N) * h
        X1, X2 = np.meshgrid(x, x, indexing="ij")
        u = np.sin(2 * np.pi * X1) * np.cos(4 * np.pi * X2)
        exact12 = -2 * np.pi * 4 * np.pi * np.cos(2 * np.pi * X1) * np.sin(4 * np.pi * X2)
        errs.append(np.max(np.abs(fd.d12(u, h) - exact12)))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(3.9 < o < 4.1 for o in orders)


@pytest.mark.parametrize("N", [8, 16, 64])
def test_simpson_weights_match_library_simpson(N):
    # scipy's composite Simpson on [0,1] with N+1 samples, endpoint value repeated (periodic)
    rng = np.random.default_rng(N)
    y = rng.standard_normal(N)
    yy = np.append(y, y[0])
    lib = integrate.simpson(yy, x=np.linspace(0.0, 1.0, N + 1))
    assert fd.simpson_weights_1d(N) @ y == pytest.approx(lib, rel=1e-13, abs=1e-14)


def test_simpson_on_fourier_modes():
    N = 32
    w = fd.simpson_weights_1d(N)
    x = np.arange(N) / N
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    for k in range(1, N // 2):
        assert abs(w @ np.cos(2 * np.pi * k * x)) < 1e-14
        assert abs(w @ np.sin(2 * np.pi * k * x)) < 1e-14
    assert w @ np.cos(np.pi * N * x) == pytest.approx(-1.0 / 3.0, abs=1e-14)


def test_simpson_rejects_odd_grids():
    with pytest.raises(ValueError):
        fd.simpson_weights_1d(9)
