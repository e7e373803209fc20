"""Pins for oracle.interp (Section 4 interpolation readings)."""

import numpy as np
import pytest

from oracle import interp


def _grid(N):
    x = np.arange(N) / N
    return np.meshgrid(x, x, indexing="ij")


def test_exact_at_nodes():
    N = 16
    F = np.random.default_rng(0).standard_normal((N, N))
    X1, X2 = _grid(N)
    assert np.array_equal(interp.bilinear(F, X1, X2), F)
    assert np.array_equal(interp.nearest(F, X1, X2), F)


def test_reproduces_bilinear_functions_inside_the_cell():
    # F = a + b i + c j + d i j sampled on nodes; away from the wrap the interpolant is exact
    N = 16
    I, J = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    F = 0.3 + 1.5 * I - 0.7 * J + 0.25 * I * J
    rng = np.random.default_rng(1)
    t1 = rng.uniform(0, N - 1, 500)
    t2 = rng.uniform(0, N - 1, 500)
    got = interp.bilinear(F, t1 / N, t2 / N)
    assert np.allclose(got, 0.3 + 1.5 * t1 - 0.7 * t2 + 0.25 * t1 * t2, rtol=1e-13, atol=1e-12)


def test_periodic_in_displacement():
    N = 16
    F = np.random.default_rng(2).standard_normal((N, N))
    rng = np.random.default_rng(3)
    y1, y2 = rng.uniform(-1, 2, 200), rng.uniform(-1, 2, 200)
    assert np.allclose(interp.bilinear(F, y1, y2), interp.bilinear(F, y1 + 1, y2 - 2), atol=1e-12)
    assert np.array_equal(interp.nearest(F, y1, y2), interp.nearest(F, y1 - 1, y2 + 1))


def test_nearest_picks_closest_node_and_rounds_ties_up():
    N = 8
    F = np.arange(N * N, dtype=float).reshape(N, N)
    assert interp.nearest(F, 0.49 / N, 0.0) == F[0, 0]
    assert interp.nearest(F, 0.51 / N, 0.0) == F[1, 0]
    assert interp.nearest(F, 0.5 / N, 0.0) == F[1, 0]
    assert interp.nearest(F, (N - 0.4) / N, 0.0) == F[0, 0]


def test_weights_are_a_partition_of_unity():
    N = 12
    rng = np.random.default_rng(4)
    y1, y2 = rng.uniform(0, 1, 300), rng.uniform(0, 1, 300)
    assert np.allclose(interp.bilinear(np.full((N, N), 2.5), y1, y2), 2.5, atol=1e-14)
