"""Periodic interpolation of grid data at displaced points.

TEST INFRASTRUCTURE ONLY (see the package header).

Section 4: when g is known only on the grid, g(x + grad u) and grad g(x + grad u)
must be approximated; the paper names linear interpolation and the closest
neighbour, reporting that the closest neighbour is good in most scenarios and
linear interpolation is better (Section 5.3).  Readings (P4):

  bilinear  t = y N, i0 = floor(t) mod N, weights from t - floor(t), applied
            periodically in both directions (the default);
  nearest   i = floor(y N + 1/2) mod N (ties round up).

Grid value F[i, j] sits at (i/N, j/N).

Pins: tests/test_oracle_interp.py (exact at nodes; reproduces x1, x2 and x1*x2
inside the fundamental cell; periodic in y; nearest picks the closest node).
"""

import numpy as np


def bilinear(F, y1, y2):
    """Periodic bilinear interpolant of grid field F at points (y1, y2)."""
    N = F.shape[0]
    t1 = np.asarray(y1, dtype=np.float64) * N
    t2 = np.asarray(y2, dtype=np.float64) * N
    f1 = np.floor(t1)
    f2 = np.floor(t2)
    a = t1 - f1
    b = t2 - f2
    i0 = f1.astype(np.int64) % N
    j0 = f2.astype(np.int64) % N
    i1 = (i0 + 1) % N
    j1 = (j0 + 1) % N
    return ((1 - a) * (1 - b) * F[i0, j0] + a * (1 - b) * F[i1, j0]
            + (1 - a) * b * F[i0, j1] + a * b * F[i1, j1])


def nearest(F, y1, y2):
    """Value of F at the grid node closest to (y1, y2), periodically."""
    N = F.shape[0]
    i = np.floor(np.asarray(y1, dtype=np.float64) * N + 0.5).astype(np.int64) % N
    j = np.floor(np.asarray(y2, dtype=np.float64) * N + 0.5).astype(np.int64) % N
    return F[i, j]
