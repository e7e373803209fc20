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

  trilinear the 3-D tensor-product form of bilinear (oracle.ma3d).

Pins: tests/test_oracle_interp.py (exact at nodes; reproduces x1, x2 and x1*x2
inside the fundamental cell; periodic in y; nearest picks the closest node);
trilinear through tests/test_oracle_ma3d.py (x3-constant data reduce to bilinear,
and a planted swap of its weights fails).
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


def trilinear(F, y1, y2, y3):
    """Periodic trilinear interpolant of the 3-D grid field F at points (y1, y2, y3):
    the tensor product of the 1-D linear interpolants, the 3-D form of reading P4."""
    N = F.shape[0]
    lo, hi, frac = [], [], []
    for y in (y1, y2, y3):
        t = np.asarray(y, dtype=np.float64) * N
        f = np.floor(t)
        frac.append(t - f)
        lo.append(f.astype(np.int64) % N)
        hi.append((f.astype(np.int64) + 1) % N)
    out = 0.0
    for c1 in (0, 1):
        for c2 in (0, 1):
            for c3 in (0, 1):
                w = ((frac[0] if c1 else 1 - frac[0]) * (frac[1] if c2 else 1 - frac[1])
                     * (frac[2] if c3 else 1 - frac[2]))
                out = out + w * F[hi[0] if c1 else lo[0], hi[1] if c2 else lo[1], hi[2] if c3 else lo[2]]
    return out
