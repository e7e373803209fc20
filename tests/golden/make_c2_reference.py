"""Writes c2_noise_2048_reference.npz: the oracle's solution of the 2048 x 2048 smooth-noise pair.

The pair is workloads.smooth_noise(2048, seed_for(2, 0)) (f, g = exp(z/2) with z periodic
Gaussian-filtered white noise of width 4 cells, scaled to mean one).  The FP64 oracle
solves it with the paper's method (spectral symbols, fixed tau = 1, GMRES(10) at 1e-4)
to rms residual 1e-12, its floor at this size.  Stored: psi and the map x + D_h psi at
every 16th node in each direction (128 x 128 samples each), max |psi| over the whole
grid, and the solve's report.  The GPU parity test compares its potential at those
nodes.  Only the oracle and the input generator are called here.

  python tests/golden/make_c2_reference.py      (about 8 minutes on one core)
"""

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import ma  # noqa: E402
from paper_1009_6039_amd import workloads as W  # noqa: E402

N, STRIDE = 2048, 16
OUT = os.path.join(HERE, "c2_noise_2048_reference.npz")


def main():
    seed = W.seed_for(2, 0)
    f, g = W.smooth_noise(N, seed)
    t0 = time.time()
    psi, mp, rep = ma.solve(f, g, tau=1.0, tol=1e-12, gmres_tol=1e-4, max_newton=40)
    if rep.status != ma.OK:
        raise SystemExit("oracle did not converge: %r" % (rep,))
    np.savez_compressed(OUT, n=N, stride=STRIDE, seed=seed, psi=psi[::STRIDE, ::STRIDE],
                        map=mp[:, ::STRIDE, ::STRIDE], psi_absmax=np.max(np.abs(psi)),
                        res_rms=rep.res_rms, newton_iters=rep.newton_iters, gmres_iters=rep.gmres_iters)
    print("wrote %s: %d Newton, %d GMRES, residual %.3e, max|psi| %.6e, %.0f s"
          % (OUT, rep.newton_iters, rep.gmres_iters, rep.res_rms, np.max(np.abs(psi)), time.time() - t0))


if __name__ == "__main__":
    main()
