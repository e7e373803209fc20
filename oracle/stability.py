"""Spectral radius of the inverse of the linearised operator by power iteration (Section 5.1).

TEST INFRASTRUCTURE ONLY (see the package header).  FP64 throughout.

Section 5.1 measures the stability of the FFT implementation by the spectral
radius of A_n^{-1}, the inverse of the discretised linearised Monge-Ampere
operator at Newton step n, with the power method: b_{k+1} = A_n^{-1} b_k /
||A_n^{-1} b_k||_2 from a b_0 with components drawn uniformly in [0, 1], where each
product A_n^{-1} b_k is computed by the method of Section 4.2 (GMRES on
L Lbar^{-1} sigma = b_k, then theta = Lbar^{-1} sigma).  The paper reports that the
iteration settles near 0.03 after about five steps, for every Newton step and grid.

Readings: A_n maps the periodic fields onto (close to) the mean-zero ones and its
inverse of Section 4.2 returns mean-zero fields (rhobar(0) = 0), so the power method
runs on the mean-zero subspace: the mean of b_0 is removed before the first product
(a constant part is outside A_n's range and would only stall the first GMRES solve).
The estimate after step k is rho_k = ||A_n^{-1} b_k||_2 for the unit vector b_k.  The
linear solves run at a tight GMRES tolerance so that rho_k measures the operator,
not the solver.

Pins: tests/test_oracle_stability.py (g = 1 at u = 0: A_n = the Laplacian, whose
inverse on mean-zero fields has spectral radius 1/(4 pi^2); constant anisotropic
coefficients with drift: the Fourier modes are the eigenvectors, radius
1 / min_k |S(k)|; the Section 5.1 value on the manufactured example).
"""

import numpy as np

from . import ma


def apply_inverse(b, coef, rho, symbol="spectral", gmres_m=10, gmres_tol=1e-8, gmres_max_restarts=50):
    """theta = A^{-1} b by Section 4.2: GMRES on L Lbar^{-1} sigma = b, theta = Lbar^{-1} sigma."""
    sigma, its, _ = ma.gmres(lambda v: ma.strain_apply(v, coef, rho, symbol), b, m=gmres_m, tol=gmres_tol,
                             max_restarts=gmres_max_restarts)
    return ma.lbar_inverse(sigma, rho), its


def power_inverse(coef, abar, b0, iters=8, symbol="spectral", **gmres_kw):
    """Power iteration on A^{-1} for the operator with coefficients `coef` and averages
    `abar`; returns (rho_k for k = 0 .. iters-1, GMRES iterations per product)."""
    N = b0.shape[0]
    rho = ma.symbol(abar, N, symbol)
    b = np.asarray(b0, dtype=np.float64)
    b = b - np.mean(b)
    b = b / np.linalg.norm(b)
    out, its = [], []
    for _ in range(iters):
        t, k = apply_inverse(b, coef, rho, symbol, **gmres_kw)
        nt = float(np.linalg.norm(t))
        out.append(nt)
        its.append(k)
        b = t / nt
    return np.array(out), its


def newton_operator(u, prob, op_mode=0):
    """Coefficients and Simpson averages of the linearised operator at iterate u."""
    ev = ma.evaluate(u, prob)
    coef = ma.coefficients(ev, op_mode)
    return coef, ma.averaged(coef)
