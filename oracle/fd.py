"""Fourth-order centred periodic finite differences and periodic Simpson weights.

TEST INFRASTRUCTURE ONLY (see the package header).

Section 4 of the paper evaluates the first and second derivatives of u_n with
fourth-order accurate centred differences, once per Newton iteration, on the
periodic N x N grid x_ij = (i h, j h), h = 1/N, where x = 0 and x = 1 coincide.
The paper names the scheme without printing its weights; the standard five-point
centred formulas are used (reading P3):

    D1 u_i  = ( u_{i-2} - 8 u_{i-1} + 8 u_{i+1} - u_{i+2}) / (12 h)
    D11 u_i = (-u_{i-2} + 16 u_{i-1} - 30 u_i + 16 u_{i+1} - u_{i+2}) / (12 h^2)
    D12 u   = D1 along x1 applied to D1 along x2

Array convention: ``u[i, j]`` is the value at (x1, x2) = (i h, j h); axis 0 is x1.

Section 4.2 averages the operator coefficients over the torus with Simpson's
rule.  On the periodic grid the composite rule with node N identified with
node 0 has 1-D weights 2h/3 at even i and 4h/3 at odd i (reading P7); the 2-D
rule is the tensor product.

Pins: tests/test_oracle_fd.py (weights reproduce derivatives of monomials to
degree 4 and fail at the next degree; closed-form symbols on Fourier modes;
Simpson weights sum to one and integrate every Fourier mode exactly except the
Nyquist mode, which they weight by -1/3).
"""

import numpy as np

# offset -> weight, before division by h (first derivative) or h^2 (second)
W1 = {-2: 1.0 / 12.0, -1: -8.0 / 12.0, 1: 8.0 / 12.0, 2: -1.0 / 12.0}
W2 = {-2: -1.0 / 12.0, -1: 16.0 / 12.0, 0: -30.0 / 12.0, 1: 16.0 / 12.0, 2: -1.0 / 12.0}


def _at(u, s, axis):
    """Periodic shift: returns v with v[i] = u[i + s] along `axis`."""
    return np.roll(u, -s, axis=axis)


def d1(u, axis, h):
    """Fourth-order centred first derivative along `axis` (Section 4)."""
    out = np.zeros(np.shape(u), dtype=np.result_type(u, np.float64))
    for s, w in W1.items():
        out += w * _at(u, s, axis)
    return out / h


def d2(u, axis, h):
    """Fourth-order centred second derivative along `axis` (Section 4)."""
    out = np.zeros(np.shape(u), dtype=np.result_type(u, np.float64))
    for s, w in W2.items():
        out += w * _at(u, s, axis)
    return out / (h * h)


def d12(u, h):
    """Mixed derivative: the first-derivative formula along x1 applied to the one along x2."""
    return d1(d1(u, 1, h), 0, h)


def derivatives(u, h):
    """(u1, u2, u11, u22, u12) at every grid point."""
    return d1(u, 0, h), d1(u, 1, h), d2(u, 0, h), d2(u, 1, h), d12(u, h)


def simpson_weights_1d(N):
    """Periodic composite Simpson weights on N nodes (N even), summing to one."""
    if N % 2:
        raise ValueError("Simpson's rule needs an even number of intervals")
    h = 1.0 / N
    w = np.where(np.arange(N) % 2 == 0, 2.0 * h / 3.0, 4.0 * h / 3.0)
    return w


def simpson_mean(a):
    """Simpson approximation of the integral over the unit torus of grid field `a`."""
    N = a.shape[0]
    w = simpson_weights_1d(N)
    return float(w @ a @ w)
