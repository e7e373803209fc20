"""The finite-difference linear step with BiCG (Section 4.1).

TEST INFRASTRUCTURE ONLY (see the package header).  FP64, SciPy sparse matrices.

What the paper fixes (Section 4.1):

* the Newton equation L theta = rhs of eq. (linma) is discretised with second-order
  centred differences for the derivatives of theta (the coefficients of L are those
  of eq. (linearmaeq), computed as in oracle.ma from fourth-order differences of u);
* the discrete system A x = b has a one-parameter family of solutions; the extra
  equation sum_k x_k = 0 is appended, then added to every other row and dropped,
  which leaves the square matrix tilde A = A + 1 1^T and the unchanged right-hand
  side (the Lemma gives the condition under which tilde A is nonsingular);
* tilde A x = b is solved by the biconjugate gradient method without a
  preconditioner, to a relative tolerance and an iteration cap (1e-4 or 1e-1, and
  1000 iterations per Newton step, in Section 5.1).

Readings taken where the paper is silent (listed with their pins in the design
notes):

* F1  grid x_ij = (i h, j h), h = 1/N, axis 0 is x1, unknowns ordered k = i N + j;
  the differences wrap periodically;
* F2  the centred second-order formulas
      D1 t  = (t_{i+1,j} - t_{i-1,j}) / (2h)
      D11 t = (t_{i+1,j} - 2 t_ij + t_{i-1,j}) / h^2
      D12 t = (t_{i+1,j+1} - t_{i+1,j-1} - t_{i-1,j+1} + t_{i-1,j-1}) / (4 h^2)
  (and the same along x2), so L_h theta = a11 D11 + 2 a12 D12 + a22 D22 + b1 D1 + b2 D2
  with pointwise coefficients (a nine-point stencil);
* F3  BiCG as in the textbooks (Fletcher's form): start x_0 = 0, shadow residual
  r~_0 = r_0, stop as soon as ||r_k||_2 <= tol ||b||_2 (the relative test GMRES uses);
  one iteration = one product with tilde A and one with tilde A^T; a zero
  denominator (breakdown) ends the iteration with the current iterate;
* F4  the Newton update u_{n+1} = u_n + x with the BiCG solution x as it comes (its
  mean is zero whenever b lies in the range of A).

Pins: tests/test_oracle_fd_bicg.py (the stencil's closed-form symbol on Fourier
modes; second-order consistency with variable coefficients; the Lemma's
construction row by row and its solution property; BiCG iterates equal to the
Petrov-Galerkin solutions that define them; the Nyquist decay rate of one Newton
step, 1/3, which the paper reports as about 0.33; the same fixed point as the
Strain implementation).
"""

import numpy as np
import scipy.sparse as sp


def _index(N, i, j):
    return (i % N) * N + (j % N)


def fd2_matrix(coef, N):
    """The P x P matrix A of L_h (reading F2), P = N^2, from the five coefficient
    planes (a11, a12, a22, b1, b2), each N x N."""
    a11, a12, a22, b1, b2 = (np.asarray(c, dtype=np.float64).reshape(N, N) for c in coef)
    h = 1.0 / N
    I, J = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    row = _index(N, I, J).ravel()
    rows, cols, vals = [], [], []

    def add(di, dj, w):
        rows.append(row)
        cols.append(_index(N, I + di, J + dj).ravel())
        vals.append(np.asarray(w).ravel())

    # second derivatives
    add(1, 0, a11 / h ** 2)
    add(-1, 0, a11 / h ** 2)
    add(0, 0, -2.0 * a11 / h ** 2)
    add(0, 1, a22 / h ** 2)
    add(0, -1, a22 / h ** 2)
    add(0, 0, -2.0 * a22 / h ** 2)
    # mixed derivative, with the factor 2 of the operator
    m = 2.0 * a12 / (4.0 * h ** 2)
    add(1, 1, m)
    add(1, -1, -m)
    add(-1, 1, -m)
    add(-1, -1, m)
    # first derivatives
    add(1, 0, b1 / (2.0 * h))
    add(-1, 0, -b1 / (2.0 * h))
    add(0, 1, b2 / (2.0 * h))
    add(0, -1, -b2 / (2.0 * h))
    P = N * N
    # duplicate (row, col) entries are summed by the conversion
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(P, P)).tocsr()


def augmented_dense(A):
    """tilde A built as the Lemma describes, densely (small systems only): the
    (P+1) x P matrix hat A with the row of ones first, that row added to every other
    row, then removed."""
    Ad = A.toarray() if sp.issparse(A) else np.asarray(A, dtype=np.float64)
    P = Ad.shape[1]
    hat = np.vstack([np.ones((1, P)), Ad])
    for k in range(1, P + 1):
        hat[k] = hat[k] + hat[0]
    return hat[1:]


def augmented_apply(A, x):
    """tilde A x = A x + (sum x) 1, without forming the dense row."""
    return A @ x + np.sum(x)


def augmented_apply_t(A, y):
    """tilde A^T y = A^T y + (sum y) 1."""
    return A.T @ y + np.sum(y)


def bicg(apply, apply_t, b, tol=1e-4, maxit=1000, history=False):
    """BiCG for apply(x) = b (reading F3).  Returns (x, iterations, converged) and,
    with history=True, also the list of iterates x_1, x_2, ...."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    hist = []
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        return (x, 0, True, hist) if history else (x, 0, True)
    r = b.copy()
    rt = r.copy()
    p = r.copy()
    pt = rt.copy()
    rho = float(rt @ r)
    its = 0
    converged = False
    while its < maxit:
        q = apply(p)
        qt = apply_t(pt)
        sigma = float(pt @ q)
        if sigma == 0.0 or not np.isfinite(sigma):
            break
        alpha = rho / sigma
        x = x + alpha * p
        r = r - alpha * q
        rt = rt - alpha * qt
        its += 1
        if history:
            hist.append(x.copy())
        if float(np.linalg.norm(r)) <= tol * bnorm:
            converged = True
            break
        rho_new = float(rt @ r)
        if rho_new == 0.0 or not np.isfinite(rho_new):
            break
        beta = rho_new / rho
        rho = rho_new
        p = r + beta * p
        pt = rt + beta * pt
    return (x, its, converged, hist) if history else (x, its, converged)


def newton_direction(coef, r, rhs_scale, tol, maxit):
    """theta solving tilde A theta = r * rhs_scale by BiCG (Section 4.1); returns
    (theta, iterations)."""
    N = r.shape[0]
    A = fd2_matrix(coef, N)
    b = (r * rhs_scale).ravel()
    x, its, _ = bicg(lambda v: augmented_apply(A, v), lambda v: augmented_apply_t(A, v), b, tol, maxit)
    return x.reshape(N, N), its
