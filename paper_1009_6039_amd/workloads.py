"""Seeded synthetic input densities.

This module holds no arithmetic of the solver: it only draws the densities f, g
that both the GPU path and the CPU oracle receive as data.  The paper's own
inputs (MRI slices, photographs) are not available, so these recipes stand in
for them; each is a positive 1-periodic density on the unit torus scaled to
grid mean one.

Recipes
-------
manufactured(N, A)
    Section 5.1 procedure with g = 1: pick psi* = A sin(2 pi x1) sin(2 pi x2) and
    set f = det(I + D^2 psi*) in closed form, which has mean exactly one.
blobs(N, seed)
    0.1 + a sum of 8 periodic Gaussian blobs: centres uniform on the torus,
    widths uniform in [0.03, 0.1], peak weights uniform in [0.5, 1.5]; each blob
    is summed over its 3 x 3 nearest periodic images; then scaled to mean one.
    Draw order per density: centres (8 x 2), widths (8), weights (8); f first,
    then g, from numpy.random.default_rng(seed).
smooth_noise(N, seed, sigma_px)
    f = exp(z / 2) with z white noise filtered by a unit-gain periodic Gaussian
    of width sigma_px grid cells; scaled to mean one.  Draws f, then g.
e1_example(N, k, gamma, alpha, rho), e1_family(N, seed)
    the Section 5.1 family u* = (1/k) cos sin, g = 1 + alpha cos cos, f from eq. ma2.
e1_example3(N, k, alpha, rho), blobs3(N, seed)
    the same construction on the 3-torus, and 3-D blob densities (N x N x N).

Grid convention everywhere: F[i, j] is the value at (x1, x2) = (i/N, j/N).
"""

import numpy as np

SEED_BASE = 20261203
SEED_CONFIGS = 100        # configs 0 .. 99
SEED_INDICES = 10 ** 7    # pair indices 0 .. 10^7 - 1 per config
_SEED_HIGH = 10 ** 9      # offset of the seeds of pair indices >= 1000


def seed_for(config, index):
    """Seed of pair `index` of input config `config`; distinct (config, index) never share one.

    The first thousand pairs of each config take SEED_BASE + 1000 config + index; pair
    indices from 1000 on take SEED_BASE + 10^9 + 10^7 config + index, a range above every
    seed of the first kind.  Both maps are injective and their ranges are disjoint, so
    training, held-out and benchmark pairs drawn from different configs never coincide.
    """
    config, index = int(config), int(index)
    if not (0 <= config < SEED_CONFIGS and 0 <= index < SEED_INDICES):
        raise ValueError("seed_for: config must lie in [0, %d) and index in [0, %d)" % (SEED_CONFIGS, SEED_INDICES))
    if index < 1000:
        return SEED_BASE + 1000 * config + index
    return SEED_BASE + _SEED_HIGH + SEED_INDICES * config + index


def grid(N):
    x = np.arange(N, dtype=np.float64) / N
    return np.meshgrid(x, x, indexing="ij")


def manufactured(N, A=0.01):
    """(f, g, psi_star) for psi* = A sin(2 pi x1) sin(2 pi x2), g = 1."""
    X1, X2 = grid(N)
    s1, s2 = np.sin(2 * np.pi * X1), np.sin(2 * np.pi * X2)
    c1, c2 = np.cos(2 * np.pi * X1), np.cos(2 * np.pi * X2)
    c = 4.0 * np.pi ** 2 * A
    psi = A * s1 * s2
    # psi_11 = psi_22 = -c s1 s2, psi_12 = c c1 c2
    f = (1.0 - c * s1 * s2) ** 2 - (c * c1 * c2) ** 2
    g = np.ones((N, N))
    return f, g, psi


def e1_example(N, k=100.0, gamma=1, alpha=0.3, rho=1):
    """(f, g, u*) of the Section 5.1 example family with the parameters it leaves open:
    u* = (1/k) cos(2 pi gamma x1) sin(2 pi gamma x2), g = 1 + alpha cos(2 pi rho x1)
    cos(2 pi rho x2), f = g(x + grad u*) det(I + D^2 u*) in closed form (the paper's
    procedure: pick u and g, compute f from eq. ma2).  Defaults: amplitude 0.01, one
    period, alpha 0.3."""
    X1, X2 = grid(N)
    tp = 2.0 * np.pi
    a, w = 1.0 / k, tp * gamma
    s1, c1 = np.sin(w * X1), np.cos(w * X1)
    s2, c2 = np.sin(w * X2), np.cos(w * X2)
    u = a * c1 * s2
    u1, u2 = -a * w * s1 * s2, a * w * c1 * c2
    u11 = u22 = -a * w * w * c1 * s2
    u12 = -a * w * w * s1 * c2
    y1, y2 = X1 + u1, X2 + u2
    gy = 1.0 + alpha * np.cos(tp * rho * y1) * np.cos(tp * rho * y2)
    f = gy * ((1.0 + u11) * (1.0 + u22) - u12 * u12)
    g = 1.0 + alpha * np.cos(tp * rho * X1) * np.cos(tp * rho * X2)
    return f, g, u


def e1_family(N, seed):
    """One member of the Section 5.1 family with its open parameters drawn from a
    seeded generator: k in [80, 200] (amplitude 1/k; with one period the Hessian of u*
    stays below 4 pi^2 / 80 < 0.5, so |x|^2/2 + u* is uniformly convex), gamma = 1,
    alpha in [0.1, 0.5], rho in {1, 2, 3}.  Returns (f, g, u*)."""
    rng = np.random.default_rng(seed)
    k = float(rng.uniform(80.0, 200.0))
    alpha = float(rng.uniform(0.1, 0.5))
    rho = int(rng.integers(1, 4))
    return e1_example(N, k=k, gamma=1, alpha=alpha, rho=rho)


def grid3(N):
    x = np.arange(N, dtype=np.float64) / N
    return np.meshgrid(x, x, x, indexing="ij")


def e1_example3(N, k=100.0, alpha=0.3, rho=1):
    """(f, g, u*) of the Section 5.1 construction in three dimensions (the method is
    stated for any dimension): u* = (1/k) cos(2 pi x1) sin(2 pi x2) cos(2 pi x3),
    g = 1 + alpha cos(2 pi rho x1) cos(2 pi rho x2) cos(2 pi rho x3), and
    f = g(x + grad u*) det(I + D^2 u*) in closed form."""
    X1, X2, X3 = grid3(N)
    tp = 2.0 * np.pi
    a, w = 1.0 / k, tp
    s1, c1 = np.sin(w * X1), np.cos(w * X1)
    s2, c2 = np.sin(w * X2), np.cos(w * X2)
    s3, c3 = np.sin(w * X3), np.cos(w * X3)
    u = a * c1 * s2 * c3
    u1, u2, u3 = -a * w * s1 * s2 * c3, a * w * c1 * c2 * c3, -a * w * c1 * s2 * s3
    d = -a * w * w * c1 * s2 * c3  # u11 = u22 = u33
    u12 = -a * w * w * s1 * c2 * c3
    u13 = a * w * w * s1 * s2 * s3
    u23 = -a * w * w * c1 * c2 * s3
    m11 = m22 = m33 = 1.0 + d
    det = (m11 * (m22 * m33 - u23 * u23) - u12 * (u12 * m33 - u23 * u13) + u13 * (u12 * u23 - m22 * u13))
    y1, y2, y3 = X1 + u1, X2 + u2, X3 + u3
    gy = 1.0 + alpha * np.cos(tp * rho * y1) * np.cos(tp * rho * y2) * np.cos(tp * rho * y3)
    g = 1.0 + alpha * np.cos(tp * rho * X1) * np.cos(tp * rho * X2) * np.cos(tp * rho * X3)
    return gy * det, g, u


def blobs3(N, seed, count=6):
    """(f, g): independent 3-D densities, each a 0.2 floor plus `count` periodic
    Gaussian blobs (centres uniform, widths 0.06..0.12, weights 0.5..1.5), scaled to
    mean one; drawn from one generator, f first."""
    rng = np.random.default_rng(seed)
    x = np.arange(N, dtype=np.float64) / N

    def one():
        c = rng.uniform(0.0, 1.0, size=(count, 3))
        sg = rng.uniform(0.06, 0.12, size=count)
        wt = rng.uniform(0.5, 1.5, size=count)
        d = np.full((N, N, N), 0.2)
        for b in range(count):
            s2 = 2.0 * sg[b] ** 2
            e = [sum(np.exp(-(x - c[b, a] - p) ** 2 / s2) for p in (-1, 0, 1)) for a in range(3)]
            d += wt[b] * np.einsum("i,j,k->ijk", e[0], e[1], e[2])
        return d / d.mean()

    f = one()
    g = one()
    return f, g


def _blob_density(N, rng):
    x = np.arange(N, dtype=np.float64) / N
    centres = rng.uniform(0.0, 1.0, size=(8, 2))
    sigmas = rng.uniform(0.03, 0.1, size=8)
    weights = rng.uniform(0.5, 1.5, size=8)
    d = np.full((N, N), 0.1)
    for b in range(8):
        # the 3 x 3 image sum of a Gaussian factorises into two 1-D image sums
        s2 = 2.0 * sigmas[b] ** 2
        e1 = sum(np.exp(-(x - centres[b, 0] - p) ** 2 / s2) for p in (-1, 0, 1))
        e2 = sum(np.exp(-(x - centres[b, 1] - p) ** 2 / s2) for p in (-1, 0, 1))
        d += weights[b] * np.outer(e1, e2)
    return d / d.mean()


def blobs(N, seed):
    """(f, g): independent blob densities drawn from one generator."""
    rng = np.random.default_rng(seed)
    f = _blob_density(N, rng)
    g = _blob_density(N, rng)
    return f, g


def _noise_density(N, rng, sigma_px):
    xi = rng.standard_normal((N, N))
    k = np.fft.fftfreq(N, d=1.0 / N)
    K2 = k[:, None] ** 2 + k[None, :] ** 2
    filt = np.exp(-2.0 * np.pi ** 2 * sigma_px ** 2 * K2 / (N * N))
    z = np.fft.ifft2(np.fft.fft2(xi) * filt).real
    d = np.exp(0.5 * z)
    return d / d.mean()


def smooth_noise(N, seed, sigma_px=4.0):
    """(f, g): exp(z/2) densities from Gaussian-filtered periodic white noise."""
    rng = np.random.default_rng(seed)
    f = _noise_density(N, rng, sigma_px)
    g = _noise_density(N, rng, sigma_px)
    return f, g


def mixed_sizes(npairs, seed, sizes=(128, 256, 384, 512)):
    """Grid sizes for a batch of uneven pairs, drawn uniformly from `sizes`."""
    rng = np.random.default_rng(seed)
    return [int(s) for s in rng.choice(np.asarray(sizes), size=npairs)]
