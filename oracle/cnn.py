"""The warm-start network in FP64: periodic 3x3 convolutions, ReLU, MSE loss, Adam.

TEST INFRASTRUCTURE ONLY (see the package header).

The network is not part of the paper; it supplies the Newton initial guess.
Layers l = 0..L-1: z_l = conv3x3_periodic(h_l, W_l) + b_l, h_{l+1} = relu(z_l) for
l < L-1 and h_L = z_{L-1} (no activation on the output).  Input channels are
(log f, log g) for densities scaled to mean one.  Linearised about psi = 0 the
equation of Section 2 reads Laplacian(psi) = log f - log g; the output c approximates
what that misses of the fourth-order difference Laplacian of the solver's potential,
and the initial guess is psi0 = (discrete Laplacian)^{-1} (c + log f - log g) with
zero mean (the head, applied outside the network).

Convolution convention: out[co, i, j] = b[co] + sum_{ci, a, b} W[co, ci, a, b] *
x[ci, (i + d(a - 1)) mod H, (j + d(b - 1)) mod W], a, b in {0, 1, 2}, with the
layer's dilation d (1 unless given).

Optional BF16 emulation (`bf16=True`): the GPU kernels store inputs, weights and
inter-layer activations in BF16 (round to nearest even) and accumulate in FP32;
the oracle then rounds the same tensors to BF16 values and accumulates in FP64.

Pins: tests/test_oracle_cnn.py (convolution against a brute-force loop and
against translation invariance; gradients against central differences; BF16
rounding against hand-computed bit patterns; Adam against its published update
written for one scalar).
"""

import numpy as np


def bf16_round(x):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(a)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def conv3x3(x, W, b, d=1):
    """Periodic 3x3 convolution of x (C_in, H, W) with W (C_out, C_in, 3, 3) plus bias,
    taps d pixels apart (dilation d)."""
    C_out = W.shape[0]
    H, Wd = x.shape[1], x.shape[2]
    out = np.zeros((C_out, H, Wd))
    for a in range(3):
        for c in range(3):
            # xs[:, i, j] = x[:, i + d(a-1), j + d(c-1)]
            xs = np.roll(np.roll(x, -d * (a - 1), axis=1), -d * (c - 1), axis=2)
            out += np.tensordot(W[:, :, a, c], xs, axes=([1], [0]))
    return out + b[:, None, None]


def conv3x3_input_grad(dz, W, d=1):
    """d(sum dz * conv(x))/dx: the correlation with the flipped kernel."""
    C_in = W.shape[1]
    H, Wd = dz.shape[1], dz.shape[2]
    dx = np.zeros((C_in, H, Wd))
    for a in range(3):
        for c in range(3):
            t = np.tensordot(W[:, :, a, c], dz, axes=([0], [0]))  # (C_in, H, W) at output positions
            dx += np.roll(np.roll(t, d * (a - 1), axis=1), d * (c - 1), axis=2)
    return dx


def conv3x3_weight_grad(dz, x, d=1):
    """d(sum dz * conv(x))/dW and /db."""
    C_out, C_in = dz.shape[0], x.shape[0]
    dW = np.zeros((C_out, C_in, 3, 3))
    for a in range(3):
        for c in range(3):
            xs = np.roll(np.roll(x, -d * (a - 1), axis=1), -d * (c - 1), axis=2)
            dW[:, :, a, c] = np.tensordot(dz, xs, axes=([1, 2], [1, 2]))
    return dW, dz.sum(axis=(1, 2))


def init_params(channels=32, layers=8, c_in=2, c_out=1, seed=0):
    """He-normal weights scaled by 1/sqrt(9 C_in), zero biases; returns a list of (W, b)."""
    rng = np.random.default_rng(seed)
    chans = [c_in] + [channels] * (layers - 1) + [c_out]
    params = []
    for l in range(layers):
        ci, co = chans[l], chans[l + 1]
        W = rng.standard_normal((co, ci, 3, 3)) * np.sqrt(2.0 / (9 * ci))
        if l == layers - 1:
            W *= 0.1
        params.append((W, np.zeros(co)))
    return params


def unflatten_params(flat, layers, channels, c_in=2, c_out=1):
    """Flat array in the order W_0, b_0, W_1, b_1, ... (W_l[co][ci][3][3]) -> [(W, b)]."""
    chans = [c_in] + [channels] * (layers - 1) + [c_out]
    out, k = [], 0
    flat = np.asarray(flat, dtype=np.float64)
    for l in range(layers):
        ci, co = chans[l], chans[l + 1]
        W = flat[k:k + co * ci * 9].reshape(co, ci, 3, 3)
        k += co * ci * 9
        out.append((W, flat[k:k + co].copy()))
        k += co
    if k != flat.size:
        raise ValueError("parameter count %d does not match %d" % (flat.size, k))
    return out


def forward(x, params, bf16=False, dilations=None):
    """Returns (output c, cache of layer inputs and pre-activations)."""
    r = bf16_round if bf16 else (lambda v: v)
    h = r(x)
    cache = []
    L = len(params)
    dil = dilations or [1] * L
    for l, (W, b) in enumerate(params):
        z = conv3x3(h, r(W), b, dil[l])
        cache.append((h, z))
        if l < L - 1:
            h = r(np.maximum(z, 0.0))
        else:
            h = z
    return h, cache


def mse(c, t):
    return float(np.mean((c - t) ** 2))


def backward(c, t, cache, params, bf16=False, count=None, dilations=None):
    """Gradients of mse(c, t) with respect to every (W, b).

    With bf16=True the gradients flowing between layers are rounded to BF16, as the
    GPU kernels store them."""
    r = bf16_round if bf16 else (lambda v: v)
    dh = 2.0 * (c - t) / (c.size if count is None else count)
    grads = [None] * len(params)
    L = len(params)
    dil = dilations or [1] * L
    for l in range(L - 1, -1, -1):
        h, z = cache[l]
        dz = r(dh if l == L - 1 else dh * (z > 0))
        W = r(params[l][0])
        dW, db = conv3x3_weight_grad(dz, h, dil[l])
        grads[l] = (dW, db)
        if l > 0:
            dh = conv3x3_input_grad(dz, W, dil[l])
    return grads


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015) with bias correction; returns (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


# ---------------------------------------------------------------------------
# Around the network: target, head and resolution changes
# ---------------------------------------------------------------------------

def laplacian_fd4(u):
    """The fourth-order difference Laplacian of Section 4 (the training target)."""
    from . import fd
    h = 1.0 / u.shape[0]
    return fd.d2(u, 0, h) + fd.d2(u, 1, h)


def inverse_laplacian_fd4(c):
    """Mean-zero solution psi of laplacian_fd4(psi) = c - mean(c) (the warm-start head)."""
    from . import ma
    N = c.shape[0]
    return ma.lbar_inverse(c, ma.symbol((1.0, 0.0, 1.0, 0.0, 0.0), N, "fd4"))


def restrict_full_weighting(x):
    """2n x 2n -> n x n: weights (1/4, 1/2, 1/4) in each direction around fine node 2a."""
    w = {-1: 0.25, 0: 0.5, 1: 0.25}
    y = np.zeros_like(x)
    for p, wp in w.items():
        for q, wq in w.items():
            y += wp * wq * np.roll(np.roll(x, -p, axis=0), -q, axis=1)
    return y[::2, ::2]


def prolong_bilinear(x):
    """n x n -> 2n x 2n periodic bilinear interpolation between coarse nodes."""
    n = x.shape[0]
    y = np.zeros((2 * n, 2 * n))
    xr = np.roll(x, -1, axis=0)
    xc = np.roll(x, -1, axis=1)
    xrc = np.roll(xr, -1, axis=1)
    y[::2, ::2] = x
    y[1::2, ::2] = 0.5 * (x + xr)
    y[::2, 1::2] = 0.5 * (x + xc)
    y[1::2, 1::2] = 0.25 * (x + xr + xc + xrc)
    return y


def network_input(f, g):
    """(log f, log g) of the densities scaled to mean one."""
    return np.stack([np.log(f / f.mean()), np.log(g / g.mean())])


def log_ratio(f, g):
    """log f - log g for mean-one densities: the Laplacian of the linearised solution."""
    return np.log(f / f.mean()) - np.log(g / g.mean())


def training_target(psi, f=None, g=None):
    """laplacian_fd4(psi) - log_ratio(f, g) (the plain Laplacian without f, g)."""
    t = laplacian_fd4(psi)
    return t if f is None else t - log_ratio(f, g)


def warm_start(f, g, params, n_net, bf16=True, dilations=None):
    """psi0 for one pair: restrict if needed, run the network, prolong, add the log
    ratio at full resolution, invert the Laplacian."""
    n = f.shape[0]
    fr, gr = (restrict_full_weighting(f), restrict_full_weighting(g)) if n == 2 * n_net else (f, g)
    c, _ = forward(network_input(fr, gr), params, bf16=bf16, dilations=dilations)
    c = c[0]
    if n == 2 * n_net:
        c = prolong_bilinear(c)
    return inverse_laplacian_fd4(c + log_ratio(f, g))
