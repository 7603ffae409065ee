"""FP64 reference of the learned surrogate's network (test infrastructure only).

The surrogate is not part of the paper: it is a small 3-D convolutional network trained
on fields that the ray march produces, used in place of the march when a cheap error
check accepts its output (the march is the fallback). This module states, in plain
NumPy FP64, what the GPU kernels of that network compute, so that their forward pass and
their gradients can be checked against it.

Layout: channels last. Activations x[n][z][y][x][c]; weights W[tap][co][ci] with
tap = ((dz + 1) * 3 + (dy + 1)) * 3 + (dx + 1) for offsets dz, dy, dx in {-1, 0, 1};
bias b[co]. A "same" convolution with zero padding reads x at v + (dz, dy, dx):

    conv(x, W, b)[v][co] = b[co] + sum_tap sum_ci W[tap][co][ci] x[v + off(tap)][ci]

Activation: GELU with the error function, gelu(z) = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2.
Network (six layers, C channels): h1 = gelu(conv(x, W1, b1)); h_l = h_{l-1} +
gelu(conv(h_{l-1}, W_l, b_l)) for l = 2..L-1; y = conv(h_{L-1}, W_L, b_L). Inputs and the
output may use fewer channels than C (the rest are zero / ignored).

Gradients are written out by the chain rule (no automatic differentiation):
    dz = dh * gelu'(z),  gelu'(z) = Phi(z) + z phi(z)
    dx[v][ci] = sum_tap sum_co W[tap][co][ci] dz[v - off(tap)][co]   (+ dh for residuals)
    dW[tap][co][ci] = sum_v dz[v][co] x[v + off(tap)][ci],  db[co] = sum_v dz[v][co]
"""

import math

import numpy as np
from scipy.special import erf

OFFSETS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
SQRT2 = math.sqrt(2.0)


def _shifted(xp, off, shape):
    """View of the zero-padded xp (pad 1 on each spatial side) at v + off for v in shape."""
    dz, dy, dx = off
    D, H, W = shape
    return xp[:, 1 + dz:1 + dz + D, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W, :]


def conv3(x, W, b=None):
    """'Same' 3x3x3 convolution, zero padding. x (N,D,H,W,Ci), W (27,Co,Ci), b (Co,)."""
    x = np.asarray(x, np.float64)
    W = np.asarray(W, np.float64)
    n, D, H, Wd, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1), (0, 0)))
    out = np.zeros((n, D, H, Wd, W.shape[1]))
    for tap, off in enumerate(OFFSETS):
        out += _shifted(xp, off, (D, H, Wd)) @ W[tap].T
    if b is not None:
        out += np.asarray(b, np.float64)
    return out


def conv3_grad_input(dz, W):
    """dL/dx of conv3 for upstream dz (N,D,H,W,Co): each output voxel v sent
    W[tap]^T dz[v] to input voxel v + off(tap)."""
    dz = np.asarray(dz, np.float64)
    W = np.asarray(W, np.float64)
    n, D, H, Wd, _ = dz.shape
    dxp = np.zeros((n, D + 2, H + 2, Wd + 2, W.shape[2]))
    for tap, (oz, oy, ox) in enumerate(OFFSETS):
        dxp[:, 1 + oz:1 + oz + D, 1 + oy:1 + oy + H, 1 + ox:1 + ox + Wd, :] += dz @ W[tap]
    return dxp[:, 1:-1, 1:-1, 1:-1, :]


def conv3_grad_weight(x, dz):
    """dL/dW (27,Co,Ci) and dL/db (Co,) of conv3."""
    x = np.asarray(x, np.float64)
    dz = np.asarray(dz, np.float64)
    n, D, H, Wd, ci = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1), (0, 0)))
    dzf = dz.reshape(-1, dz.shape[-1])
    dW = np.zeros((27, dz.shape[-1], ci))
    for tap, off in enumerate(OFFSETS):
        dW[tap] = dzf.T @ _shifted(xp, off, (D, H, Wd)).reshape(-1, ci)
    return dW, dzf.sum(axis=0)


def gelu(z):
    z = np.asarray(z, np.float64)
    return 0.5 * z * (1.0 + erf(z / SQRT2))


def gelu_grad(z):
    z = np.asarray(z, np.float64)
    return 0.5 * (1.0 + erf(z / SQRT2)) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(params, x):
    """params: list of (W, b) per layer. Returns (y, cache) with y (N,D,H,W,Co_last)."""
    h = np.asarray(x, np.float64)
    cache = []
    L = len(params)
    for l, (W, b) in enumerate(params):
        z = conv3(h, W, b)
        cache.append((h, z))
        if l == L - 1:
            h = z
        elif l == 0:
            h = gelu(z)
        else:
            h = h + gelu(z)
    return h, cache


def backward(params, cache, dy):
    """Gradients [(dW, db)] of sum(dy * y) through forward()."""
    L = len(params)
    grads = [None] * L
    dh = np.asarray(dy, np.float64)
    for l in range(L - 1, -1, -1):
        W, _ = params[l]
        h_in, z = cache[l]
        dz = dh if l == L - 1 else dh * gelu_grad(z)
        grads[l] = conv3_grad_weight(h_in, dz)
        dx = conv3_grad_input(dz, W)
        dh = dx + dh if 0 < l < L - 1 else dx
    return grads


def features(j, kappa, cheap, stats):
    """Network input of one sample, FP64, as (cells, 4) plus the sample scale s.

    c = max(cheap, 0) is the few-ray march; s = sqrt(mean c^2) its root-mean-square. The
    four input channels are the standardised log opacity, the scaled emissivity, the cheap
    field in units of s and the standardised log of the cheap field:
        ((log max(kappa, 1e-30) - m_k) i_k,  j i_j,  c / s,  (log(c + f) - m_c) i_c)
    with stats = (m_k, i_k, i_j, m_c, i_c, f) fixed from training data.
    """
    st = [float(v) for v in np.asarray(stats, np.float32)]
    c = np.maximum(np.asarray(cheap, np.float64).ravel(), 0.0)
    s = max(math.sqrt(np.sum(c * c) / c.size), 1e-30)
    k = np.asarray(kappa, np.float64).ravel()
    jj = np.asarray(j, np.float64).ravel()
    x = np.stack([(np.log(np.maximum(k, 1e-30)) - st[0]) * st[1], jj * st[2], c / s,
                  (np.log(c + st[5]) - st[3]) * st[4]], axis=1)
    return x, s


def output(y0, cheap):
    """Prediction from the network's channel 0 and the error-check sums, FP64.

    The network predicts a correction to the cheap field in units of its scale s:
    J = max(0, c + s y0), with c = max(cheap, 0). The check sums are sum (J - c)^2 and
    sum c^2; their square-root ratio is the prediction's relative L2 distance from c.
    Returns (J, (sum (J - c)^2, sum c^2)).
    """
    c = np.maximum(np.asarray(cheap, np.float64).ravel(), 0.0)
    s = max(math.sqrt(np.sum(c * c) / c.size), 1e-30)
    J = np.maximum(0.0, c + s * np.asarray(y0, np.float64).ravel())
    return J, (float(np.sum((J - c) ** 2)), float(np.sum(c * c)))
