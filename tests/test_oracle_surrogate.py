"""Pins of the FP64 surrogate-network oracle (CPU).

conv3 against torch's conv3d in float64 (an independent implementation), an impulse
response written out by hand, GELU against its closed-form values, and every gradient
against central finite differences (and torch's autograd for the convolution).
"""

import math

import numpy as np
import pytest
import torch

from oracle import surrogate as S


def to_torch_ncdhw(x):
    return torch.from_numpy(np.ascontiguousarray(np.moveaxis(x, -1, 1)))


def torch_weight(W):
    # W[tap][co][ci], tap = ((dz+1)*3 + (dy+1))*3 + (dx+1) -> (co, ci, kz, ky, kx)
    co, ci = W.shape[1], W.shape[2]
    return torch.from_numpy(np.ascontiguousarray(W.reshape(3, 3, 3, co, ci).transpose(3, 4, 0, 1, 2)))


@pytest.mark.parametrize("shape,ci,co", [((1, 5, 4, 6), 3, 2), ((2, 4, 4, 4), 8, 8)])
def test_conv3_matches_torch_conv3d(shape, ci, co):
    rng = np.random.default_rng(1)
    x = rng.normal(size=shape + (ci,))
    W = rng.normal(size=(27, co, ci))
    b = rng.normal(size=co)
    got = S.conv3(x, W, b)
    want = torch.nn.functional.conv3d(to_torch_ncdhw(x), torch_weight(W), torch.from_numpy(b), padding=1)
    np.testing.assert_allclose(got, np.moveaxis(want.numpy(), 1, -1), rtol=1e-12, atol=1e-12)


def test_conv3_impulse_response():
    """A unit impulse at voxel u, channel i, gives out[u - off(tap)][co] = W[tap][co][i]."""
    rng = np.random.default_rng(2)
    W = rng.normal(size=(27, 2, 3))
    x = np.zeros((1, 5, 5, 5, 3))
    x[0, 2, 2, 2, 1] = 1.0
    out = S.conv3(x, W)
    for tap, (dz, dy, dx) in enumerate(S.OFFSETS):
        np.testing.assert_array_equal(out[0, 2 - dz, 2 - dy, 2 - dx], W[tap, :, 1])
    # zero padding: an impulse in a corner reaches only the in-box outputs
    x = np.zeros((1, 3, 3, 3, 1))
    x[0, 0, 0, 0, 0] = 1.0
    W1 = np.ones((27, 1, 1))
    assert S.conv3(x, W1).sum() == 8.0


def test_gelu_closed_forms():
    assert S.gelu(0.0) == 0.0
    assert abs(S.gelu(1.0) - 0.8413447460685429) < 1e-15          # Phi(1)
    assert abs(S.gelu(-1.0) + 0.15865525393145707) < 1e-15        # -(1 - Phi(1))
    assert abs(S.gelu(10.0) - 10.0) < 1e-12
    z = np.linspace(-4, 4, 81)
    h = 1e-6
    fd = (S.gelu(z + h) - S.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(S.gelu_grad(z), fd, rtol=1e-7, atol=1e-9)
    assert abs(S.gelu_grad(0.0) - 0.5) < 1e-15


def test_conv3_gradients_match_torch_autograd():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(2, 4, 5, 3, 4))
    W = rng.normal(size=(27, 3, 4))
    b = rng.normal(size=3)
    dz = rng.normal(size=(2, 4, 5, 3, 3))
    xt = to_torch_ncdhw(x).requires_grad_(True)
    Wt = torch_weight(W).requires_grad_(True)
    bt = torch.from_numpy(b).requires_grad_(True)
    out = torch.nn.functional.conv3d(xt, Wt, bt, padding=1)
    out.backward(to_torch_ncdhw(dz))
    np.testing.assert_allclose(S.conv3_grad_input(dz, W), np.moveaxis(xt.grad.numpy(), 1, -1), rtol=1e-11, atol=1e-11)
    dW, db = S.conv3_grad_weight(x, dz)
    want_W = Wt.grad.numpy().transpose(2, 3, 4, 0, 1).reshape(27, 3, 4)
    np.testing.assert_allclose(dW, want_W, rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(db, bt.grad.numpy(), rtol=1e-12, atol=1e-12)


def small_net(rng, c=4, cin=2, cout=1, layers=6, scale=0.3):
    params = []
    for l in range(layers):
        ci = cin if l == 0 else c
        co = cout if l == layers - 1 else c
        params.append((scale * rng.normal(size=(27, co, ci)), 0.1 * rng.normal(size=co)))
    return params


def test_network_backward_matches_finite_differences():
    rng = np.random.default_rng(4)
    params = small_net(rng)
    x = rng.normal(size=(1, 4, 3, 4, 2))
    dy = rng.normal(size=(1, 4, 3, 4, 1))
    y, cache = S.forward(params, x)
    grads = S.backward(params, cache, dy)
    h = 1e-6
    for l in (0, 2, 5):
        for idx in [(0, 0, 0), (13, 0, 1), (26, -1, -1)]:
            W, b = params[l]
            Wp = W.copy(); Wp[idx] += h
            Wm = W.copy(); Wm[idx] -= h
            pp = list(params); pp[l] = (Wp, b)
            pm = list(params); pm[l] = (Wm, b)
            fd = ((S.forward(pp, x)[0] - S.forward(pm, x)[0]) * dy).sum() / (2 * h)
            assert abs(grads[l][0][idx] - fd) <= 1e-6 * max(1.0, abs(fd)), (l, idx)
        bp = b.copy(); bp[0] += h
        bm = b.copy(); bm[0] -= h
        pp = list(params); pp[l] = (W, bp)
        pm = list(params); pm[l] = (W, bm)
        fd = ((S.forward(pp, x)[0] - S.forward(pm, x)[0]) * dy).sum() / (2 * h)
        assert abs(grads[l][1][0] - fd) <= 1e-6 * max(1.0, abs(fd)), l


def test_zero_residual_blocks_are_identity():
    rng = np.random.default_rng(5)
    params = small_net(rng)
    for l in range(1, 5):
        params[l] = (np.zeros_like(params[l][0]), np.zeros_like(params[l][1]))
    x = rng.normal(size=(1, 3, 3, 3, 2))
    _, cache = S.forward(params, x)
    h1 = S.gelu(cache[0][1])
    np.testing.assert_array_equal(cache[5][0], h1)


def test_feature_transform_invariants():
    """With the statistics taken from the sample itself, the standardised channels have
    mean 0 and standard deviation 1, the scaled j peaks at 1, and the linear cheap channel
    has root-mean-square 1 (it is the field over its own root-mean-square)."""
    rng = np.random.default_rng(8)
    shape = (6, 7, 8)
    kap = np.exp(rng.normal(-3.0, 1.0, size=shape))
    j = rng.random(shape) * 3.0
    cheap = rng.random(shape) ** 3
    floor = 1e-4
    lk, lc = np.log(kap), np.log(cheap + floor)
    stats = [lk.mean(), 1.0 / lk.std(), 1.0 / j.max(), lc.mean(), 1.0 / lc.std(), floor]
    x, s = S.features(j, kap, cheap, np.asarray(stats, np.float64))
    assert abs(s - np.sqrt(np.mean(cheap ** 2))) <= 1e-12 * s
    assert abs(np.sqrt(np.mean(x[:, 2] ** 2)) - 1.0) < 1e-12
    for ch in (0, 3):   # float32 statistics: standardised to about 1e-6
        assert abs(x[:, ch].mean()) < 1e-5 and abs(x[:, ch].std() - 1.0) < 1e-5
    assert abs(x[:, 1].max() - 1.0) < 1e-6


def test_output_transform_special_cases():
    """y = 0 returns the cheap field (distance 0); y = 1 adds exactly s to every voxel
    (distance 1, since s is the root-mean-square); a very negative y clips to zero
    (distance 1); negative cheap values count as zero."""
    rng = np.random.default_rng(9)
    cheap = rng.random(500) - 0.1
    c = np.maximum(cheap, 0.0)
    J, (a, b) = S.output(np.zeros(500), cheap)
    assert np.array_equal(J, c) and a == 0.0 and abs(b - np.sum(c * c)) <= 1e-12 * b
    J, (a, b) = S.output(np.ones(500), cheap)
    s = np.sqrt(np.mean(c * c))
    assert np.allclose(J, c + s, rtol=1e-15, atol=0) and abs(np.sqrt(a / b) - 1.0) < 1e-12
    J, (a, b) = S.output(np.full(500, -1e9), cheap)
    assert not J.any() and abs(np.sqrt(a / b) - 1.0) < 1e-12
