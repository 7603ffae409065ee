"""The surrogate network's bf16 matrix-core kernels against the FP64 oracle.

Operands are rounded to bf16 before the oracle sees them, so the oracle and the GPU
multiply the same numbers; what remains is fp32 accumulation (bounded here by 1e-5 of the
sum of |terms|) and, for bf16 outputs, one bf16 rounding (2^-8 relative).
"""

import sys

import numpy as np
import pytest
import torch

from oracle import surrogate as S

pytestmark = pytest.mark.gpu
C = 32


def note(msg):
    print(f"[gpu-conv] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch.device("cuda:0")


def bf16(a, dev):
    return torch.from_numpy(np.asarray(a, np.float32)).to(dev).to(torch.bfloat16).contiguous()


def f64(t):
    return t.float().cpu().numpy().astype(np.float64)


def case(rng, dev, shape, scale_w=0.1):
    x = bf16(rng.normal(size=shape + (C,)), dev)
    w = bf16(scale_w * rng.normal(size=(27, C, C)), dev)
    b = torch.from_numpy(rng.normal(size=C).astype(np.float32)).to(dev)
    return x, w, b


SHAPES = [(1, 4, 5, 32), (2, 3, 3, 16), (1, 6, 7, 13), (1, 1, 1, 1)]


@pytest.mark.parametrize("shape", SHAPES)
def test_forward_matches_oracle(rt, dev, shape):
    rng = np.random.default_rng(11)
    x, w, b = case(rng, dev, shape)
    z = torch.empty(shape + (C,), dtype=torch.float32, device=dev)
    y = rt.conv3d_forward(x, w, bias=b, gelu=False, z=z)
    want = S.conv3(f64(x), f64(w), f64(b))
    bound = S.conv3(np.abs(f64(x)), np.abs(f64(w)), np.abs(f64(b)))
    err = np.abs(f64(z) - want)
    assert (err <= 1e-5 * bound + 1e-30).all(), err.max()
    # the bf16 output is z rounded once
    assert np.allclose(f64(y), want, rtol=2 ** -8, atol=1e-6 * bound.max())
    note(f"forward {shape}: max |z - oracle| / bound = {(err / (bound + 1e-30)).max():.2e}")


def test_forward_gelu_residual(rt, dev):
    rng = np.random.default_rng(12)
    shape = (1, 5, 4, 32)
    x, w, b = case(rng, dev, shape, scale_w=0.2)
    res = bf16(rng.normal(size=shape + (C,)), dev)
    y = rt.conv3d_forward(x, w, bias=b, residual=res, gelu=True)
    want = f64(res) + S.gelu(S.conv3(f64(x), f64(w), f64(b)))
    assert np.allclose(f64(y), want, rtol=2 ** -7, atol=1e-3)


@pytest.mark.parametrize("shape", SHAPES)
def test_backward_data_matches_oracle(rt, dev, shape):
    rng = np.random.default_rng(13)
    dz, w, _ = case(rng, dev, shape)
    res = torch.from_numpy(rng.normal(size=shape + (C,)).astype(np.float32)).to(dev)
    zprev = torch.from_numpy(rng.normal(size=shape + (C,)).astype(np.float32)).to(dev)
    dh = torch.empty(shape + (C,), dtype=torch.float32, device=dev)
    dzp = torch.empty(shape + (C,), dtype=torch.bfloat16, device=dev)
    rt.conv3d_backward_data(dz, w, residual=res, zprev=zprev, dh=dh, dz_prev=dzp)
    g = S.conv3_grad_input(f64(dz), f64(w)) + f64(res)
    bound = S.conv3_grad_input(np.abs(f64(dz)), np.abs(f64(w))) + np.abs(f64(res))
    err = np.abs(f64(dh) - g)
    assert (err <= 1e-5 * bound + 1e-30).all(), err.max()
    want = g * S.gelu_grad(f64(zprev))
    assert np.allclose(f64(dzp), want, rtol=2 ** -7, atol=1e-5 * bound.max())


@pytest.mark.parametrize("shape", [(1, 4, 5, 32), (2, 3, 3, 16), (1, 2, 2, 64), (1, 2, 3, 80), (2, 8, 20, 16)])
def test_backward_weight_matches_oracle(rt, dev, shape):
    rng = np.random.default_rng(14)
    x, _, _ = case(rng, dev, shape)
    dz = bf16(rng.normal(size=shape + (C,)), dev)
    dw = torch.zeros((27, C, C), dtype=torch.float32, device=dev)
    db = torch.zeros(C, dtype=torch.float32, device=dev)
    rt.conv3d_backward_weight(x, dz, dw, db)
    want_w, want_b = S.conv3_grad_weight(f64(x), f64(dz))
    bound_w, _ = S.conv3_grad_weight(np.abs(f64(x)), np.abs(f64(dz)))
    err = np.abs(dw.cpu().numpy() - want_w)
    assert (err <= 1e-5 * bound_w + 1e-30).all(), err.max()
    np.testing.assert_allclose(db.cpu().numpy(), want_b, rtol=1e-5, atol=1e-4)


def test_backward_weight_accumulates_in_a_fixed_order(rt, dev):
    """dw and db are added to, and the per-work-group partial sums are summed in a fixed
    order: a second call on the same inputs adds exactly the same bits again."""
    rng = np.random.default_rng(15)
    shape = (1, 24, 20, 48)
    x, _, _ = case(rng, dev, shape)
    dz = bf16(rng.normal(size=shape + (C,)), dev)
    dw = torch.zeros((27, C, C), dtype=torch.float32, device=dev)
    db = torch.zeros(C, dtype=torch.float32, device=dev)
    rt.conv3d_backward_weight(x, dz, dw, db)
    once_w, once_b = dw.clone(), db.clone()
    rt.conv3d_backward_weight(x, dz, dw, db)
    assert torch.equal(dw, 2.0 * once_w) and torch.equal(db, 2.0 * once_b)
    want_w, _ = S.conv3_grad_weight(f64(x), f64(dz))
    bound_w, _ = S.conv3_grad_weight(np.abs(f64(x)), np.abs(f64(dz)))
    assert (np.abs(once_w.cpu().numpy() - want_w) <= 1e-5 * bound_w + 1e-30).all()


def test_backward_weight_rejects_odd_rows(rt, dev):
    x = torch.zeros((1, 2, 2, 13, C), dtype=torch.bfloat16, device=dev)
    dw = torch.zeros((27, C, C), device=dev)
    db = torch.zeros(C, device=dev)
    with pytest.raises(rt.RtmiError):
        rt.conv3d_backward_weight(x, x, dw, db)


def test_mse_and_adam(rt, dev):
    rng = np.random.default_rng(15)
    y = bf16(rng.normal(size=(2, 3, 3, 16, C)), dev)
    t = torch.from_numpy(rng.normal(size=(2, 3, 3, 16)).astype(np.float32)).to(dev)
    dz = torch.empty_like(y)
    loss = torch.zeros(1, device=dev)
    rt.mse_loss(y, t, 0.5, dz, loss)
    d = f64(y)[..., 0] - t.double().cpu().numpy()
    assert abs(loss.item() - 0.5 * (d * d).sum()) <= 1e-5 * (d * d).sum()
    assert np.allclose(f64(dz)[..., 0], d, rtol=2 ** -8, atol=1e-6)
    assert (f64(dz)[..., 1:] == 0).all()
    # Adam, two steps, against the textbook update in FP64
    w0 = rng.normal(size=100).astype(np.float32)
    g = [rng.normal(size=100).astype(np.float32) for _ in range(2)]
    w = torch.from_numpy(w0.copy()).to(dev)
    m = torch.zeros(100, device=dev)
    v = torch.zeros(100, device=dev)
    wb = torch.empty(100, dtype=torch.bfloat16, device=dev)
    mw, mm, mv = w0.astype(np.float64), np.zeros(100), np.zeros(100)
    for step in (1, 2):
        rt.adam_step(w, m, v, torch.from_numpy(g[step - 1]).to(dev), wb, 1e-2, step)
        mm = 0.9 * mm + 0.1 * g[step - 1]
        mv = 0.999 * mv + 0.001 * g[step - 1].astype(np.float64) ** 2
        mw = mw - 1e-2 * (mm / (1 - 0.9 ** step)) / (np.sqrt(mv / (1 - 0.999 ** step)) + 1e-8)
    np.testing.assert_allclose(w.cpu().numpy(), mw, rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(wb.float().cpu().numpy(), mw, rtol=2 ** -8, atol=1e-6)
