"""The learned surrogate on the GPU: network gradients against the FP64 oracle, training
with the library's kernels, and the fallback that keeps every returned field close to the
full march.
"""

import sys

import numpy as np
import pytest
import torch

from oracle import surrogate as S
from paper_2511_09389_amd import surrogate as sg

pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[gpu-surrogate] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch.device("cuda:0")


def f64(t):
    return t.float().cpu().numpy().astype(np.float64)


def test_network_gradients_match_oracle(rt, dev):
    """Forward and backward of the whole six-layer network against the oracle run on the
    same bf16 weights and input. The GPU keeps activations in bf16 between layers, so the
    agreement is to bf16 precision, not fp32."""
    net = sg.SurrogateNet(dev, seed=3, residual_scale=0.5)
    for l in range(sg.LAYERS):   # make every layer matter
        net.b[l].copy_(torch.linspace(-0.2, 0.2, sg.C, device=dev))
    net.w[-1][:, 0, :] = torch.randn(27, sg.C, generator=torch.Generator().manual_seed(9)).to(dev) * 0.05
    net.wb = [w.to(torch.bfloat16).contiguous() for w in net.w]
    rng = np.random.default_rng(21)
    x = np.zeros((1, 6, 5, 16, sg.C), np.float32)
    x[..., :sg.N_FEATURES] = rng.normal(size=(1, 6, 5, 16, sg.N_FEATURES))
    xb = torch.from_numpy(x).to(dev).to(torch.bfloat16).contiguous()
    y, cache = net.forward(xb, keep=True)
    dy = torch.zeros_like(y)
    dy[..., 0] = torch.from_numpy(rng.normal(size=(1, 6, 5, 16)).astype(np.float32)).to(dev).to(torch.bfloat16)
    dw, db = net.backward(cache, dy.contiguous())
    params = [(f64(net.wb[l]), f64(net.b[l])) for l in range(sg.LAYERS)]
    want_y, ocache = S.forward(params, f64(xb))
    grads = S.backward(params, ocache, f64(dy))
    ey = np.linalg.norm(f64(y)[..., 0] - want_y[..., 0]) / np.linalg.norm(want_y[..., 0])
    gw = np.concatenate([f64(dw[l]).ravel() for l in range(sg.LAYERS)] + [f64(db[l]).ravel() for l in range(sg.LAYERS)])
    ow = np.concatenate([grads[l][0].ravel() for l in range(sg.LAYERS)] + [grads[l][1].ravel() for l in range(sg.LAYERS)])
    eg = np.linalg.norm(gw - ow) / np.linalg.norm(ow)
    cos = gw @ ow / (np.linalg.norm(gw) * np.linalg.norm(ow))
    note(f"network output rel L2 {ey:.2e}; gradient rel L2 {eg:.2e}, cosine {cos:.6f}")
    assert ey < 2e-2
    assert eg < 3e-2 and cos > 0.999


def test_feature_and_output_kernels_match_oracle(rt, dev):
    """rtmi_surrogate_features and rtmi_surrogate_output against the FP64 statement of the
    transforms (oracle.surrogate.features / output) on a turbulent sample: the bf16 input
    channels to bf16 rounding, the channels past the features exactly zero, the fp32
    prediction and the error-check sums to binary32 rounding (float atomics for the sums)."""
    w, j, k, cheap, full = sg.make_sample(77, dev, n=24, n_src=4, num_rays=512, c=24.0)
    stats = sg.input_stats([(w, j, k, cheap, full)])
    x, sums = rt.surrogate_features(j, k, cheap, stats)
    want_x, s = S.features(f64(j), f64(k), f64(cheap), stats)
    got_x = f64(x).reshape(-1, sg.C)
    assert not got_x[:, sg.N_FEATURES:].any()
    # bf16 keeps 8 significant bits; the 1e-5 absolute term covers binary32 cancellation in
    # the standardised channels (values of order 1 that happen to be near zero)
    err = np.abs(got_x[:, :sg.N_FEATURES] - want_x)
    assert np.all(err <= 2.0 ** -8 * np.abs(want_x) + 1e-5), float(err.max())
    assert abs(float(torch.sqrt(sums[0] / cheap.numel())) - s) <= 1e-5 * s
    rng = np.random.default_rng(5)
    y = torch.zeros((1,) + tuple(cheap.shape) + (sg.C,), dtype=torch.bfloat16, device=dev)
    y[..., 0] = torch.from_numpy(rng.normal(0.0, 0.3, size=cheap.shape).astype(np.float32)).to(dev)
    field, check = rt.surrogate_output(y.contiguous(), cheap, sums)
    want_J, (a, b) = S.output(f64(y)[..., 0], f64(cheap))
    got_J = f64(field).ravel()
    assert np.all(np.abs(got_J - want_J) <= 1e-6 * (np.abs(want_J) + s))
    c = f64(check)
    assert abs(c[0] - a) <= 1e-5 * a and abs(c[1] - b) <= 1e-5 * b


def test_train_and_fallback(rt, dev):
    """A small run of the whole recipe: generate samples with the march, train, calibrate
    the check on validation samples, and evaluate on held-out ones. The loss must fall; the
    network must bring the cheap march closer to the full one (what the learned part gains
    at the cheap march's cost); and every returned field must be within 1 % of the full
    march, the target the check was calibrated for. A returned field is either a surrogate
    prediction the check accepted or the full march itself: when no prediction passes the
    check (accepted = 0 in the printed summary), this test exercises the fallback only and
    says nothing about predictions within 1 %."""
    kw = dict(n=32, n_src=6, num_rays=1024, c=32.0)
    train = [sg.make_sample(s, dev, **kw) for s in range(24)]
    val = [sg.make_sample(1000 + s, dev, **kw) for s in range(8)]
    held = [sg.make_sample(2000 + s, dev, **kw) for s in range(8)]
    model, losses = sg.train(train, dev, epochs=6, lr=2e-3, log=note)
    assert losses[-1] < 0.7 * losses[0]
    thr, pairs = sg.calibrate(model, val, target=0.01)
    cheap_err = [sg.rel_l2(s[3], s[4]) for s in held]
    res = sg.evaluate(model, held, reps=2)
    note(f"threshold {thr:.4f}; validation (check, error): {[(round(a, 4), round(b, 4)) for a, b in pairs]}")
    note(f"held-out: {res}; cheap march alone: mean error {np.mean(cheap_err):.4f}")
    assert np.median([p[1] for p in pairs]) < np.mean([sg.rel_l2(s[3], s[4]) for s in val])
    note(f"accepted {res['accepted']} of {res['samples']} held-out predictions; "
         f"surrogate path {res['surrogate_fields_per_s']:.0f} fields/s, plain march "
         f"{res['march_fields_per_s']:.0f} fields/s")
    assert res["max_err"] <= 0.01
