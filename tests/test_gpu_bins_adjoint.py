"""GPU adjoint of the frequency-bin march (rtmi_trace_bins_vjp, through the C ABI) against
the FP64 oracle VJP, its autograd binding, and the amplitude + opacity-scale fit that runs
on it (Sec. 4, gradient-based inversion, over the bins of Sec. 2).

Tolerances as for the one-bin adjoint: relative L2 <= 1e-5 for dL/dj and dL/dkappa and a
per-voxel bound of 1e-4 relative to the oracle gradient for |G| (which bounds what was
summed in a voxel); the bin scales' gradients to 1e-5 relative.
"""

import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2511_09389_amd import autograd, inputs, inverse

pytestmark = pytest.mark.gpu

SCALES = np.array([1.0, 1.5 ** -3, 2.0 ** -3, 3.0 ** -3], np.float32)   # the uneven workload's bins


def note(msg):
    print(f"[gpu-bins-adjoint] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch.device("cuda:0")


def to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)


def rel_l2(got, want):
    return float(np.linalg.norm(np.asarray(got, np.float64) - want) / np.linalg.norm(want))


def per_voxel(got, want, scale, tol=1e-4, floor=1e-6):
    got = np.asarray(got, np.float64)
    scale = np.abs(scale)
    mask = scale > floor * scale.max()
    rel = np.abs(got[mask] - want[mask]) / scale[mask]
    assert rel.max() <= tol, f"max per-voxel error {rel.max():.3e} > {tol}"
    return float(rel.max())


def case(seed, shape=(17, 13, 19), n_bins=4):
    rng = np.random.default_rng(seed)
    kap = (0.3 * rng.random(shape)).astype(np.float32)
    j = rng.random(shape).astype(np.float32)
    G = rng.normal(size=(n_bins,) + shape).astype(np.float32)
    src = np.array([[8.2, 6.1, 9.4], [-2.0, 11.5, 3.0], [15.5, 0.5, 17.0]], np.float32)
    return j, kap, G, src, [96, 160, 64], [0, 19, 0]


def check(gj, gk, wj, wk, sj, sk, what):
    ej, ek = rel_l2(gj, wj), rel_l2(gk, wk)
    pj, pk = per_voxel(gj, wj, sj), per_voxel(gk, wk, sk)
    note(f"  {what}: rel L2 dL/dj {ej:.2e}, dL/dkappa {ek:.2e}; per voxel {pj:.2e}, {pk:.2e}")
    assert ej <= 1e-5 and ek <= 1e-5


def test_shared_maps_with_scales(rt, dev):
    """One j and one kappa for four bins with kappa_b = s_b kappa: dL/dj sums the bins,
    dL/dkappa sums s_b dL/dkappa_b, and dL/ds_b = sum_v kappa dL/dkappa_b."""
    j, kap, G, src, rays, caps = case(31)
    gj, gk, gs = rt.trace_bins_vjp(to_dev(j, dev), to_dev(kap, dev), src, rays, 0.5, 16.0, 1.0, to_dev(G, dev),
                                   kappa_scale=SCALES, substep_cap=caps, scale_grad=True)
    wj, wk, ws = oracle.trace_bins_vjp(j, kap, SCALES, src, rays, 0.5, 16.0, 1.0, G, caps=caps)
    sj, sk, _ = oracle.trace_bins_vjp(j, kap, SCALES, src, rays, 0.5, 16.0, 1.0, np.abs(G), caps=caps)
    check(gj.cpu().numpy(), gk.cpu().numpy(), wj, wk, sj, sk, "shared j and kappa")
    got_s = gs.cpu().numpy().astype(np.float64)
    rel_s = np.abs(got_s - ws) / np.abs(ws)
    note(f"  dL/ds_b {got_s} vs {ws}: max rel {rel_s.max():.2e}")
    assert rel_s.max() <= 1e-5


def test_per_bin_j_and_per_bin_kappa(rt, dev):
    """A stack of j maps with a shared scaled kappa, then a shared j with per-bin kappa
    maps: per-bin gradients come back per bin."""
    j, kap, G, src, rays, caps = case(32, n_bins=3)
    jb = np.stack([j, 0.5 * j, 2.0 * j]).astype(np.float32)
    sc = SCALES[:3]
    gj, gk, gs = rt.trace_bins_vjp(to_dev(jb, dev), to_dev(kap, dev), src, rays, 0.5, 16.0, 1.0, to_dev(G, dev),
                                   kappa_scale=sc, substep_cap=caps)
    assert gs is None and tuple(gj.shape) == jb.shape and tuple(gk.shape) == kap.shape
    wj, wk, _ = oracle.trace_bins_vjp(jb, kap, sc, src, rays, 0.5, 16.0, 1.0, G, caps=caps)
    sj, sk, _ = oracle.trace_bins_vjp(jb, kap, sc, src, rays, 0.5, 16.0, 1.0, np.abs(G), caps=caps)
    check(gj.cpu().numpy(), gk.cpu().numpy(), wj, wk, sj, sk, "per-bin j, shared scaled kappa")
    kb = np.stack([kap, 0.4 * kap, 1.7 * kap]).astype(np.float32)
    gj, gk, _ = rt.trace_bins_vjp(to_dev(j, dev), to_dev(kb, dev), src, rays, 0.5, 16.0, 1.0, to_dev(G, dev),
                                  substep_cap=caps)
    assert tuple(gk.shape) == kb.shape and tuple(gj.shape) == j.shape
    wj, wk, ws = oracle.trace_bins_vjp(j, None, None, src, rays, 0.5, 16.0, 1.0, G, caps=caps, kappa_maps=kb)
    sj, sk, _ = oracle.trace_bins_vjp(j, None, None, src, rays, 0.5, 16.0, 1.0, np.abs(G), caps=caps,
                                      kappa_maps=kb)
    assert ws is None
    check(gj.cpu().numpy(), gk.cpu().numpy(), wj, wk, sj, sk, "shared j, per-bin kappa maps")
    # a scale gradient needs a shared kappa: refused through the C ABI before any work
    jd, kd, Gd = to_dev(j, dev), to_dev(kb, dev), to_dev(G, dev)
    oj, ok, osc = torch.empty_like(jd), torch.empty_like(kd), torch.empty(3, device=dev)
    nr = np.asarray(rays, np.int32)
    code = rt.lib.rtmi_trace_bins_vjp(jd.data_ptr(), 0, kd.data_ptr(), j.size, None, 3, *j.shape, 3,
                                      src.ctypes.data, nr.ctypes.data, None, 0.5, 16.0, 1.0, Gd.data_ptr(),
                                      oj.data_ptr(), ok.data_ptr(), osc.data_ptr(), None)
    assert code == rt.ERR_INVALID_ARG and "shared" in rt.lib.rtmi_last_error().decode()


def test_one_bin_equals_trace_vjp(rt, dev):
    j, kap, G, src, rays, caps = case(33, n_bins=1)
    a = rt.trace_bins_vjp(to_dev(j, dev), to_dev(kap, dev), src, rays, 0.5, 16.0, 1.0, to_dev(G, dev),
                          kappa_scale=[1.0], substep_cap=caps)
    b = rt.trace_vjp(to_dev(j, dev), to_dev(kap, dev), src, rays, 0.5, 16.0, 1.0, to_dev(G[0], dev),
                     substep_cap=caps)
    assert rel_l2(a[0].cpu().numpy(), b[0].cpu().numpy().astype(np.float64)) <= 1e-6
    assert rel_l2(a[1].cpu().numpy(), b[1].cpu().numpy().astype(np.float64)) <= 1e-6


def test_march_bins_autograd(rt, dev):
    """loss = sum_b <G_b, J_b>: autograd through MarchBins returns the library adjoint for
    j, kappa and the bin scales."""
    j, kap, G, src, rays, caps = case(34)
    jt = to_dev(j, dev).requires_grad_(True)
    kt = to_dev(kap, dev).requires_grad_(True)
    st = to_dev(SCALES, dev).requires_grad_(True)
    Gt = to_dev(G, dev)
    J = autograd.march_bins(jt, kt, st, src, rays, 0.5, 16.0, 1.0, substep_cap=caps)
    (J * Gt).sum().backward()
    wj, wk, ws = oracle.trace_bins_vjp(j, kap, SCALES, src, rays, 0.5, 16.0, 1.0, G, caps=caps)
    assert rel_l2(jt.grad.cpu().numpy(), wj) <= 1e-5
    assert rel_l2(kt.grad.cpu().numpy(), wk) <= 1e-5
    assert np.max(np.abs(st.grad.cpu().numpy() - ws) / np.abs(ws)) <= 1e-5


def test_dot_and_scaled_copy(rt, dev):
    rng = np.random.default_rng(35)
    a = rng.normal(size=100003).astype(np.float32)
    b = rng.normal(size=100003).astype(np.float32)
    got = float(rt.dot(to_dev(a, dev), to_dev(b, dev)).cpu())
    want = float(np.dot(a.astype(np.float64), b.astype(np.float64)))
    assert abs(got - want) <= 1e-6 * np.dot(np.abs(a), np.abs(b))
    s = to_dev(np.array([0.0, -2.5], np.float32), dev)
    out = rt.scaled_copy(to_dev(a, dev), s[1:2]).cpu().numpy()
    assert np.array_equal(out, (np.float32(-2.5) * a).astype(np.float32))


def test_fit_amplitude_and_opacity_over_bins(rt, dev):
    """Targets traced at A = 1.6, alpha = 0.7 over the four bins of the uneven workload;
    the fit from (1, 1) recovers both through the bins' adjoint."""
    w = inputs.turbulent(n=40, n_src=3, kappa_mean=0.08, num_rays=512, c=32.0, config_id=9)
    j0, k0 = to_dev(w.j_map, dev), to_dev(w.kappa_map, dev)
    a_true, alpha_true = 1.6, 0.7
    targets = rt.trace_bins(a_true * j0, alpha_true * k0, w.source_pos, w.num_rays, w.step_size,
                            w.radiation_velocity, w.time_step, kappa_scale=SCALES)
    A, alpha, losses = inverse.fit_amplitude_and_opacity(j0, k0, SCALES, targets, w.source_pos, w.num_rays,
                                                         w.step_size, w.radiation_velocity, w.time_step,
                                                         iters=200, lr=2e-2)
    note(f"fit: A {A:.4f} (true {a_true}), alpha {alpha:.4f} (true {alpha_true}); "
         f"loss {losses[0]:.3e} -> {losses[-1]:.3e}")
    assert abs(A - a_true) <= 0.02 * a_true
    assert abs(alpha - alpha_true) <= 0.03 * alpha_true
    assert losses[-1] <= 1e-3 * losses[0]
