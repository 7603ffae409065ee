"""GPU adjoint (through the C ABI) against the FP64 oracle VJP and finite differences."""

import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2511_09389_amd import inputs

pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[gpu-adjoint] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch.device("cuda:0")


def to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)


def rel_l2(got, want):
    return float(np.linalg.norm(np.asarray(got, np.float64) - want) / np.linalg.norm(want))


def per_voxel(got, want, scale, tol=1e-4, floor=1e-6):
    """Per-voxel check of a gradient: |got - want| <= tol * scale wherever scale exceeds
    floor * max(scale). With a sign-definite upstream gradient, scale = |want| (the
    field criterion). With a mixed-sign one, terms of both signs meet in a voxel and the
    gradient can cancel to nearly nothing; then scale is the oracle gradient for |G|,
    which bounds the sum of the terms' magnitudes (every other factor of a term is
    non-negative for j >= 0), so the check is relative to what was summed."""
    got = np.asarray(got, np.float64)
    scale = np.abs(scale)
    mask = scale > floor * scale.max()
    rel = np.abs(got[mask] - want[mask]) / scale[mask]
    assert rel.max() <= tol, f"max per-voxel error {rel.max():.3e} > {tol}"
    return float(rel.max())


@pytest.mark.parametrize("shape,src,rays,caps", [
    ((16, 16, 16), [[7.5, 8.2, 6.9], [2.0, 13.0, 14.5]], [64, 200], [0, 21]),
    ((19, 14, 22), [[-3.0, 5.0, 10.0], [18.5, 13.5, 0.5], [9.0, 7.0, 11.0]], [129, 64, 333], [0, 0, 17]),
])
def test_vjp_matches_oracle(rt, dev, shape, src, rays, caps):
    rng = np.random.default_rng(21)
    kap = (0.15 * rng.random(shape)).astype(np.float32)
    j = rng.random(shape).astype(np.float32)
    G = rng.normal(size=shape).astype(np.float32)
    src = np.asarray(src, np.float32)
    note(f"vjp {shape} rays={rays}")
    gj, gk = rt.trace_vjp(to_dev(j, dev), to_dev(kap, dev), src, rays, 0.5, 18.0, 1.0, to_dev(G, dev),
                          substep_cap=caps)
    wj, wk = oracle.trace_multi_vjp(j, kap, src, rays, 0.5, 18.0, 1.0, G, caps=caps)
    sj, sk = oracle.trace_multi_vjp(j, kap, src, rays, 0.5, 18.0, 1.0, np.abs(G), caps=caps)
    ej, ek = rel_l2(gj.cpu().numpy(), wj), rel_l2(gk.cpu().numpy(), wk)
    pj, pk = per_voxel(gj.cpu().numpy(), wj, sj), per_voxel(gk.cpu().numpy(), wk, sk)
    note(f"  rel L2: dL/dj {ej:.2e}, dL/dkappa {ek:.2e}; per voxel {pj:.2e}, {pk:.2e}")
    assert ej <= 1e-5
    assert ek <= 1e-5


def test_vjp_many_sources_span_launches(rt, dev):
    """70 sources (three launches of up to 32) with caps, some outside the box: each
    launch recomputes its tile schedule and chunk records into the one record buffer,
    and both deposits of every launch add into the gradients."""
    rng = np.random.default_rng(5)
    shape = (20, 18, 22)
    src = rng.uniform(-2, 20, size=(70, 3)).astype(np.float32)
    rays = rng.integers(8, 120, size=70)
    caps = rng.integers(0, 30, size=70)
    kap = (0.15 * rng.random(shape)).astype(np.float32)
    j = rng.random(shape).astype(np.float32)
    G = rng.normal(size=shape).astype(np.float32)
    note(f"vjp {shape}, 70 sources (3 launches)")
    gj, gk = rt.trace_vjp(to_dev(j, dev), to_dev(kap, dev), src, rays, 0.5, 18.0, 1.0, to_dev(G, dev),
                          substep_cap=caps)
    wj, wk = oracle.trace_multi_vjp(j, kap, src, rays, 0.5, 18.0, 1.0, G, caps=caps)
    sj, sk = oracle.trace_multi_vjp(j, kap, src, rays, 0.5, 18.0, 1.0, np.abs(G), caps=caps)
    assert rel_l2(gj.cpu().numpy(), wj) <= 1e-5
    assert rel_l2(gk.cpu().numpy(), wk) <= 1e-5
    per_voxel(gj.cpu().numpy(), wj, sj)
    per_voxel(gk.cpu().numpy(), wk, sk)


def test_vjp_full_inverse_configuration(rt, dev):
    """The inverse-problem workload at its full size (64^3 turbulent kappa, 8 sources,
    N_Omega = 2048, N_s = 128) with a positive upstream gradient, so both gradients are
    sign-definite (dL/dj >= 0, dL/dkappa <= 0) and the field criterion applies voxel by
    voxel: relative L2 <= 1e-5 and per-voxel relative error <= 1e-4 wherever the oracle
    gradient exceeds 1e-6 of its largest magnitude."""
    w = inputs.inverse()
    rng = np.random.default_rng(64)
    G = rng.random(w.shape).astype(np.float32)
    note("vjp 64^3, 8 sources x 2048 rays x 128 substeps, G >= 0")
    gj, gk = rt.trace_vjp(to_dev(w.j_map, dev), to_dev(w.kappa_map, dev), w.source_pos, w.num_rays,
                          w.step_size, w.radiation_velocity, w.time_step, to_dev(G, dev))
    wj, wk = oracle.trace_multi_vjp(w.j_map, w.kappa_map, w.source_pos, w.num_rays, w.step_size,
                                    w.radiation_velocity, w.time_step, G)
    assert wj.min() >= 0.0 and wk.max() <= 0.0
    gj, gk = gj.cpu().numpy(), gk.cpu().numpy()
    ej, ek = rel_l2(gj, wj), rel_l2(gk, wk)
    pj, pk = per_voxel(gj, wj, wj), per_voxel(gk, wk, wk)
    note(f"  rel L2: dL/dj {ej:.2e}, dL/dkappa {ek:.2e}; per voxel {pj:.2e}, {pk:.2e}")
    assert ej <= 1e-5 and ek <= 1e-5


def test_vjp_matches_central_differences(rt, dev):
    """16^3, 64 rays: dL/dkappa and dL/dj against central differences (h = 1e-3) of the
    FP64 oracle, for L = <G, J>."""
    rng = np.random.default_rng(4)
    shape = (16, 16, 16)
    w = inputs.inverse(n=16, n_src=2, num_rays=64, c=12.0)
    j, kap = w.j_map, w.kappa_map.astype(np.float64)
    G = rng.normal(size=shape)
    gj, gk = rt.trace_vjp(to_dev(j, dev), to_dev(kap, dev), w.source_pos, 64, 0.5, 12.0, 1.0,
                          to_dev(G, dev))
    gj, gk = gj.cpu().numpy(), gk.cpu().numpy()

    def loss(jj, kk):
        return float(np.sum(G * oracle.trace_multi(jj, kk, w.source_pos, 64, 0.5, 12.0, 1.0)))

    h = 1e-3
    for v in np.argsort(-np.abs(gk.ravel()))[:6]:
        e = np.zeros(kap.size)
        e[v] = h
        fd = (loss(j, kap + e.reshape(shape)) - loss(j, kap - e.reshape(shape))) / (2 * h)
        assert abs(gk.ravel()[v] - fd) <= 2e-4 * abs(fd) + 1e-6, (v, gk.ravel()[v], fd)
    for v in np.argsort(-np.abs(gj.ravel()))[:6]:
        e = np.zeros(j.size)
        e[v] = h
        fd = (loss(j + e.reshape(shape), kap) - loss(j - e.reshape(shape), kap)) / (2 * h)
        assert abs(gj.ravel()[v] - fd) <= 2e-5 * abs(fd) + 1e-6, (v, gj.ravel()[v], fd)


def test_autograd_function_and_amplitude_recovery(rt, dev):
    """Sec. 4: j = A e0 with a fixed template; gradient descent on A through autograd
    reaches the closed-form MSE minimiser <F, I_ref>/<F, F> (here A_true)."""
    from paper_2511_09389_amd.autograd import march_field
    w = inputs.inverse(n=24, n_src=3, num_rays=256, c=16.0)
    e0 = to_dev(w.j_map, dev)
    kap = to_dev(w.kappa_map, dev)
    a_true = 1.7
    ref = a_true * march_field(e0, kap, w.source_pos, 256, 0.5, 16.0, 1.0).detach()
    F = march_field(e0, kap, w.source_pos, 256, 0.5, 16.0, 1.0).detach()
    a_star = float((F * ref).sum() / (F * F).sum())
    assert abs(a_star - a_true) < 1e-5
    A = torch.tensor(0.2, device=dev, requires_grad=True)
    opt = torch.optim.Adam([A], lr=0.1)
    for _ in range(150):
        opt.zero_grad()
        loss = torch.mean((march_field(A * e0, kap, w.source_pos, 256, 0.5, 16.0, 1.0) - ref) ** 2)
        loss.backward()
        opt.step()
    assert abs(float(A) - a_star) < 2e-3, float(A)
    # dL/dA through autograd equals <dL/dJ, F> exactly
    A2 = torch.tensor(1.1, device=dev, requires_grad=True)
    out = march_field(A2 * e0, kap, w.source_pos, 256, 0.5, 16.0, 1.0)
    Gt = torch.randn_like(out)
    (out * Gt).sum().backward()
    # <G, F> cancels (G has random signs): judge the error against sum |G F|
    scale = float((Gt * F).abs().sum())
    assert abs(float(A2.grad) - float((Gt * F).sum())) <= 1e-5 * scale


def test_inverse_problem_reduces_loss(rt, dev):
    from paper_2511_09389_amd.inverse import recover_emissivity
    w = inputs.inverse(n=32, n_src=4, num_rays=512, c=32.0)
    kap = to_dev(w.kappa_map, dev)
    target = rt.trace_multi(to_dev(w.j_map, dev), kap, w.source_pos, 512, 0.5, 32.0, 1.0)
    j, losses = recover_emissivity(kap, target, w.source_pos, 512, 0.5, 32.0, 1.0, iters=40, lr=1e-2)
    note(f"inverse: loss {losses[0]:.3e} -> {losses[-1]:.3e}")
    assert losses[-1] < 0.2 * losses[0]


def test_inverse_problem_full_configuration(rt, dev):
    """The inverse-problem workload as specified: 64^3 turbulent kappa (mean 0.03), the
    true j made of 8 blobs with a source at each, N_Omega = 2048, N_s = 128, Adam
    (lr 1e-2) for 200 iterations from j = 0 on the mean squared field error."""
    import time
    from paper_2511_09389_amd.inverse import recover_emissivity
    w = inputs.inverse()
    kap = to_dev(w.kappa_map, dev)
    j_true = to_dev(w.j_map, dev)
    target = rt.trace_multi(j_true, kap, w.source_pos, w.num_rays, w.step_size, w.radiation_velocity,
                            w.time_step)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    j, losses = recover_emissivity(kap, target, w.source_pos, w.num_rays, w.step_size,
                                   w.radiation_velocity, w.time_step, iters=200, lr=1e-2)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    field = rt.trace_multi(j, kap, w.source_pos, w.num_rays, w.step_size, w.radiation_velocity, w.time_step)
    f_err = float((field - target).norm() / target.norm())
    j_err = float((j - j_true).norm() / j_true.norm())
    note(f"inverse 64^3: loss {losses[0]:.3e} -> {losses[-1]:.3e} in 200 Adam steps ({dt:.2f} s); "
         f"field rel L2 {f_err:.3e}, j rel L2 {j_err:.3e}")
    assert losses[-1] < 0.05 * losses[0]
    assert f_err < 0.25


def test_inverse_problem_resumes_from_a_checkpoint(rt, dev, tmp_path):
    """Twenty Adam steps, a save and a load of the optimiser state, then twenty more, end
    where forty steps in one go end (up to float-atomic summation order)."""
    from paper_2511_09389_amd.inverse import InverseState, recover_emissivity
    w = inputs.inverse(n=24, n_src=3, num_rays=256, c=16.0)
    kap = to_dev(w.kappa_map, dev)
    target = rt.trace_multi(to_dev(w.j_map, dev), kap, w.source_pos, 256, 0.5, 16.0, 1.0)
    args = (w.source_pos, 256, 0.5, 16.0, 1.0)
    j_once, losses_once = recover_emissivity(kap, target, *args, iters=40)
    st = InverseState.start(target)
    recover_emissivity(kap, target, *args, iters=20, state=st)
    st.save(tmp_path / "inv.pt")
    back = InverseState.load(tmp_path / "inv.pt", dev)
    assert back.step == 20 and len(back.losses) == 20
    j_two, _ = recover_emissivity(kap, target, *args, iters=20, state=back)
    assert back.step == 40 and len(back.losses) == 40
    assert np.allclose(back.losses, losses_once, rtol=1e-4, atol=0)
    assert float((j_two - j_once).norm() / j_once.norm()) < 1e-4
