"""Plans (the batched march set up once): equal to the stateless routine, reusable,
capturable in a HIP graph, and tunable.

A plan computes exactly what rtmi_trace_bins computes (the multi-source sum of Sec. 2
over sources with their own N_Omega and caps, times bins scaling kappa): the same kernels
run on the same arguments, only the tile schedule is computed once. So the deterministic
mode must agree bit for bit, and the float mode to float-atomic reordering.
"""

import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2511_09389_amd import autotune, inputs

pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[gpu-plan] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def batch(dev):
    """A small uneven batch: 40 sources (two launches of up to 32), N_Omega in
    {256..4096}, substep caps, three bins scaling kappa."""
    w = inputs.turbulent(n=48, n_src=40, kappa_mean=0.03, num_rays=1, ds=0.5, c=40.0, dt=1.0,
                         config_id=7)
    rng = np.random.default_rng(77)
    rays = rng.choice(np.array([256, 512, 1024, 4096]), size=40).astype(np.int32)
    caps = rng.integers(10, 81, size=40).astype(np.int32)
    scale = np.array([1.0, 0.3, 0.05], np.float32)
    j = torch.from_numpy(w.j_map).to(dev)
    k = torch.from_numpy(w.kappa_map).to(dev)
    return w, rays, caps, scale, j, k


def rel_l2(a, b):
    a, b = a.double(), b.double()
    return float((a - b).norm() / b.norm())


def test_plan_equals_trace_bins(rt, dev, batch):
    w, rays, caps, scale, j, k = batch
    want = rt.trace_bins(j, k, w.source_pos, rays, w.step_size, w.radiation_velocity, w.time_step,
                         kappa_scale=scale, substep_cap=caps)
    plan = rt.Plan(w.shape, w.source_pos, rays, w.step_size, w.radiation_velocity, w.time_step,
                   n_bins=3, kappa_scale=scale, substep_cap=caps)
    assert plan.workspace_bytes > 0
    got = plan.execute(j, k)
    err = rel_l2(got, want)
    note(f"plan vs trace_bins rel L2 {err:.2e}, workspace {plan.workspace_bytes / 2**20:.1f} MiB")
    assert err < 1e-6


def test_plan_deterministic_is_bitwise_trace_bins(rt, dev, batch):
    w, rays, caps, scale, j, k = batch
    want = rt.trace_bins(j, k, w.source_pos, rays, w.step_size, w.radiation_velocity, w.time_step,
                         kappa_scale=scale, substep_cap=caps, deterministic=True)
    plan = rt.Plan(w.shape, w.source_pos, rays, w.step_size, w.radiation_velocity, w.time_step,
                   n_bins=3, kappa_scale=scale, substep_cap=caps, deterministic=True,
                   tile_item_chunks=333)
    for _ in range(3):
        got = plan.execute(j, k)
        assert torch.equal(got.view(torch.int32), want.view(torch.int32))


@pytest.mark.parametrize("ds,c,outside", [(0.9, 20.0, False), (1.7, 40.0, True), (4.5, 60.0, True)])
def test_stateless_record_bound_drops_nothing(rt, dev, ds, c, outside):
    """A stateless call sizes its chunk-record buffer by an upper bound on the tiles that
    can list one chunk (it grows with the step size); a plan counts its records and
    allocates exactly. A record dropped for want of space would change the deterministic
    field, so the two must agree bit for bit, here with large steps and with sources
    outside the box whose rays run along its faces; and both must match the oracle."""
    rng = np.random.default_rng(int(ds * 10))
    shape = (40, 36, 44)
    j = rng.random(shape).astype(np.float32)
    kap = (0.05 * rng.random(shape)).astype(np.float32)
    src = rng.uniform(0, 35, size=(6, 3)).astype(np.float32)
    if outside:
        src[:3] = np.array([[-7.5, 10.0, 20.0], [45.0, -3.0, 50.0], [20.0, 18.0, -12.0]], np.float32)
    rays = [512, 300, 1000, 64, 777, 2048]
    note(f"record bound: ds {ds}, c dt {c}, sources outside the box: {outside}")
    jd, kd = torch.from_numpy(j).to(dev), torch.from_numpy(kap).to(dev)
    want = rt.trace_bins(jd, kd, src, rays, ds, c, 1.0, deterministic=True)
    plan = rt.Plan(shape, src, rays, ds, c, 1.0, deterministic=True)
    got = plan.execute(jd, kd)
    assert torch.equal(got.view(torch.int32), want.view(torch.int32))
    ref = oracle.trace_multi(j, kap, src, rays, ds, c, 1.0)
    err = np.linalg.norm(want[0].cpu().numpy() - ref) / np.linalg.norm(ref)
    assert err <= 1e-5, err


def test_plan_matches_oracle_small(rt, dev):
    """Parity of a plan with the FP64 oracle on a small two-source, two-bin case."""
    w = inputs.uniform_blob()
    src = np.array([[16.0, 16.0, 16.0], [9.5, 20.25, 12.0]], np.float32)
    scale = np.array([1.0, 0.5], np.float32)
    j = torch.from_numpy(w.j_map).to(dev)
    k = torch.from_numpy(w.kappa_map).to(dev)
    plan = rt.Plan(w.shape, src, [256, 128], w.step_size, w.radiation_velocity, w.time_step,
                   n_bins=2, kappa_scale=scale, substep_cap=[0, 20])
    got = plan.execute(j, k).cpu().numpy().astype(np.float64)
    want = oracle.trace_bins(w.j_map, w.kappa_map, scale, src, [256, 128], w.step_size,
                             w.radiation_velocity, w.time_step, caps=[0, 20])
    for b in range(2):
        err = np.linalg.norm(got[b] - want[b]) / np.linalg.norm(want[b])
        assert err <= 1e-5, (b, err)


def test_plan_reuse_with_new_maps(rt, dev, batch):
    """One plan, new maps each time: the field is linear in j (P6)."""
    w, rays, caps, scale, j, k = batch
    plan = rt.Plan(w.shape, w.source_pos, rays, w.step_size, w.radiation_velocity, w.time_step,
                   n_bins=3, kappa_scale=scale, substep_cap=caps)
    a = plan.execute(j, k).clone()
    b = plan.execute(2.5 * j, k)
    assert rel_l2(b, 2.5 * a) < 1e-6


def test_graph_replay_equals_eager(rt, dev, batch):
    """Capture plan.execute in a CUDA/HIP graph; every replay (with eager work and
    synchronisations between them, and the input changed in place) equals eager."""
    w, rays, caps, scale, j, k = batch
    plan = rt.Plan(w.shape, w.source_pos, rays, w.step_size, w.radiation_velocity, w.time_step,
                   n_bins=3, kappa_scale=scale, substep_cap=caps, deterministic=True)
    j_in = j.clone()
    out = torch.empty((3,) + w.shape, device=dev)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.execute(j_in, k, out)          # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.execute(j_in, k, out)
    for rep in range(4):
        factor = 1.0 + 0.5 * rep
        j_in.copy_(j * factor)
        _ = rt.trace_multi(j, k, w.source_pos[:3], 256, w.step_size, w.radiation_velocity, w.time_step)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        eager = plan.execute(j_in, k)
        torch.cuda.synchronize()
        assert torch.equal(out.view(torch.int32), eager.view(torch.int32)), rep
    note("4 graph replays equal eager executions bit for bit (deterministic mode)")


def test_plan_errors(rt, dev, batch):
    w, rays, caps, scale, j, k = batch
    with pytest.raises(rt.RtmiError):
        rt.Plan(w.shape, w.source_pos, rays, -1.0, w.radiation_velocity, w.time_step)
    plan = rt.Plan(w.shape, w.source_pos, rays, w.step_size, w.radiation_velocity, w.time_step)
    with pytest.raises(ValueError):
        plan.execute(j[:-1], k)
    plan.close()
    with pytest.raises(RuntimeError):
        plan.execute(j, k)


def test_autotune_picks_and_caches(rt, dev, batch, tmp_path, monkeypatch):
    w, rays, caps, scale, j, k = batch
    monkeypatch.setenv("RTMI_TUNE_CACHE", str(tmp_path / "tune.json"))
    best, timings = autotune.tune_item_chunks(j, k, w.source_pos, rays, w.step_size,
                                              w.radiation_velocity, w.time_step, n_bins=3,
                                              kappa_scale=scale, substep_cap=caps,
                                              candidates=(256, 1024, 4096), reps=2)
    assert best in (256, 1024, 4096) and len(timings) == 3
    note(f"autotune timings (ms): {timings} -> {best}")
    again, t2 = autotune.tune_item_chunks(j, k, w.source_pos, rays, w.step_size,
                                          w.radiation_velocity, w.time_step, n_bins=3,
                                          kappa_scale=scale, substep_cap=caps,
                                          candidates=(256, 1024, 4096), reps=2)
    assert again == best and t2 == {}
    knobs, t3 = autotune.tune(j, k, w.source_pos, rays, w.step_size, w.radiation_velocity, w.time_step,
                              n_bins=3, kappa_scale=scale, substep_cap=caps, reps=2,
                              candidates={"tile_item_chunks": (1024, 4096)})
    note(f"knob search (ms): {t3} -> {knobs}")
    # coordinate descent: 2 item sizes, then 2 more occupancy settings, 3 more gather
    # settings and 1 more launch split (40 sources)
    assert len(t3) == 8 and set(knobs) == set(autotune.DEFAULTS)
    assert knobs["tile_item_chunks"] in (1024, 4096) and knobs["gather_table"] in (0, 1, 2, 3)
    again, t4 = autotune.tune(j, k, w.source_pos, rays, w.step_size, w.radiation_velocity, w.time_step,
                              n_bins=3, kappa_scale=scale, substep_cap=caps, reps=2,
                              candidates={"tile_item_chunks": (1024, 4096)})
    assert again == knobs and t4 == {}
    plan = autotune.tuned_plan(j, k, w.source_pos, rays, w.step_size, w.radiation_velocity,
                               w.time_step, n_bins=3, kappa_scale=scale, substep_cap=caps)
    want = rt.trace_bins(j, k, w.source_pos, rays, w.step_size, w.radiation_velocity, w.time_step,
                         kappa_scale=scale, substep_cap=caps)
    assert rel_l2(plan.execute(j, k), want) < 1e-6
    for knob, values in (("tile_groups_per_cu", (1, 2)), ("gather_table", (2, 3)), ("sources_per_launch", (7,))):
        for v in values:
            p2 = rt.Plan(w.shape, w.source_pos, rays, w.step_size, w.radiation_velocity, w.time_step, n_bins=3,
                         kappa_scale=scale, substep_cap=caps, deterministic=True, **{knob: v})
            p1 = rt.Plan(w.shape, w.source_pos, rays, w.step_size, w.radiation_velocity, w.time_step, n_bins=3,
                         kappa_scale=scale, substep_cap=caps, deterministic=True)
            a, b = p2.execute(j, k), p1.execute(j, k)
            if knob == "gather_table":
                # the maps round the interpolation on the box faces differently (weights
                # 1, 0 against 1 - f, f on one clamped voxel), and the gather pass computes
                # the table's interpolation in another kernel: the field to rounding
                assert rel_l2(a, b) < 1e-6, (knob, v)
                note(f"deterministic field, gather_table={v} vs the default: bitwise equal {torch.equal(a, b)}")
            else:   # the launch shape: not a bit of the field changes
                assert torch.equal(a, b), (knob, v)
            p1.close()
            p2.close()


def test_plan_per_bin_maps(rt, dev, batch):
    """Per-bin j and kappa maps (bin strides = nx*ny*nz) through a plan equal trace_bins."""
    w, rays, caps, scale, j, k = batch
    jb = torch.stack([j, 0.5 * j, 2.0 * j]).contiguous()
    kb = torch.stack([k, 0.3 * k, 1.7 * k]).contiguous()
    want = rt.trace_bins(jb, kb, w.source_pos, rays, w.step_size, w.radiation_velocity, w.time_step,
                         substep_cap=caps, deterministic=True)
    plan = rt.Plan(w.shape, w.source_pos, rays, w.step_size, w.radiation_velocity, w.time_step,
                   n_bins=3, per_bin_j=True, per_bin_kappa=True, substep_cap=caps, deterministic=True)
    got = plan.execute(jb, kb)
    assert torch.equal(got.view(torch.int32), want.view(torch.int32))


@pytest.mark.parametrize("chunks", [1, 100, 100000])
def test_schedule_does_not_change_the_bits(rt, dev, batch, chunks):
    """In the deterministic mode the work-item size (1 chunk: every tile split into the
    maximum number of items; 100000: one item per tile) leaves the field bit for bit."""
    w, rays, caps, scale, j, k = batch
    want = rt.trace_bins(j, k, w.source_pos, rays, w.step_size, w.radiation_velocity, w.time_step,
                         kappa_scale=scale, substep_cap=caps, deterministic=True)
    got = rt.trace_bins(j, k, w.source_pos, rays, w.step_size, w.radiation_velocity, w.time_step,
                        kappa_scale=scale, substep_cap=caps, deterministic=True, tile_item_chunks=chunks)
    assert torch.equal(got.view(torch.int32), want.view(torch.int32))
