"""rtmi_trace_bins_static: the stateless batched march with no allocation, its scratch
carved from the library's static per-device array.

It runs the same kernels on the same arguments as rtmi_trace_bins, so the deterministic
mode must agree bit for bit and the float mode to float-atomic reordering (checked at the
field tolerances of the parity tests: relative L2 <= 1e-5, per voxel <= 1e-4 where the
field exceeds 1e-6 of its maximum). Two calls in a row, the second smaller, check that
what the first call leaves in the shared array does not leak into the second.
"""

import ctypes
import sys

import numpy as np
import pytest
import torch

from paper_2511_09389_amd import inputs

pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[gpu-static] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch.device("cuda:0")


def field_close(got, want):
    got, want = got.double().cpu().numpy(), want.double().cpu().numpy()
    rel = float(np.linalg.norm(got - want) / np.linalg.norm(want))
    mask = np.abs(want) > 1e-6 * np.abs(want).max()
    per_voxel = float(np.max(np.abs(got[mask] - want[mask]) / np.abs(want[mask])))
    return rel, per_voxel


def case(dev, n, n_src, rays_choice, caps_range, scale, seed):
    """A turbulent grid of n^3 with n_src sources of mixed N_Omega and substep caps."""
    w = inputs.turbulent(n=n, n_src=n_src, kappa_mean=0.03, num_rays=1, ds=0.5, c=float(n), dt=1.0,
                         config_id=seed)
    rng = np.random.default_rng(seed)
    rays = rng.choice(np.array(rays_choice), size=n_src).astype(np.int32)
    caps = rng.integers(caps_range[0], caps_range[1], size=n_src).astype(np.int32)
    j = torch.from_numpy(w.j_map).to(dev)
    k = torch.from_numpy(w.kappa_map).to(dev)
    return w, rays, caps, np.asarray(scale, np.float32), j, k


CASES = [
    # (grid, sources, N_Omega choices, cap range, kappa scales): two launches of sources
    # and three bins first, then a smaller single-launch, single-bin call
    (64, 40, (256, 512, 1024, 2048), (16, 129), (1.0, 0.3, 0.05)),
    (20, 2, (64, 96), (4, 41), (1.0,)),
]


@pytest.mark.parametrize("deterministic", [False, True])
@pytest.mark.parametrize("path", ["tiled", "tiled_gather_pass", "direct"])
def test_static_equals_trace_bins_twice(rt, dev, deterministic, path):
    """(tiled_gather_pass: the gather pass's rows live in the static array too, and the
    second call's rows must come from its own gather pass, not the first call's.)"""
    p = rt.PATH_DIRECT if path == "direct" else rt.PATH_TILED
    gather = 3 if path == "tiled_gather_pass" else 0
    for i, (n, n_src, choice, caps_range, scale) in enumerate(CASES):
        note(f"call {i}: {n}^3, {n_src} sources, bins {len(scale)}, det {deterministic}, path {path}")
        w, rays, caps, sc, j, k = case(dev, n, n_src, choice, caps_range, scale, seed=50 + i)
        for r in sorted(set(int(v) for v in rays)):
            rt.prepare(r)
        out = torch.full((len(sc),) + w.shape, float("nan"), dtype=torch.float32, device=dev)
        got = rt.trace_bins_static(j, k, w.source_pos, rays, w.step_size, w.radiation_velocity,
                                   w.time_step, kappa_scale=sc, substep_cap=caps, out=out,
                                   deterministic=deterministic, path=p, gather_table=gather)
        want = rt.trace_bins(j, k, w.source_pos, rays, w.step_size, w.radiation_velocity, w.time_step,
                             kappa_scale=sc, substep_cap=caps, deterministic=deterministic, path=p,
                             gather_table=gather)
        torch.cuda.synchronize()
        assert got.data_ptr() == out.data_ptr()
        assert torch.isfinite(got).all()
        if deterministic:
            assert torch.equal(got.view(torch.int32), want.view(torch.int32)), f"call {i}"
        else:
            rel, per_voxel = field_close(got, want)
            note(f"call {i}: rel L2 {rel:.2e}, per voxel {per_voxel:.2e}")
            assert rel <= 1e-5 and per_voxel <= 1e-4, (i, rel, per_voxel)
    assert rt.dropped_records() == 0


def test_static_errors_before_enqueue(rt, dev):
    assert rt.static_scratch_bytes() == 384 << 20
    # a grid whose gather table alone (64 bytes per voxel) exceeds the static array (the
    # table is asked for: at this size the default is the gather pass, which fits)
    n = 256
    j = torch.zeros((n, n, n), dtype=torch.float32, device=dev)
    k = torch.zeros_like(j)
    out = torch.full((1, n, n, n), 7.0, dtype=torch.float32, device=dev)
    rt.prepare(256)
    with pytest.raises(rt.RtmiError) as e:
        rt.trace_bins_static(j, k, [[128.0, 128.0, 128.0]], [256], 0.5, 8.0, 1.0, out=out, gather_table=1)
    assert e.value.code == rt.ERR_RANGE and "static scratch" in str(e.value)
    # an N_Omega without a prepared direction table
    js = torch.zeros((8, 8, 8), dtype=torch.float32, device=dev)
    outs = torch.full((1, 8, 8, 8), 7.0, dtype=torch.float32, device=dev)
    with pytest.raises(rt.RtmiError) as e:
        rt.trace_bins_static(js, js, [[4.0, 4.0, 4.0]], [1237], 0.5, 2.0, 1.0, out=outs)
    assert e.value.code == rt.ERR_UNSUPPORTED and "rtmi_prepare" in str(e.value)
    torch.cuda.synchronize()
    assert bool((out == 7.0).all()) and bool((outs == 7.0).all())   # nothing was enqueued


def test_static_through_raw_c_abi(rt, dev):
    """The entry point called directly through ctypes (no binding), on a 16^3 grid."""
    w = inputs.uniform_blob(n=16, num_rays=128, c=6.0)
    rt.prepare(128)
    j = torch.from_numpy(w.j_map).to(dev)
    k = torch.from_numpy(w.kappa_map).to(dev)
    out = torch.empty((1,) + w.shape, dtype=torch.float32, device=dev)
    raw = ctypes.CDLL(rt.LIB_PATH)
    fn = raw.rtmi_trace_bins_static
    fn.restype = ctypes.c_int32
    P, I32, I64, F32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    fn.argtypes = [P, I64, P, I64, P, I32, I32, I32, I32, I32, P, P, P, F32, F32, F32, P, P, P]
    src = np.ascontiguousarray(w.source_pos, np.float32)
    nr = np.array([128], np.int32)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    code = fn(j.data_ptr(), 0, k.data_ptr(), 0, None, 1, 16, 16, 16, 1, src.ctypes.data, nr.ctypes.data, None,
              w.step_size, w.radiation_velocity, w.time_step, out.data_ptr(), None, stream)
    assert code == 0
    want = rt.trace_single(j, k, w.source_pos[0], 128, w.step_size, w.radiation_velocity, w.time_step)
    torch.cuda.synchronize()
    rel, per_voxel = field_close(out[0], want)
    assert rel <= 1e-5 and per_voxel <= 1e-4, (rel, per_voxel)
