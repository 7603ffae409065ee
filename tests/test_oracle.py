"""CPU tests of the FP64 oracle against its pins (no GPU needed)."""

import json
import math
import os
import types

import numpy as np
import pytest

import oracle
from oracle import march as oracle_march
from paper_2511_09389_amd import inputs

from oracle_pins import ALL_PINS, FOUR_PI

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.parametrize("pin", ALL_PINS, ids=lambda p: p.__name__)
def test_pin(pin):
    pin(oracle)


# Plausible mistakes, planted in a copy of the oracle's source on the CPU. Every one of them
# must make at least one pin fail; this shows the pins constrain each step of the method.
MUTANTS = {
    "emission without exp(-tau_k)": ("j_k * np.exp(-tau) * ds", "j_k * ds"),
    "no attenuation over the step": ("intensity * np.exp(-kappa_k * ds)", "intensity"),
    "emission uses tau_{k+1}": ("j_k * np.exp(-tau) * ds", "j_k * np.exp(-(tau + kappa_k * ds)) * ds"),
    "deposit without stencil weight": ("w_ray * w * intensity", "w_ray * intensity"),
    "deposit pre-update intensity": [("        intensity = intensity * np.exp", "        prev_i = intensity\n        intensity = intensity * np.exp"),
                                     ("np.add.at(field, idx, w_ray * w * intensity)", "np.add.at(field, idx, w_ray * w * prev_i)")],
    "transposed flat index": ("(ia * shape[1] + ib) * shape[2] + ic", "(ic * shape[1] + ib) * shape[0] + ia"),
    "kappa at floor": ('near = np.rint(x)', 'near = np.floor(x)'),
    "kappa at x_{k+1}": ('near = np.rint(x)', 'near = np.rint(_positions(k + 1, source_pos, dirs, ds, geometry))'),
    "swapped 1-D weights": ("wa = frac[:, 0] if cx else 1.0 - frac[:, 0]", "wa = 1.0 - frac[:, 0] if cx else frac[:, 0]"),
    "weight 4pi/(N+1)": ("FOUR_PI / n_rays if weight", "FOUR_PI / (n_rays + 1) if weight"),
    "one substep too many": ("n = int(math.ceil((c * dt) / ds))", "n = int(math.ceil((c * dt) / ds)) + 1"),
    "floor instead of ceil": ("n = int(math.ceil((c * dt) / ds))", "n = int(math.floor((c * dt) / ds))"),
    "closed-lattice z": ("z = 1.0 - (2.0 * i + 1.0) / n", "z = 1.0 - 2.0 * i / max(n - 1, 1)"),
    "reversed azimuth": ("g = (3.0 - math.sqrt(5.0)) / 2.0", "g = (math.sqrt(5.0) - 1.0) / 2.0"),
    "x and y swapped in directions": ("out[i, 0] = r * math.cos(phi)", "out[i, 0] = r * math.sin(phi)"),
    "positions from x_1": ("t = np.float32(np.float32(k) * np.float32(ds))", "t = np.float32(np.float32(k + 1) * np.float32(ds))"),
    "no clamp on hi": ("hi = np.clip(i0 + 1, 0, shape - 1)", "hi = np.clip(i0 + 1, 0, shape)"),
    "lo clamp at 1": ("lo = np.clip(i0, 0, shape - 1)", "lo = np.clip(i0, 1, shape - 1)"),
    "tau not accumulated": ("tau = tau + kappa_k * ds", "tau = kappa_k * ds"),
}


def _mutant(edits):
    src = open(oracle_march.__file__).read()
    for old, new in ([edits] if isinstance(edits, tuple) else edits):
        assert old in src, old
        src = src.replace(old, new, 1)
    mod = types.ModuleType("oracle_mutant")
    exec(compile(src, "oracle_mutant", "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name):
    mod = _mutant(MUTANTS[name])
    failed = []
    for pin in ALL_PINS:
        try:
            pin(mod)
        except Exception:  # noqa: BLE001 - any failure (assert, index error) counts
            failed.append(pin.__name__)
    assert failed, f"no pin catches: {name}"


def test_multi_is_sum_of_singles():
    w = inputs.small_turbulent(n=12, n_src=3, num_rays=20, c=6.0)
    caps = [0, 5, 9]
    nr = [20, 7, 33]
    tot = oracle.trace_multi(w.j_map, w.kappa_map, w.source_pos, nr, 0.5, 6.0, 1.0, caps=caps)
    acc = sum(oracle.trace_single(w.j_map, w.kappa_map, w.source_pos[s], nr[s], 0.5, 6.0, 1.0,
                                  cap=caps[s]) for s in range(3))
    assert np.array_equal(tot, acc)


def test_bins_are_independent_problems():
    w = inputs.small_turbulent(n=10, n_src=2, num_rays=16, c=5.0)
    scale = np.array([1.0, 0.5, 0.125], np.float32)
    out = oracle.trace_bins(w.j_map, w.kappa_map, scale, w.source_pos, 16, 0.5, 5.0, 1.0)
    assert out.shape == (3,) + w.shape
    for b in range(3):
        ref = oracle.trace_multi(w.j_map, w.kappa_map.astype(np.float64) * float(scale[b]),
                                 w.source_pos, 16, 0.5, 5.0, 1.0)
        assert np.array_equal(out[b], ref)
    # more opacity, less light
    assert out[0].sum() < out[1].sum() < out[2].sum()
    js = np.stack([w.j_map, 2 * w.j_map])
    out2 = oracle.trace_bins(js, w.kappa_map, [1.0, 1.0], w.source_pos, 16, 0.5, 5.0, 1.0)
    assert np.allclose(out2[1], 2 * out2[0], rtol=1e-13)


def test_zero_substeps_gives_zero_field():
    w = inputs.small_turbulent(n=8, n_src=1, num_rays=8, c=4.0)
    f = oracle.trace_single(w.j_map, w.kappa_map, w.source_pos[0], 8, 0.5, 4.0, 0.0)
    assert not f.any()


def test_fp32_geometry_is_close_to_fp64_geometry():
    """The fp32 sample points differ from the exact ones by ~1e-6 cells; on a smooth
    problem the fields agree to that order, away from flipped index decisions."""
    w = inputs.uniform_blob(n=16, num_rays=64, c=8.0)
    a = oracle.trace_single(w.j_map, w.kappa_map, w.source_pos[0], 64, 0.5, 8.0, 1.0)
    b = oracle.trace_single(w.j_map, w.kappa_map, w.source_pos[0], 64, 0.5, 8.0, 1.0, geometry="fp64")
    assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-5


def _point_source_error(n_rays, n=33, kappa0=0.05, c=14.0):
    """Mean relative error against Eq. (3) for one narrow Gaussian source, excluding the
    source voxel and a one-voxel border (Sec. 3, "Analytical validation"). The luminosity
    of Eq. (3) is not printed; it follows from the scheme: past the blob each ray carries
    I = e^{-kappa r} S with S the mean of sum_m j_m e^{kappa ds} ds, and the deposits of
    N rays spaced ds apart give J = S e^{-kappa r} / (ds r^2), i.e. L = 4 pi S / ds."""
    c0 = n // 2
    ds = 0.5
    j = inputs.gaussian_blobs(n, [np.array([c0] * 3, np.float32)], [0.6], [1.0], cutoff=1e9)
    kap = np.full((n, n, n), kappa0, np.float32)
    field, rays_i, rays_tau = oracle.trace_single(j, kap, (c0, c0, c0), n_rays, ds, c, 1.0,
                                                  return_rays=True)
    s_mean = float(np.mean(rays_i[:, -1] * np.exp(rays_tau[:, -1])))
    grid = np.indices((n, n, n)).astype(np.float64) - c0
    r = np.sqrt((grid ** 2).sum(axis=0))
    ref = (FOUR_PI * s_mean / ds) / (FOUR_PI * np.maximum(r, 1e-9) ** 2) * np.exp(-kappa0 * r)
    mask = np.zeros_like(r, bool)
    mask[1:-1, 1:-1, 1:-1] = True
    mask &= (r > 0) & (r < c - 1.0)
    return float(np.mean(np.abs(field[mask] - ref[mask]) / ref[mask]))


def test_point_source_matches_eq3_and_converges_in_rays():
    errs = [_point_source_error(nr) for nr in (256, 1024, 4096)]
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.10, errs          # a few per cent, as in the paper's benchmark


def test_paper_numbers_fixture():
    with open(os.path.join(HERE, "golden", "paper_numbers.json")) as fh:
        g = json.load(fh)
    t = g["timing"]
    # "top 0.1 % density peaks" and "2,097 sources" describe the same 128^3 workload
    assert math.floor(0.001 * t["grid"] ** 3) == t["sources"]
    w = inputs.peaks()
    assert w.n_src == t["sources"] and w.shape == (t["grid"],) * 3
    assert int(w.num_rays[0]) == t["rays_per_source"]
    # the ray-substep count the stand-in workload implies at 256 substeps
    assert t["sources"] * t["rays_per_source"] * 256 == 2_198_863_872


def test_voxel_sampled_oracle_equals_full_oracle():
    """oracle.trace_voxels (the march restricted to the rays that can reach a few voxels)
    gives the full oracle's value at every interior voxel: several sources, one outside
    the box, a substep cap, and a bin scale on kappa."""
    rng = np.random.default_rng(1)
    shape = (20, 17, 23)
    j = rng.random(shape).astype(np.float32)
    k = (0.2 * rng.random(shape)).astype(np.float32)
    src = np.array([[5.5, 8.2, 11.0], [-3.0, 4.0, 25.0], [19.2, 0.1, 3.3]], np.float32)
    rays, caps = [200, 64, 129], [0, 17, 0]
    vox = np.stack(np.meshgrid(*[np.arange(1, n - 1) for n in shape], indexing="ij"), -1).reshape(-1, 3)
    full = oracle.trace_multi(j, k, src, rays, 0.5, 20.0, 1.0, caps=caps)
    got = oracle.march.trace_voxels(j, k, src, rays, 0.5, 20.0, 1.0, vox, caps=caps)
    want = full[vox[:, 0], vox[:, 1], vox[:, 2]]
    assert np.max(np.abs(got - want)) <= 1e-13 * np.abs(want).max()
    scale = np.float32(0.296296)
    binned = oracle.trace_bins(j, k, [1.0, scale], src, rays, 0.5, 20.0, 1.0, caps=caps)[1]
    sub = vox[::7]
    got = oracle.march.trace_voxels(j, k, src, rays, 0.5, 20.0, 1.0, sub, caps=caps, kappa_scale=scale)
    want = binned[sub[:, 0], sub[:, 1], sub[:, 2]]
    assert np.max(np.abs(got - want)) <= 1e-13 * np.abs(want).max()
    with pytest.raises(ValueError):
        oracle.march.trace_voxels(j, k, src, rays, 0.5, 20.0, 1.0, [[0, 3, 3]])
