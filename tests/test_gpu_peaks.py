"""The rate microbenchmarks of librtmi_peaks.so (the peaks the benchmark's rooflines are
quoted against): every call succeeds, reports the work of one launch as stated in its
header, and the rates are ordered as the hardware allows (a random-slot LDS add is no
faster than a consecutive-slot one; L2-resident gathers beat HBM-resident ones)."""

import sys

import pytest
import torch

pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[gpu-peaks] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def peaks():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2511_09389_amd import peaks
    return peaks


def test_copy_and_gathers(peaks):
    rate, moved = peaks.copy(64 << 20, reps=2)
    assert moved == 2 * (64 << 20) and rate > 1e11
    l2, g_l2 = peaks.gather(2 << 20, iters=16, reps=2)
    hbm, g_hbm = peaks.gather(1 << 30, iters=4, reps=2)
    note(f"copy {rate / 1e12:.2f} TB/s, gather L2 {l2 / 1e12:.2f} TB/s, HBM {hbm / 1e12:.2f} TB/s")
    assert g_l2 > 0 and g_hbm > 0 and l2 > hbm


def test_lds_atomics(peaks):
    rates = {k: peaks.lds_atomic(k, iters=240, reps=2) for k in peaks.LDS_KINDS}
    note({k: f"{v[0] / 1e12:.3f} T/s" for k, v in rates.items()})
    full = {k: v[1] for k, v in rates.items() if k in ("f64", "u64", "f32", "f64_random", "u64_random")}
    assert len(set(full.values())) == 1 and rates["f64"][1] > 0   # the same adds per launch
    assert rates["f64_random_half"][1] * 2 == rates["f64"][1]
    assert rates["f64_random_eighth"][1] * 8 == rates["f64"][1]
    assert all(v[0] > 0 for v in rates.values())
    assert rates["f64_random"][0] <= 1.1 * rates["f64"][0]
    # fewer adding lanes cost less per instruction but more per add
    assert rates["f64_random_eighth"][0] < rates["f64_random"][0]
    with pytest.raises(RuntimeError):
        peaks.lds_atomic("f64", iters=7)       # iters must be a multiple of the slots per lane


def test_global_atomics(peaks):
    co, n = peaks.global_atomic(16 << 20, scattered=False, iters=8, reps=2)
    sc, _ = peaks.global_atomic(16 << 20, scattered=True, iters=8, reps=2)
    note(f"global f32 atomics: coalesced {co / 1e9:.1f} G/s, scattered {sc / 1e9:.1f} G/s")
    assert n > 0 and co > sc > 0
