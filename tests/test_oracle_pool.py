"""The process-pool oracle helper (used by the large GPU parity tests) returns what the
oracle returns in one process: the same sum over sources, split into groups."""

import numpy as np

import oracle
import oracle_pool
from paper_2511_09389_amd import inputs


def test_pool_sum_equals_single_process_oracle():
    kw = {"n": 20, "n_src": 5, "num_rays": 64, "c": 12.0, "seed_sample": 3}
    w = inputs.small_turbulent(**kw)
    picks = [4, 0, 2, 3]
    got = oracle_pool.trace_bins_subset("small_turbulent", kw, picks, workers=3)
    want = oracle.trace_multi(w.j_map, w.kappa_map, w.source_pos[picks], w.num_rays[picks], w.step_size,
                              w.radiation_velocity, w.time_step)
    assert got.shape == (1,) + w.shape
    assert np.max(np.abs(got[0] - want)) <= 1e-13 * want.max()
    vox = [np.array([[3, 4, 5], [10, 10, 10], [18, 1, 7]])]
    v = oracle_pool.trace_voxels_bins("small_turbulent", kw, vox, workers=1)[0]
    full = oracle.trace_multi(w.j_map, w.kappa_map, w.source_pos, w.num_rays, w.step_size,
                              w.radiation_velocity, w.time_step)
    assert np.allclose(v, full[vox[0][:, 0], vox[0][:, 1], vox[0][:, 2]], rtol=1e-13, atol=0)
