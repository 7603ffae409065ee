"""The FP64 oracle spread over host processes (test infrastructure).

Fields add over sources (Sec. 2, loop-and-sum) and bins are independent problems (Sec. 2,
"Frequency-bin agnosticism"), so a large multi-source, multi-bin oracle field is the sum
of the fields of disjoint groups of (source, bin) items. Each worker process regenerates the
seeded workload itself (nothing but the workload's name, arguments and source indices
crosses the process boundary), runs the unmodified oracle on its group, and returns its
FP64 partial field; the parent adds the partials in worker order, so the result does not
depend on scheduling. Workers are started with the "spawn" method: fresh interpreters that
never touch the GPU.
"""

import multiprocessing
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np


def host_workers(cap=8):
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(cap, n))


def _workload(name, kwargs):
    from paper_2511_09389_amd import inputs
    return getattr(inputs, name)(**kwargs)


def _group_bins(args):
    """Partial (B, nx, ny, nz) field of a group of (source, bin) items."""
    name, kwargs, items = args
    import oracle
    w = _workload(name, kwargs)
    scale = np.ones(1, np.float32) if w.kappa_scale is None else w.kappa_scale
    out = np.zeros((scale.size,) + w.shape)
    for b in range(scale.size):
        picks = [p for p, bb in items if bb == b]
        if not picks:
            continue
        caps = None if w.substep_cap is None else w.substep_cap[picks]
        out[b] = oracle.trace_bins(w.j_map, w.kappa_map, scale[b:b + 1], w.source_pos[picks], w.num_rays[picks],
                                   w.step_size, w.radiation_velocity, w.time_step, caps=caps)[0]
    return out


def _voxels(args):
    name, kwargs, bin_index, voxels = args
    import oracle
    w = _workload(name, kwargs)
    scale = 1.0 if w.kappa_scale is None else float(w.kappa_scale[bin_index])
    return oracle.trace_voxels(w.j_map, w.kappa_map, w.source_pos, w.num_rays, w.step_size,
                               w.radiation_velocity, w.time_step, voxels, caps=w.substep_cap,
                               kappa_scale=scale)


def _pool(n):
    return ProcessPoolExecutor(max_workers=n, mp_context=multiprocessing.get_context("spawn"))


def trace_bins_subset(name, kwargs, picks, workers=None):
    """oracle.trace_bins of workload inputs.<name>(**kwargs) restricted to sources `picks`,
    as a (B, nx, ny, nz) FP64 array. The (source, bin) items are split into groups of
    about equal work (longest first), one group per worker."""
    w = _workload(name, kwargs)
    n_bins = 1 if w.kappa_scale is None else w.kappa_scale.size
    items = [(int(p), b) for p in picks for b in range(n_bins)]
    cost = np.array([w.num_rays[p] * (w.substep_cap[p] if w.substep_cap is not None else 1) for p, _ in items],
                    dtype=np.int64)
    workers = min(host_workers() if workers is None else workers, len(items))
    groups, load = [[] for _ in range(workers)], np.zeros(workers, np.int64)
    for i in np.argsort(-cost, kind="stable"):
        g = int(np.argmin(load))
        groups[g].append(items[i])
        load[g] += cost[i]
    groups = [g for g in groups if g]
    total = None
    with _pool(len(groups)) as ex:
        for part in ex.map(_group_bins, [(name, kwargs, g) for g in groups]):
            total = part if total is None else total + part
    return total


def trace_voxels_bins(name, kwargs, voxels_per_bin, workers=None):
    """[oracle.trace_voxels of bin b at voxels_per_bin[b]] for workload inputs.<name>."""
    jobs = [(name, kwargs, b, np.asarray(v)) for b, v in enumerate(voxels_per_bin)]
    workers = min(host_workers() if workers is None else workers, len(jobs))
    with _pool(workers) as ex:
        return list(ex.map(_voxels, jobs))
