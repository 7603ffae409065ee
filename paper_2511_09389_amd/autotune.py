"""Autotuner for the tile schedule of a plan.

The tile kernel splits each 16^3 output tile into work items of about `tile_item_chunks`
ray chunks; the best size depends on the grid, the sources and the device. tune_item_chunks
times each candidate on the device with the caller's maps (plans built once, executions
timed with HIP events on the current stream) and keeps the fastest per workload signature
in a JSON cache, so later plans of the same shape skip the search.
"""

import hashlib
import json
import os

import numpy as np
import torch

from . import rtmi

CANDIDATES = (512, 768, 1024, 1536, 2048, 3072)


def cache_path():
    return os.environ.get("RTMI_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "rtmi", "tune.json"))


def signature(grid, source_pos, num_rays, substep_cap, n_substeps, n_bins, device):
    """Key of a workload: device, library version, grid, bins, N_s and the multisets of
    per-source ray counts and caps, with source positions rounded to whole tiles."""
    src = np.asarray(source_pos, np.float64).reshape(-1, 3)
    nr = np.broadcast_to(np.asarray(num_rays, np.int64), (src.shape[0],))
    caps = np.zeros(src.shape[0], np.int64) if substep_cap is None else \
        np.broadcast_to(np.asarray(substep_cap, np.int64), (src.shape[0],))
    h = hashlib.sha256()
    h.update(np.floor(src / 16.0).astype(np.int64).tobytes())
    desc = {"device": torch.cuda.get_device_name(device), "version": rtmi.version(),
            "grid": list(map(int, grid)), "bins": int(n_bins), "n_s": int(n_substeps),
            "rays": sorted(map(int, nr)), "caps": sorted(map(int, caps)), "tiles": h.hexdigest()[:16]}
    return hashlib.sha256(json.dumps(desc, sort_keys=True).encode()).hexdigest()[:24]


def _load_cache(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _save_cache(path, data):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_plan(plan, j_maps, kappa_maps, out, reps=5, warmup=1):
    """Mean milliseconds per execution (HIP events on the current stream)."""
    for _ in range(warmup):
        plan.execute(j_maps, kappa_maps, out)
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        plan.execute(j_maps, kappa_maps, out)
    end.record()
    end.synchronize()
    return start.elapsed_time(end) / reps


def tune_item_chunks(j_maps, kappa_maps, source_pos, num_rays, step_size, radiation_velocity,
                     time_step, n_bins=1, kappa_scale=None, substep_cap=None,
                     candidates=CANDIDATES, reps=5, use_cache=True, **plan_kw):
    """Return (best tile_item_chunks, {candidate: ms}) for this workload; the timings are
    empty when the answer came from the cache."""
    grid = tuple(j_maps.shape[-3:])
    n_s = rtmi.num_substeps(step_size, radiation_velocity, time_step)
    key = signature(grid, source_pos, num_rays, substep_cap, n_s, n_bins, j_maps.device)
    path = cache_path()
    cache = _load_cache(path) if use_cache else {}
    if key in cache:
        return int(cache[key]["tile_item_chunks"]), {}
    per_bin_j = j_maps.dim() == 4 and n_bins > 1
    per_bin_k = kappa_maps.dim() == 4 and n_bins > 1
    out = torch.empty((n_bins,) + grid, dtype=torch.float32, device=j_maps.device)
    timings = {}
    for c in candidates:
        plan = rtmi.Plan(grid, source_pos, num_rays, step_size, radiation_velocity, time_step,
                         n_bins=n_bins, kappa_scale=kappa_scale, per_bin_j=per_bin_j,
                         per_bin_kappa=per_bin_k, substep_cap=substep_cap, tile_item_chunks=c,
                         device=j_maps.device, **plan_kw)
        timings[int(c)] = time_plan(plan, j_maps, kappa_maps, out, reps=reps)
        plan.close()
    best = min(timings, key=timings.get)
    if use_cache:
        cache = _load_cache(path)
        cache[key] = {"tile_item_chunks": best, "ms": timings[best]}
        _save_cache(path, cache)
    return best, timings


def tuned_plan(j_maps, kappa_maps, source_pos, num_rays, step_size, radiation_velocity,
               time_step, n_bins=1, kappa_scale=None, substep_cap=None, **plan_kw):
    """A Plan with the tuned work-item size (searched once per workload signature)."""
    best, _ = tune_item_chunks(j_maps, kappa_maps, source_pos, num_rays, step_size,
                               radiation_velocity, time_step, n_bins=n_bins,
                               kappa_scale=kappa_scale, substep_cap=substep_cap, **plan_kw)
    grid = tuple(j_maps.shape[-3:])
    return rtmi.Plan(grid, source_pos, num_rays, step_size, radiation_velocity, time_step,
                     n_bins=n_bins, kappa_scale=kappa_scale,
                     per_bin_j=j_maps.dim() == 4 and n_bins > 1,
                     per_bin_kappa=kappa_maps.dim() == 4 and n_bins > 1,
                     substep_cap=substep_cap, tile_item_chunks=best, device=j_maps.device,
                     **plan_kw)
