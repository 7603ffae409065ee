"""Autotuner for the tiled march of a plan.

The best launch shape depends on the grid, the sources and the device. `tune` times
candidate settings of four knobs on the device with the caller's maps (plans built once per
candidate, executions timed with HIP events on the current stream) and keeps the fastest
per workload signature in a JSON cache, so later plans of the same shape skip the search:

* tile_item_chunks: the tile work-item size (chunk records per item); a 16^3 output tile
  with C chunks is split into ceil(C / size) items that separate work-groups take;
* tile_groups_per_cu: resident work-groups of the persistent tile pass per compute unit
  (0 = as many as fit; fewer trade latency hiding for L2 and LDS pressure);
* gather_table: where the record pass gets j and kappa (0: the library's choice by grid
  size, 1: the per-call 64-byte table, 3: the rows of the gather pass, 2: the maps);
* sources_per_launch: all sources in one record launch (0) or in groups of a cap.

The search is coordinate descent from the defaults, one knob at a time, in that order.
The launch-shape knobs do not change the field (in the deterministic mode, not a bit of
it); the gather source changes it by rounding only.
"""

import hashlib
import json
import os

import numpy as np
import torch

from . import rtmi

CANDIDATES = (512, 768, 1024, 1536, 2048, 3072, 4096, 6144, 8192)
GROUPS_PER_CU = (0, 2, 1)
GATHER_TABLE = (0, 1, 3, 2)
SOURCES_PER_LAUNCH = (0, 32)
DEFAULTS = {"tile_item_chunks": 1024, "tile_groups_per_cu": 0, "gather_table": 0, "sources_per_launch": 0}


def cache_path():
    return os.environ.get("RTMI_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "rtmi", "tune.json"))


def signature(grid, source_pos, num_rays, substep_cap, n_substeps, n_bins, device, what="knobs"):
    """Key of a workload: device, library version, grid, bins, N_s and the multisets of
    per-source ray counts and caps, with source positions rounded to whole tiles."""
    src = np.asarray(source_pos, np.float64).reshape(-1, 3)
    nr = np.broadcast_to(np.asarray(num_rays, np.int64), (src.shape[0],))
    caps = np.zeros(src.shape[0], np.int64) if substep_cap is None else \
        np.broadcast_to(np.asarray(substep_cap, np.int64), (src.shape[0],))
    h = hashlib.sha256()
    h.update(np.floor(src / 16.0).astype(np.int64).tobytes())
    desc = {"device": torch.cuda.get_device_name(device), "version": rtmi.version(), "what": what,
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


def _time_knobs(knobs, j_maps, kappa_maps, source_pos, num_rays, step_size, radiation_velocity, time_step,
                n_bins, kappa_scale, substep_cap, reps, out, plan_kw):
    grid = tuple(j_maps.shape[-3:])
    plan = rtmi.Plan(grid, source_pos, num_rays, step_size, radiation_velocity, time_step,
                     n_bins=n_bins, kappa_scale=kappa_scale, per_bin_j=j_maps.dim() == 4 and n_bins > 1,
                     per_bin_kappa=kappa_maps.dim() == 4 and n_bins > 1, substep_cap=substep_cap,
                     device=j_maps.device, **knobs, **plan_kw)
    try:
        return time_plan(plan, j_maps, kappa_maps, out, reps=reps)
    finally:
        plan.close()


def tune(j_maps, kappa_maps, source_pos, num_rays, step_size, radiation_velocity, time_step,
         n_bins=1, kappa_scale=None, substep_cap=None, reps=5, use_cache=True,
         candidates=None, **plan_kw):
    """Return (best knobs as a dict of Plan keyword arguments, {description: ms}) for this
    workload; the timings are empty when the answer came from the cache. `candidates`
    maps a knob to the values to try (defaults: the module's lists)."""
    grid = tuple(j_maps.shape[-3:])
    n_s = rtmi.num_substeps(step_size, radiation_velocity, time_step)
    key = signature(grid, source_pos, num_rays, substep_cap, n_s, n_bins, j_maps.device)
    path = cache_path()
    if use_cache:
        cache = _load_cache(path)
        if key in cache:
            return {k: int(cache[key][k]) for k in DEFAULTS}, {}
    shared = j_maps.dim() == 3 and kappa_maps.dim() == 3
    n_src = np.asarray(source_pos).reshape(-1, 3).shape[0]
    space = {"tile_item_chunks": CANDIDATES, "tile_groups_per_cu": GROUPS_PER_CU,
             "gather_table": GATHER_TABLE if shared else (0,),
             "sources_per_launch": SOURCES_PER_LAUNCH if n_src > 32 else (0,)}
    space.update(candidates or {})
    out = torch.empty((n_bins,) + grid, dtype=torch.float32, device=j_maps.device)
    best = dict(DEFAULTS)
    timings = {}
    best_ms = None
    for knob in ("tile_item_chunks", "tile_groups_per_cu", "gather_table", "sources_per_launch"):
        for v in space[knob]:
            trial = dict(best, **{knob: int(v)})
            desc = ",".join(f"{k}={trial[k]}" for k in DEFAULTS)
            if desc not in timings:
                timings[desc] = _time_knobs(trial, j_maps, kappa_maps, source_pos, num_rays, step_size,
                                            radiation_velocity, time_step, n_bins, kappa_scale, substep_cap,
                                            reps, out, plan_kw)
            if best_ms is None or timings[desc] < best_ms:
                best_ms, best = timings[desc], trial
    if use_cache:
        cache = _load_cache(path)
        cache[key] = dict(best, ms=best_ms)
        _save_cache(path, cache)
    return best, timings


def tune_item_chunks(j_maps, kappa_maps, source_pos, num_rays, step_size, radiation_velocity,
                     time_step, n_bins=1, kappa_scale=None, substep_cap=None,
                     candidates=CANDIDATES, reps=5, use_cache=True, **plan_kw):
    """Return (best tile_item_chunks, {candidate: ms}), searching that knob alone (the
    others at their defaults); the timings are empty when the answer came from the cache."""
    grid = tuple(j_maps.shape[-3:])
    n_s = rtmi.num_substeps(step_size, radiation_velocity, time_step)
    key = signature(grid, source_pos, num_rays, substep_cap, n_s, n_bins, j_maps.device, what="item_chunks")
    path = cache_path()
    cache = _load_cache(path) if use_cache else {}
    if key in cache:
        return int(cache[key]["tile_item_chunks"]), {}
    out = torch.empty((n_bins,) + grid, dtype=torch.float32, device=j_maps.device)
    timings = {}
    for c in candidates:
        timings[int(c)] = _time_knobs({"tile_item_chunks": int(c)}, j_maps, kappa_maps, source_pos, num_rays,
                                      step_size, radiation_velocity, time_step, n_bins, kappa_scale,
                                      substep_cap, reps, out, plan_kw)
    best = min(timings, key=timings.get)
    if use_cache:
        cache = _load_cache(path)
        cache[key] = {"tile_item_chunks": best, "ms": timings[best]}
        _save_cache(path, cache)
    return best, timings


def tuned_plan(j_maps, kappa_maps, source_pos, num_rays, step_size, radiation_velocity,
               time_step, n_bins=1, kappa_scale=None, substep_cap=None, **plan_kw):
    """A Plan with the tuned knobs (searched once per workload signature)."""
    best, _ = tune(j_maps, kappa_maps, source_pos, num_rays, step_size, radiation_velocity, time_step,
                   n_bins=n_bins, kappa_scale=kappa_scale, substep_cap=substep_cap, **plan_kw)
    grid = tuple(j_maps.shape[-3:])
    return rtmi.Plan(grid, source_pos, num_rays, step_size, radiation_velocity, time_step,
                     n_bins=n_bins, kappa_scale=kappa_scale,
                     per_bin_j=j_maps.dim() == 4 and n_bins > 1,
                     per_bin_kappa=kappa_maps.dim() == 4 and n_bins > 1,
                     substep_cap=substep_cap, device=j_maps.device, **best, **plan_kw)
