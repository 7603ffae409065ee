#!/usr/bin/env python3
"""Throughput of the emission-absorption ray march on one MI355X (gfx950).

One step is one pass of the whole hot path over one batch of synthetic input: the
multi-source march of Ray-trax (arXiv 2511.09389, Sec. 2) on a 128^3 lognormal turbulent
medium (mean kappa 0.02 per cell, sigma_ln 1, k^-11/3 spectrum) with 16 Gaussian emitters
and a source at each, 4096 Fibonacci rays per source, ds = 0.5 cell, c dt = 128 cells
(N_s = 256): 16 * 4096 * 256 = 16,777,216 ray-substeps per step. Inputs are resident in
HBM before the timed region starts; the output field is overwritten every step.

Prints one JSON line: ray-substeps/s, the roofline position of the march kernel (its
average duration measured with HIP events recorded on its own launch stream during the
timed region) and the FP64 CPU oracle timed on this host as a baseline.
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ray-substeps/s per GPU + L2/atomic roofline %; surrogate fields/s at ≤1% rel L2"
HBM_PEAK = 8.0e12                 # MI355X HBM3E, bytes/s
# Algorithmic bytes per ray-substep of each kernel of the tiled path:
#   record: 8 j corners + 1 kappa gathered (36 B) + the deposit value written (4 B)
#   tile:   the deposit value read back (4 B); the field itself (4 B per voxel) is added per launch
BYTES_PER_UNIT = {"record": 40, "tile": 4}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "march_turbulent128_traffic.json")
KERNEL_SOURCES = ["paper_2511_09389_amd/csrc/tiled.hip", "paper_2511_09389_amd/csrc/common.h",
                  "paper_2511_09389_amd/csrc/device_common.h"]


def kernel_source_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, per_launch_units):
    """HBM bytes per launch of `kernel` from the committed counter summary, if it was taken
    on the current kernel source and workload; otherwise None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    if t.get("ray_substeps_per_launch") != per_launch_units:
        return None
    return t.get("hbm_bytes_per_launch", {}).get(kernel)


def workload_units(w, n_s):
    """Ray-substeps of one step: sum over sources and bins of N_Omega * N_s (capped)."""
    caps = w.substep_cap if w.substep_cap is not None else [0] * w.n_src
    total = 0
    for nr, cap in zip(w.num_rays, caps):
        total += int(nr) * (min(n_s, int(cap)) if int(cap) > 0 else n_s)
    return total * w.n_bins


def cpu_baseline(w, n_s, budget_s=20.0):
    """The FP64 oracle, as it stands, on the workload's sources in order until about
    budget_s of CPU time is spent (the whole workload when it fits), one core."""
    import numpy as np
    import oracle
    caps = w.substep_cap if w.substep_cap is not None else np.zeros(w.n_src, np.int32)
    scale = w.kappa_scale if w.kappa_scale is not None else np.ones(1, np.float32)
    t0 = time.perf_counter()
    done, work = 0, 0
    while done < w.n_src and time.perf_counter() - t0 < budget_s:
        for b in range(len(scale)):
            oracle.trace_single(w.j_map, w.kappa_map.astype(np.float64) * float(scale[b]),
                                w.source_pos[done], int(w.num_rays[done]), w.step_size,
                                w.radiation_velocity, w.time_step, cap=int(caps[done]))
        cap = int(caps[done])
        work += int(w.num_rays[done]) * (min(n_s, cap) if cap > 0 else n_s) * len(scale)
        done += 1
    dt = time.perf_counter() - t0
    what = "full workload" if done == w.n_src else f"first {done} of {w.n_src} sources"
    return {"value": work / dt, "unit": "ray-substeps/s", "cores": 1, "kind": "oracle",
            "sample": f"{what}, all bins: {work} ray-substeps in {dt:.2f} s, NumPy FP64, "
                      f"single process"}


WORKLOADS = {
    "turbulent": "turbulent 128^3, 16 sources x 4096 rays x 256 substeps",
    "uneven": "uneven 256^3, 64 sources, N_Omega in {1024..16384}, caps U[64,512], 4 bins",
    "peaks": "peaks 128^3, 2097 sources at the top 0.1% kappa voxels x 4096 rays x 256 substeps",
}
# the paper's only timing (Sec. 2): 128^3, 4,096 rays from 2,097 sources, 4.49 s on one H200
PAPER_CONTEXT = {"wall_s": 4.49, "hardware": "1x NVIDIA H200", "grid": 128, "rays": 4096,
                 "sources": 2097, "note": "substep count and JIT inclusion not stated"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="turbulent")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="also run device copies of this many bytes (counter calibration only)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the design of the source-sharded version is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2511_09389_amd import inputs, rtmi

    w = {"turbulent": inputs.turbulent, "uneven": inputs.uneven_bins, "peaks": inputs.peaks}[args.workload]()
    dev = torch.device("cuda:0")
    j = torch.from_numpy(w.j_map).to(dev)
    kap = torch.from_numpy(w.kappa_map).to(dev)
    out = torch.empty((w.n_bins,) + w.shape, dtype=torch.float32, device=dev)
    n_s = rtmi.num_substeps(w.step_size, w.radiation_velocity, w.time_step)
    units = workload_units(w, n_s)
    for n in sorted(set(int(v) for v in w.num_rays)):
        rtmi.prepare(n)

    def step():
        if w.n_bins == 1 and w.substep_cap is None:
            rtmi.trace_multi(j, kap, w.source_pos, w.num_rays, w.step_size, w.radiation_velocity,
                             w.time_step, out=out[0])
        else:
            rtmi.trace_bins(j, kap, w.source_pos, w.num_rays, w.step_size, w.radiation_velocity,
                            w.time_step, kappa_scale=w.kappa_scale, substep_cap=w.substep_cap,
                            out=out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    rtmi.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timed = {name: rtmi.timing_read(kind) for name, kind in
             (("record", rtmi.KERNEL_RECORD), ("tile", rtmi.KERNEL_TILE))}
    rtmi.timing_enable(False)

    # The same step as a plan (geometry set up once, outside the timing, with the tile
    # work-item size picked by the autotuner) captured in one HIP graph and replayed: what
    # a time-stepping caller with fixed sources runs.
    import tempfile
    from paper_2511_09389_amd import autotune
    os.environ.setdefault("RTMI_TUNE_CACHE", os.path.join(tempfile.gettempdir(), "rtmi_bench_tune.json"))
    best_chunks, tune_ms = autotune.tune_item_chunks(j, kap, w.source_pos, w.num_rays, w.step_size,
                                                     w.radiation_velocity, w.time_step, n_bins=w.n_bins,
                                                     kappa_scale=w.kappa_scale, substep_cap=w.substep_cap,
                                                     reps=3)
    plan = rtmi.Plan(w.shape, w.source_pos, w.num_rays, w.step_size, w.radiation_velocity,
                     w.time_step, n_bins=w.n_bins, kappa_scale=w.kappa_scale,
                     substep_cap=w.substep_cap, tile_item_chunks=best_chunks)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.execute(j, kap, out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.execute(j, kap, out)
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    g0 = time.perf_counter()
    for _ in range(args.steps):
        graph.replay()
    torch.cuda.synchronize()
    g1 = time.perf_counter()
    plan_graph = {"ms_per_step": 1e3 * (g1 - g0) / args.steps, "value": units * args.steps / (g1 - g0),
                  "tile_item_chunks": best_chunks,
                  "autotune_ms": {str(c): round(t, 4) for c, t in tune_ms.items()},
                  "note": "plan made once (tables, workspace, tile schedules and chunk records), step replayed as one graph"}
    del graph
    plan.close()

    if args.copy_bytes > 0:
        src = torch.empty(args.copy_bytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()

    elapsed = t1 - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = units * args.steps / elapsed
    cells = int(np.prod(w.shape))
    kernels = {}
    for name, (ms, launches) in timed.items():
        avg_s = (ms / max(launches, 1)) * 1e-3
        per_launch_units = units * args.steps // max(launches, 1)   # launches split the sources
        algo_bytes = BYTES_PER_UNIT[name] * per_launch_units + (4 * cells * w.n_bins if name == "tile" else 0)
        kernels[name] = {"avg_ms": avg_s * 1e3, "launches": launches,
                         "units_per_launch": per_launch_units, "algorithmic_bytes": algo_bytes,
                         "achieved_GBps": algo_bytes / avg_s / 1e9 if avg_s > 0 else None}
    dom = max(kernels, key=lambda k: kernels[k]["avg_ms"])
    kd = kernels[dom]
    achieved = kd["algorithmic_bytes"] / (kd["avg_ms"] * 1e-3)
    roofline = {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "frac": achieved / HBM_PEAK, "traffic": measured_traffic(dom, kd["units_per_launch"]),
                "kernel": dom, "kernel_avg_ms": kd["avg_ms"], "launches": kd["launches"],
                "bytes_per_unit": BYTES_PER_UNIT[dom], "units_per_launch": kd["units_per_launch"],
                "kernels": kernels}

    result = {
        "metric": METRIC, "value": value, "unit": "ray-substeps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "grid": list(w.shape), "sources": w.n_src,
                   "rays_per_source": sorted(set(int(v) for v in w.num_rays)), "substeps": n_s,
                   "bins": w.n_bins, "step_size": w.step_size, "ray_substeps_per_step": units},
        "roofline": roofline,
        "plan_graph": plan_graph,
    }
    if args.workload == "peaks":
        result["paper_context"] = dict(PAPER_CONTEXT, this_run_s=elapsed / args.steps)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(w, n_s)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
