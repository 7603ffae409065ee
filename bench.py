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
BYTES_PER_RAY_SUBSTEP = 68        # 8 j corners + 1 kappa gathered (36 B) + 8 FP32 deposits (32 B)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "march_turbulent128_traffic.json")
KERNEL_SOURCES = ["paper_2511_09389_amd/csrc/march.hip", "paper_2511_09389_amd/csrc/common.h"]


def kernel_source_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(per_launch_units):
    """HBM bytes per launch from the committed counter summary, if it was taken on the
    current kernel source; otherwise None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    if t.get("ray_substeps_per_launch") != per_launch_units:
        return None
    return t.get("hbm_bytes_per_launch")


def cpu_baseline(w):
    """The FP64 oracle, as it stands, on the whole workload (all 16 sources), one core."""
    import numpy as np  # noqa: F401
    import oracle
    t0 = time.perf_counter()
    oracle.trace_multi(w.j_map, w.kappa_map, w.source_pos, w.num_rays, w.step_size,
                       w.radiation_velocity, w.time_step)
    dt = time.perf_counter() - t0
    work = int(sum(int(n) for n in w.num_rays)) * 256
    return {"value": work / dt, "unit": "ray-substeps/s", "cores": 1, "kind": "oracle",
            "sample": f"full workload: 16 sources x 4096 rays x 256 substeps ({work} ray-substeps) "
                      f"in {dt:.2f} s, NumPy FP64, single process"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
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

    w = inputs.turbulent()
    dev = torch.device("cuda:0")
    j = torch.from_numpy(w.j_map).to(dev)
    kap = torch.from_numpy(w.kappa_map).to(dev)
    out = torch.empty(w.shape, dtype=torch.float32, device=dev)
    n_s = rtmi.num_substeps(w.step_size, w.radiation_velocity, w.time_step)
    units = int(np.sum(w.num_rays.astype(np.int64))) * n_s
    rtmi.prepare(int(w.num_rays[0]))

    def step():
        rtmi.trace_multi(j, kap, w.source_pos, w.num_rays, w.step_size, w.radiation_velocity,
                         w.time_step, out=out)

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
    kernel_ms, launches = rtmi.timing_read()
    rtmi.timing_enable(False)

    if args.copy_bytes > 0:
        src = torch.empty(args.copy_bytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()

    elapsed = t1 - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = units * args.steps / elapsed
    avg_kernel_s = (kernel_ms / launches) * 1e-3
    per_launch_units = units * args.steps // max(launches, 1)
    achieved = BYTES_PER_RAY_SUBSTEP * per_launch_units / avg_kernel_s
    roofline = {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "frac": achieved / HBM_PEAK, "traffic": measured_traffic(per_launch_units),
                "kernel": "march_kernel", "kernel_avg_ms": avg_kernel_s * 1e3,
                "launches": launches, "bytes_per_unit": BYTES_PER_RAY_SUBSTEP,
                "units_per_launch": per_launch_units}

    result = {
        "metric": METRIC, "value": value, "unit": "ray-substeps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "turbulent 128^3, 16 sources x 4096 rays x 256 substeps",
                   "grid": list(w.shape), "sources": w.n_src, "rays_per_source": int(w.num_rays[0]),
                   "substeps": n_s, "step_size": w.step_size, "ray_substeps_per_step": units},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
