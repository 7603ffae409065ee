#!/usr/bin/env python3
"""Throughput of the emission-absorption ray march on one MI355X (gfx950).

One step is one pass of the whole hot path over one batch of synthetic input: the
multi-source, multi-bin march of Ray-trax (arXiv 2511.09389, Sec. 2: Eq. (2) per ray and
substep, loop-and-sum over sources, frequency bins as a batch axis). The default workload
is the uneven batch: a 256^3 lognormal turbulent medium (mean kappa 0.01 per cell, sigma_ln
1, k^-11/3 spectrum) with 64 Gaussian emitters and a source at each, N_Omega drawn from
{1024, 2048, 4096, 8192, 16384}, per-source substep caps U[64, 512] (c dt = 256 cells,
ds = 0.5), and 4 frequency bins with kappa_nu = kappa (nu/nu0)^-3. The step is a plan
(direction tables, workspace and the tile schedules, which depend on the source geometry
only, set up once, with the tile work-item size chosen by the autotuner) executed on the
maps and replayed as one HIP graph. Inputs are resident in HBM before the timed region; the
fields are overwritten every step.

Prints one JSON line: ray-substeps/s; the roofline position of each march kernel (average
launch durations from HIP events recorded on the launch stream, against peaks measured in
the same run by the microbenchmarks of librtmi_peaks.so, with counter-derived L2/HBM bytes
from the committed rocprofv3 summary while it matches the kernel sources); the 128^3
turbulent workload as a second key; the learned surrogate's fields/s at <= 1 % against
the plain march's; and the FP64 CPU oracle timed on this host.
"""

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ray-substeps/s per GPU + L2/atomic roofline %; surrogate fields/s at ≤1% rel L2"
HBM_PEAK_DATASHEET = 8.0e12
CUS, CLOCK_HZ = 256, 2.4e9   # MI355X compute units and peak engine clock
GATHER_BYTES = 36        # per lane-substep: 8 j corners + the nearest kappa (shared by a lane's bins)
DEPOSIT_VALUE_BYTES = 4  # per ray-substep: the recorded deposit value, written once, read back once
DEPOSITS = 8             # per ray-substep: trilinear corners
ROW_JK_BYTES = 8         # per lane-substep with the gather pass: (j, kappa) written once, read back once
COUNTER_FILES = {"uneven": "profiles/march_uneven256_counters.json",
                 "turbulent": "profiles/march_turbulent128_counters.json"}
WORKLOADS = {
    "uneven": "uneven 256^3: 64 sources, N_Omega in {1024..16384}, caps U[64,512], c dt 256, ds 0.5, "
              "4 bins with kappa (nu/nu0)^-3",
    "turbulent": "turbulent 128^3: 16 sources x 4096 rays x 256 substeps, ds 0.5",
    "blob": "uniform blob 32^3: 1 source x 256 rays x 32 substeps, ds 0.5",
    "peaks": "peaks 128^3: 2097 sources at the top 0.1% kappa voxels x 4096 rays x 256 substeps",
}
# the paper's only timing (Sec. 2): 128^3, 4,096 rays from 2,097 sources, 4.49 s on one H200
PAPER_CONTEXT = {"wall_s": 4.49, "hardware": "1x NVIDIA H200", "grid": 128, "rays": 4096,
                 "sources": 2097, "note": "substep count and JIT inclusion not stated"}


def load_workload(name):
    from paper_2511_09389_amd import inputs
    return {"uneven": inputs.uneven_bins, "turbulent": inputs.turbulent, "blob": inputs.uniform_blob,
            "peaks": inputs.peaks}[name]()


def source_substeps(w, n_s):
    caps = w.substep_cap if w.substep_cap is not None else [0] * w.n_src
    return [min(n_s, int(c)) if int(c) > 0 else n_s for c in caps]


def workload_units(w, n_s):
    """Ray-substeps of one step: sum over sources and bins of N_Omega * N_s (capped)."""
    return sum(int(nr) * ns for nr, ns in zip(w.num_rays, source_substeps(w, n_s))) * w.n_bins


class Setup:
    """Device inputs, output and a tuned plan of one workload."""

    def __init__(self, name, tune_reps=3, knobs=None):
        import torch
        from paper_2511_09389_amd import autotune, rtmi
        self.name = name
        self.w = w = load_workload(name)
        dev = torch.device("cuda:0")
        self.j = torch.from_numpy(w.j_map).to(dev)
        self.k = torch.from_numpy(w.kappa_map).to(dev)
        self.out = torch.empty((w.n_bins,) + w.shape, dtype=torch.float32, device=dev)
        self.n_s = rtmi.num_substeps(w.step_size, w.radiation_velocity, w.time_step)
        self.units = workload_units(w, self.n_s)
        for n in sorted(set(int(v) for v in w.num_rays)):
            rtmi.prepare(n)
        self.tuned, self.tune_ms = dict(autotune.DEFAULTS), {}
        if knobs:   # fixed knobs (e.g. to profile the configuration another run tuned)
            self.tuned.update({k: int(v) for k, v in knobs.items()})
        elif tune_reps > 0:
            import tempfile
            os.environ.setdefault("RTMI_TUNE_CACHE", os.path.join(tempfile.gettempdir(), "rtmi_bench_tune.json"))
            self.tuned, self.tune_ms = autotune.tune(
                self.j, self.k, w.source_pos, w.num_rays, w.step_size, w.radiation_velocity, w.time_step,
                n_bins=w.n_bins, kappa_scale=w.kappa_scale, substep_cap=w.substep_cap, reps=tune_reps)
        self.plan = rtmi.Plan(w.shape, w.source_pos, w.num_rays, w.step_size, w.radiation_velocity,
                              w.time_step, n_bins=w.n_bins, kappa_scale=w.kappa_scale,
                              substep_cap=w.substep_cap, **self.tuned)

    def execute(self):
        self.plan.execute(self.j, self.k, self.out)

    def stateless(self):
        from paper_2511_09389_amd import rtmi
        w = self.w
        rtmi.trace_bins(self.j, self.k, w.source_pos, w.num_rays, w.step_size, w.radiation_velocity,
                        w.time_step, kappa_scale=w.kappa_scale, substep_cap=w.substep_cap, out=self.out,
                        **self.tuned)

    def close(self):
        self.plan.close()


def time_graph(setup, steps, warmup):
    """Warm up, then time `steps` replays of the plan captured as one HIP graph."""
    import torch
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        setup.execute()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        setup.execute()
    for _ in range(warmup):
        graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.replay()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    del graph
    return elapsed


def time_kernels(run, steps, warmup):
    """Eager executions with the library's per-kernel HIP-event hooks (events recorded on
    each kernel's launch stream): step time and {kernel: (avg ms, launches per step)}."""
    import torch
    from paper_2511_09389_amd import rtmi
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    rtmi.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kinds = {"record": rtmi.KERNEL_RECORD, "tile": rtmi.KERNEL_TILE, "table": rtmi.KERNEL_TABLE,
             "gather_pass": rtmi.KERNEL_GATHER}
    out = {}
    for name, kind in kinds.items():
        ms, launches = rtmi.timing_read(kind)
        if launches:
            out[name] = (ms / launches, launches / steps)
    rtmi.timing_enable(False)
    return elapsed, out


def committed_counters(name, units):
    """The committed counter summary of this workload, if it was taken on the current
    kernel sources and workload; else None."""
    from paper_2511_09389_amd import counters
    path = os.path.join(ROOT, COUNTER_FILES.get(name, ""))
    try:
        with open(path) as fh:
            doc = json.load(fh)
    except (OSError, ValueError):
        return None
    if doc.get("kernel_source_hash") != counters.kernel_source_hash() or doc.get("ray_substeps_per_step") != units:
        return None
    return doc


def rooflines(setup, kern, peaks, counters_doc):
    """Per kernel: algorithmic rate against its bound's measured peak, plus the
    counter-measured L2 and HBM traffic rates against theirs (when the committed counter
    summary describes the current kernels)."""
    w, units = setup.w, setup.units
    nb_lane = min(4, w.n_bins)          # bins a record lane carries (one gather serves them all)
    out = {}
    cnt = (counters_doc or {}).get("kernels", {})
    for name, (avg_ms, per_step) in kern.items():
        t = avg_ms * 1e-3
        units_launch = units / per_step if name != "table" else 0
        r = {"avg_ms": avg_ms, "launches_per_step": per_step, "ray_substeps_per_launch": units_launch}
        if name == "record" and "gather_pass" in kern:
            # (j, kappa) rows of the gather pass read back in whole pieces, deposit values written
            read = ROW_JK_BYTES * units_launch / nb_lane
            written = DEPOSIT_VALUE_BYTES * units_launch
            r.update(bound="hbm", algorithmic_bytes=read + written,
                     frac_vs_copy_peak=(read + written) / t / peaks["copy_Bps"])
        elif name == "record":
            gathered = GATHER_BYTES * units_launch / nb_lane
            written = DEPOSIT_VALUE_BYTES * units_launch
            r.update(bound="l2", algorithmic_bytes=gathered + written,
                     gather_Bps=gathered / t, frac_gather_vs_l2_peak=gathered / t / peaks["gather_l2_Bps"],
                     frac_gather_vs_mall_peak=gathered / t / peaks["gather_mall_Bps"])
        elif name == "gather_pass":
            # the maps read once, one (j, kappa) pair written per lane-substep
            cells = int(w.j_map.size)
            moved = 8 * cells + ROW_JK_BYTES * units_launch / nb_lane
            r.update(bound="hbm", algorithmic_bytes=moved, lane_substeps_per_launch=units_launch / nb_lane,
                     frac_vs_copy_peak=moved / t / peaks["copy_Bps"])
        elif name == "tile":
            adds = DEPOSITS * units_launch
            r.update(bound="lds_atomic", algorithmic_adds=adds, adds_per_s=adds / t,
                     frac_adds_vs_lds_f64_peak=adds / t / peaks["lds_add_f64_per_s"],
                     frac_adds_vs_lds_f64_random_peak=adds / t / peaks["lds_add_f64_random_per_s"],
                     algorithmic_bytes=DEPOSIT_VALUE_BYTES * units_launch + 4 * int(w.j_map.size))
        else:
            cells = int(w.j_map.size)
            r.update(bound="hbm", algorithmic_bytes=8 * cells + 64 * cells,
                     frac_vs_copy_peak=72 * cells / t / peaks["copy_Bps"])
        c = cnt.get(name)
        if c:
            hbm = c.get("hbm_read_bytes", 0.0) + c.get("hbm_write_bytes", 0.0)
            r["counters"] = {"hbm_bytes_per_launch": hbm, "hbm_Bps": hbm / t, "frac_hbm_vs_copy_peak": hbm / t / peaks["copy_Bps"],
                             "l2_hit_rate": c.get("l2_hit_rate")}
            if "l2_read_bytes" in c:
                l2 = c["l2_read_bytes"] + c.get("l2_write_bytes", 0.0)
                r["counters"].update(l2_bytes_per_launch=l2, l2_Bps=l2 / t,
                                     frac_l2_vs_gather_l2_peak=l2 / t / peaks["gather_l2_Bps"])
            elif "l2_read_request_bytes" in c:
                l2 = c["l2_read_request_bytes"] + c.get("l2_write_request_bytes", 0.0)
                r["counters"].update(l2_request_bytes_per_launch=l2, l2_Bps=l2 / t,
                                     frac_l2_vs_gather_l2_peak=l2 / t / peaks["gather_l2_Bps"])
            sq = c.get("counters", {})
            if sq.get("SQ_INSTS_LDS_ATOMIC"):
                r["counters"]["lds_atomic_wave_instructions"] = sq["SQ_INSTS_LDS_ATOMIC"]
            if sq.get("SQ_INSTS_VALU"):
                # a SIMD issues one wave64 VALU instruction per 4 cycles (256 CUs x 4 SIMDs, 2.4 GHz)
                r["counters"]["valu_issue_frac"] = sq["SQ_INSTS_VALU"] / (CUS * 4 * CLOCK_HZ * t / 4)
            if sq.get("SQ_WAVE_CYCLES") and "SQ_WAIT_ANY" in sq:
                r["counters"]["wave_wait_frac"] = sq["SQ_WAIT_ANY"] / sq["SQ_WAVE_CYCLES"]
        out[name] = r
    return out


def contract_roofline(rl, counters_doc):
    """The roofline object for the kernel with the most time per step."""
    dom = max(rl, key=lambda k: rl[k]["avg_ms"] * rl[k]["launches_per_step"])
    r = rl[dom]
    traffic = r.get("counters", {}).get("hbm_bytes_per_launch")
    if dom == "tile":
        return {"bound": "lds_atomic", "achieved": r["adds_per_s"] / 1e9, "peak": r["adds_per_s"] / 1e9 /
                r["frac_adds_vs_lds_f64_peak"], "unit": "G LDS f64 adds/s", "frac": r["frac_adds_vs_lds_f64_peak"],
                "traffic": traffic, "kernel": dom, "kernel_avg_ms": r["avg_ms"],
                "units_per_launch": r["ray_substeps_per_launch"], "per_unit": f"{DEPOSITS} deposits",
                "frac_vs_random_address_peak": r["frac_adds_vs_lds_f64_random_peak"]}
    if dom == "record" and "gather_Bps" in r:
        return {"bound": "l2", "achieved": r["gather_Bps"] / 1e9, "peak": r["gather_Bps"] / 1e9 /
                r["frac_gather_vs_l2_peak"], "unit": "GB/s", "frac": r["frac_gather_vs_l2_peak"],
                "traffic": traffic, "kernel": dom, "kernel_avg_ms": r["avg_ms"],
                "units_per_launch": r["ray_substeps_per_launch"], "per_unit": f"{GATHER_BYTES} B per lane-substep"}
    return {"bound": "hbm", "achieved": r["algorithmic_bytes"] / (r["avg_ms"] * 1e-3) / 1e9,
            "peak": HBM_PEAK_DATASHEET / 1e9, "unit": "GB/s",
            "frac": r["algorithmic_bytes"] / (r["avg_ms"] * 1e-3) / HBM_PEAK_DATASHEET, "traffic": traffic,
            "kernel": dom, "kernel_avg_ms": r["avg_ms"], "frac_vs_measured_copy": r.get("frac_vs_copy_peak")}


def measure(name, steps, warmup, peaks, tune_reps=3, knobs=None):
    import torch
    s = Setup(name, tune_reps=tune_reps, knobs=knobs)
    elapsed = time_graph(s, steps, warmup)
    eager_elapsed, kern = time_kernels(s.execute, steps, warmup)
    stateless_elapsed, _ = time_kernels(s.stateless, steps, warmup)
    counters_doc = committed_counters(name, s.units)
    rl = rooflines(s, kern, peaks, counters_doc)
    res = {"workload": WORKLOADS[name], "grid": list(s.w.shape), "sources": s.w.n_src,
           "rays_per_source": sorted(set(int(v) for v in s.w.num_rays)), "bins": s.w.n_bins,
           "ray_substeps_per_step": s.units, "value": s.units * steps / elapsed,
           "ms_per_step": 1e3 * elapsed / steps,
           "eager_plan_ms_per_step": 1e3 * eager_elapsed / steps,
           "stateless_ms_per_step": 1e3 * stateless_elapsed / steps,
           "stateless_value": s.units * steps / stateless_elapsed,
           "tuned": s.tuned, "autotune_ms": {str(c): round(t, 4) for c, t in s.tune_ms.items()},
           "kernels": rl, "counters_file": COUNTER_FILES.get(name) if counters_doc else None,
           "roofline": contract_roofline(rl, counters_doc)}
    s.close()
    del s
    torch.cuda.empty_cache()
    return res


def surrogate_rates(n_train=300, n_val=30, n_eval=30):
    """The learned surrogate with the march as fallback (64^3 turbulent samples, 16 sources x
    4096 rays, 128 substeps): a short training on the GPU by the library's kernels, the 1 %
    calibration, then fields/s of the surrogate path (with its fallbacks), of the network's
    own path and of the plain march, and how many fields the surrogate itself returned."""
    import torch
    from paper_2511_09389_amd import surrogate as sg
    dev = torch.device("cuda:0")
    cd = 4
    train = [sg.make_sample(s, dev, cheap_divisor=cd) for s in range(n_train)]
    val = [sg.make_sample(5000 + s, dev, cheap_divisor=cd) for s in range(n_val)]
    ev = [sg.make_sample(10000 + s, dev, cheap_divisor=cd) for s in range(n_eval)]
    model, losses = sg.train(train, dev, epochs=6, lr=2e-3, batch=4, warmup=20, schedule="cosine",
                             cheap_divisor=cd)
    thr, pairs = sg.calibrate(model, val, target=0.01)
    res = sg.evaluate(model, ev)
    errs = sorted(p[1] for p in pairs)
    out = {"metric": "fields/s at <= 1% rel L2 (surrogate with fallback) vs the plain march",
           "surrogate_fields_per_s": res["surrogate_fields_per_s"], "plain_fields_per_s": res["march_fields_per_s"],
           "network_path_fields_per_s": res["network_path_fields_per_s"], "accepted": res["accepted"],
           "samples": res["samples"], "max_returned_error": res["max_err"], "threshold": thr,
           "validation_error_median": errs[len(errs) // 2], "validation_error_best": errs[0],
           "training": f"{n_train} samples, 6 epochs, batch 4, cheap march N_Omega/{cd}",
           "note": "a short training inside the benchmark; the 2000-sample runs are summarised in "
                   "profiles/surrogate_c5_64_training.md",
           "conv_kernels_64": sg.conv_rates(dev)}
    del train, val, ev
    torch.cuda.empty_cache()
    return out


def cpu_info():
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}


CPU_SECONDS_PER_CLASS = 2.5


def cpu_baseline(name):
    """The FP64 oracle as it stands, one process, on this host. The uneven workload is
    sampled: per N_Omega class, whole sources of that class (bin 0) until about
    CPU_SECONDS_PER_CLASS seconds of oracle time, extrapolated linearly in ray-substeps (per
    class) to every source and bin (the bins differ only in kappa's scale, which costs
    nothing); the 32^3 blob runs in full."""
    import numpy as np
    import oracle
    w = load_workload(name)
    from paper_2511_09389_amd import rtmi
    n_s = rtmi.num_substeps(w.step_size, w.radiation_velocity, w.time_step)
    subs = source_substeps(w, n_s)
    caps = w.substep_cap if w.substep_cap is not None else np.zeros(w.n_src, np.int32)
    rate_by_rays = {}
    sampled_work, sampled_s = 0, 0.0
    n_sampled = 0
    for nr in sorted(set(int(v) for v in w.num_rays)):
        work, spent = 0, 0.0
        for s in (i for i in range(w.n_src) if int(w.num_rays[i]) == nr):
            t0 = time.perf_counter()
            oracle.trace_single(w.j_map, w.kappa_map, w.source_pos[s], nr, w.step_size, w.radiation_velocity,
                                w.time_step, cap=int(caps[s]))
            spent += time.perf_counter() - t0
            work += nr * subs[s]
            n_sampled += 1
            if spent >= CPU_SECONDS_PER_CLASS:
                break
        rate_by_rays[nr] = work / spent
        sampled_work += work
        sampled_s += spent
    total_s = sum(int(nr) * ns / rate_by_rays[int(nr)] for nr, ns in zip(w.num_rays, subs)) * w.n_bins
    units = workload_units(w, n_s)
    exact = n_sampled == w.n_src and w.n_bins == 1
    blob = load_workload("blob")
    t0, reps = time.perf_counter(), 0
    while time.perf_counter() - t0 < 1.0:
        oracle.trace_single(blob.j_map, blob.kappa_map, blob.source_pos[0], int(blob.num_rays[0]), blob.step_size,
                            blob.radiation_velocity, blob.time_step)
        reps += 1
    blob_rate = reps * int(blob.num_rays[0]) * rtmi.num_substeps(blob.step_size, blob.radiation_velocity,
                                                                  blob.time_step) / (time.perf_counter() - t0)
    return dict({"value": units / total_s, "unit": "ray-substeps/s", "cores": 1, "kind": "oracle",
                 "sample": (f"{'full workload' if exact else 'extrapolated'}: {n_sampled} whole sources over the "
                            f"N_Omega classes {sorted(rate_by_rays)} (about {CPU_SECONDS_PER_CLASS:g} s each), bin 0, "
                            f"{sampled_work} ray-substeps in {sampled_s:.1f} s, "
                            f"scaled per class to all {w.n_src} sources x {w.n_bins} bins "
                            f"({units} ray-substeps, {total_s:.0f} s estimated); NumPy FP64, one process "
                            f"(elementwise NumPy runs on one thread)"),
                 "blob32_full_value": blob_rate}, **cpu_info())


def counters_run(name, known_out, executions=2, knobs=None):
    """A short run for rocprofv3 counter passes and kernel traces: a few plan executions of
    the workload (default or given knobs), then the calibration kernels of known size
    (device copy, L2-resident line gather)."""
    import torch
    from paper_2511_09389_amd import peaks
    s = Setup(name, tune_reps=0, knobs=knobs)
    for _ in range(executions):
        s.execute()
    torch.cuda.synchronize()
    s.close()
    copy_bytes = 256 << 20
    _, moved = peaks.copy(copy_bytes, reps=1)
    _, gathered = peaks.gather(2 << 20, iters=64, reps=1)
    known = {"copy_read_bytes": moved / 2, "copy_write_bytes": moved / 2, "gather_bytes": gathered,
             "ray_substeps_per_step": s.units, "executions": executions}
    os.makedirs(os.path.dirname(known_out) or ".", exist_ok=True)
    with open(known_out, "w") as fh:
        json.dump(known, fh)
    print(json.dumps(known), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="uneven")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-second", action="store_true", help="skip the 128^3 turbulent key")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate fields/s key")
    ap.add_argument("--counters-run", metavar="KNOWN_JSON", default=None,
                    help="only run a short profiling sequence (for rocprofv3 --pmc passes)")
    ap.add_argument("--executions", type=int, default=2, help="plan executions of --counters-run")
    ap.add_argument("--knobs", default=None,
                    help='fixed plan knobs instead of the autotuner, as JSON (e.g. \'{"tile_item_chunks": 2048}\')')
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (a source-sharded "
              "version would give each GPU a share of the sources and sum the partial fields with one "
              "all-reduce)", file=sys.stderr)
        sys.exit(2)
    knobs = json.loads(args.knobs) if args.knobs else None
    if args.counters_run:
        counters_run(args.workload, args.counters_run, args.executions, knobs)
        return

    from paper_2511_09389_amd import peaks as peaks_lib
    print("[bench] peak microbenchmarks", file=sys.stderr, flush=True)
    peaks = peaks_lib.measure_all()
    print(f"[bench] {args.workload}: plan + graph, {args.warmup} warm-up and {args.steps} timed steps",
          file=sys.stderr, flush=True)
    main_res = measure(args.workload, args.steps, args.warmup, peaks, knobs=knobs)
    second = None
    if args.workload == "uneven" and not args.no_second:
        print("[bench] turbulent 128^3 as the second key", file=sys.stderr, flush=True)
        second = measure("turbulent", max(args.steps, 20), args.warmup, peaks)
    result = {
        "metric": METRIC, "value": main_res["value"], "unit": "ray-substeps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": main_res["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": main_res["workload"], "grid": main_res["grid"], "sources": main_res["sources"],
                   "rays_per_source": main_res["rays_per_source"], "bins": main_res["bins"],
                   "ray_substeps_per_step": main_res["ray_substeps_per_step"],
                   "execution": "plan (geometry set up once, knobs autotuned) replayed as one HIP graph"},
        "roofline": main_res["roofline"],
        "detail": {k: v for k, v in main_res.items() if k not in ("roofline",)},
        "peaks_measured": peaks,
    }
    if second:
        result["turbulent_128"] = second
    if args.workload == "peaks":
        result["paper_context"] = dict(PAPER_CONTEXT, this_run_s=main_res["ms_per_step"] / 1e3)
    if not args.no_surrogate:
        print("[bench] surrogate (short training, calibration, evaluation)", file=sys.stderr, flush=True)
        result["surrogate"] = surrogate_rates()
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
