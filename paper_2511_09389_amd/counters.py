"""Reduce rocprofv3 hardware-counter runs of the march into one JSON summary.

Usage (after one `rocprofv3 --pmc ... --output-format csv -d DIR/passN -- python3 bench.py
--counters-run ...` per counter pass):

    python -m paper_2511_09389_amd.counters OUT.json DIR/pass1 DIR/pass2 ... \
        --workload NAME --command "the profiling command"

Per kernel of the march (record, tile, gather table) and of the calibration kernels the
counter run also launches (a device copy and an L2-resident line gather of known size), it
averages every counter over that kernel's dispatches. HBM bytes come from FETCH_SIZE and
WRITE_SIZE (KiB per dispatch), each scaled by the factor that makes the copy kernel's
counter read the bytes it is known to move. L2 bytes are the 32-byte sectors the L2
(TCC) reads and writes; L2 request bytes are TCP->TCC requests times 64 bytes (a request
carries 64 or 128 bytes, so this undercounts coalesced traffic; the copy and gather
kernels of known size show by how much). The summary records the hash of the kernel sources, so that a benchmark can tell
whether it still describes the current kernels.
"""

import argparse
import csv
import glob
import hashlib
import json
import os
import re
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = ["paper_2511_09389_amd/csrc/tiled.hip", "paper_2511_09389_amd/csrc/common.h",
                  "paper_2511_09389_amd/csrc/device_common.h", "paper_2511_09389_amd/csrc/api.hip"]
# kernel-name fragment -> short name
KERNELS = {"record_kernel": "record", "tile_kernel": "tile", "cell_table_kernel": "table", "gather_pass_kernel": "gather_pass",
           "copy_kernel": "copy", "gather_kernel": "gather", "lds_atomic_kernel": "lds_atomic"}
L2_REQUEST_BYTES = 64


def kernel_source_hash():
    """Hash of the kernel sources with comments and blank space taken out, so that an edit
    of a comment leaves the committed counters valid."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def short_name(kernel_name):
    for frag, short in KERNELS.items():
        if frag in kernel_name:
            return short
    return None


def read_pass(directory):
    """{short kernel name: {counter: [value per dispatch]}} from one pass's CSV files."""
    per_dispatch = defaultdict(float)   # (kernel, dispatch, counter) -> value (summed over rows)
    for path in glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True):
        with open(path, newline="") as fh:
            for row in csv.DictReader(fh):
                k = short_name(row.get("Kernel_Name", ""))
                if k is None:
                    continue
                per_dispatch[(k, row["Dispatch_Id"], row["Counter_Name"])] += float(row["Counter_Value"])
    out = defaultdict(lambda: defaultdict(list))
    for (k, _, counter), v in per_dispatch.items():
        out[k][counter].append(v)
    return out


def reduce(passes, known):
    """Average each counter per dispatch; derive bytes with the copy-kernel calibration."""
    merged = defaultdict(dict)
    for directory in passes:
        for k, counters in read_pass(directory).items():
            for c, vals in counters.items():
                merged[k][c] = {"mean": sum(vals) / len(vals), "dispatches": len(vals)}
    cal = {}
    copy = merged.get("copy", {})
    if "FETCH_SIZE" in copy:
        cal["fetch_factor"] = known["copy_read_bytes"] / (copy["FETCH_SIZE"]["mean"] * 1024.0)
    if "WRITE_SIZE" in copy:
        cal["write_factor"] = known["copy_write_bytes"] / (copy["WRITE_SIZE"]["mean"] * 1024.0)
    if "TCC_READ_SECTORS_sum" in copy:
        cal["l2_read_sector_factor"] = known["copy_read_bytes"] / (copy["TCC_READ_SECTORS_sum"]["mean"] * 32.0)
    g = merged.get("gather", {})
    if "TCP_TCC_READ_REQ_sum" in g:
        cal["gather_l2_request_bytes_over_known"] = (g["TCP_TCC_READ_REQ_sum"]["mean"] * L2_REQUEST_BYTES /
                                                     known["gather_bytes"])
    if "TCC_READ_SECTORS_sum" in g:
        cal["gather_l2_sector_bytes_over_known"] = g["TCC_READ_SECTORS_sum"]["mean"] * 32.0 / known["gather_bytes"]
    summary = {}
    for k, counters in merged.items():
        m = {c: v["mean"] for c, v in counters.items()}
        d = {"dispatches": max(v["dispatches"] for v in counters.values()), "counters": m}
        if "FETCH_SIZE" in m and "fetch_factor" in cal:
            d["hbm_read_bytes"] = m["FETCH_SIZE"] * 1024.0 * cal["fetch_factor"]
        if "WRITE_SIZE" in m and "write_factor" in cal:
            d["hbm_write_bytes"] = m["WRITE_SIZE"] * 1024.0 * cal["write_factor"]
        if "TCP_TCC_READ_REQ_sum" in m:
            d["l2_read_request_bytes"] = m["TCP_TCC_READ_REQ_sum"] * L2_REQUEST_BYTES
        if "TCP_TCC_WRITE_REQ_sum" in m:
            d["l2_write_request_bytes"] = m["TCP_TCC_WRITE_REQ_sum"] * L2_REQUEST_BYTES
        if "TCC_READ_SECTORS_sum" in m:
            d["l2_read_bytes"] = m["TCC_READ_SECTORS_sum"] * 32.0
        if "TCC_WRITE_SECTORS_sum" in m:
            d["l2_write_bytes"] = m["TCC_WRITE_SECTORS_sum"] * 32.0
        if "TCC_HIT_sum" in m and "TCC_MISS_sum" in m and m["TCC_HIT_sum"] + m["TCC_MISS_sum"] > 0:
            d["l2_hit_rate"] = m["TCC_HIT_sum"] / (m["TCC_HIT_sum"] + m["TCC_MISS_sum"])
        summary[k] = d
    return summary, cal


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("out")
    ap.add_argument("passes", nargs="+")
    ap.add_argument("--workload", required=True)
    ap.add_argument("--command", required=True)
    ap.add_argument("--known", default=None, help="JSON of the calibration kernels' known sizes "
                    "(written by bench.py --counters-run)")
    args = ap.parse_args()
    known_path = args.known or os.path.join(args.passes[0], "known.json")
    with open(known_path) as fh:
        known = json.load(fh)
    kernels, cal = reduce(args.passes, known)
    doc = {"workload": args.workload, "command": args.command, "kernel_source_hash": kernel_source_hash(),
           "ray_substeps_per_step": known.get("ray_substeps_per_step"), "calibration": cal,
           "l2_request_bytes": L2_REQUEST_BYTES, "known": known, "kernels": kernels}
    with open(args.out, "w") as fh:
        json.dump(doc, fh, indent=1, sort_keys=True)
    print(json.dumps({k: {kk: vv for kk, vv in v.items() if kk != "counters"} for k, v in kernels.items()},
                     indent=1))


if __name__ == "__main__":
    main()
