"""Compile librtmi.so for gfx950 with hipcc (in-tree, next to this file)."""

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "librtmi.so")
SOURCES = ["api.hip", "march.hip", "tiled.hip", "adjoint.hip", "conv.hip"]
PEAKS_LIB = os.path.join(PKG, "librtmi_peaks.so")
PEAK_SOURCES = ["peaks.hip"]
HOST_FEATURE_NOTE = "'-packed-fp32-ops' is not a recognized feature for this target"


def hipcc():
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found; the HIP library cannot be built")


def _compile(sources, out, verbose):
    tmp = out + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
           # packed FP32 instructions stay off in all device code
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           # host code: no contraction into FMA (direction tables are binary64 -> binary32)
           "-Xarch_host", "-ffp-contract=off",
           "-Wall", "-Wno-unused-result",
           "-I", INCLUDE, "-o", tmp] + [os.path.join(CSRC, s) for s in sources]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, cwd=PKG, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    # The feature flag above must reach the device pass, and hipcc forwards it to the host
    # pass too (-Xarch_device refuses options that take arguments, such as -Xclang), whose
    # x86 backend prints one harmless "not a recognized feature" line per source file.
    # Those lines are dropped; everything else the compiler prints is passed on.
    lines = [ln for ln in res.stdout.splitlines() if HOST_FEATURE_NOTE not in ln]
    if lines:
        print("\n".join(lines), file=sys.stderr, flush=True)
    if res.returncode != 0:
        raise subprocess.CalledProcessError(res.returncode, cmd, output=res.stdout)
    os.replace(tmp, out)
    return out


def build(verbose=False):
    """Build librtmi.so and the peak microbenchmarks (librtmi_peaks.so); always
    recompiles. Raises CalledProcessError on failure."""
    _compile(PEAK_SOURCES, PEAKS_LIB, verbose)
    return _compile(SOURCES, LIB, verbose)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
