"""Binding of librtmi_peaks.so (ctypes): the device-rate microbenchmarks that the march's
rooflines are quoted against. Each call runs on the current device, allocates and frees
its own buffers and synchronises; importing fails loudly if the library is not built."""

import ctypes
import os

# torch first: its HIP runtime must be the process's one, so that the library below binds
# to it (loaded first, the system runtime would be a second copy and torch would find no
# device)
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librtmi_peaks.so")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2511_09389_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    I32, I64, D = ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
    sig = {
        "rtmi_peak_copy": [I64, I32, D, D],
        "rtmi_peak_gather": [I64, I32, I32, D, D],
        "rtmi_peak_lds_atomic": [I32, I32, I32, D, D],
        "rtmi_peak_global_atomic": [I64, I32, I32, I32, D, D],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.restype = I32
        fn.argtypes = args
    return lib


lib = _load()


def _run(fn, *args):
    rate, amount = ctypes.c_double(0.0), ctypes.c_double(0.0)
    code = fn(*args, ctypes.byref(rate), ctypes.byref(amount))
    if code != 0:
        raise RuntimeError(f"{fn.__name__} failed with code {code}")
    return rate.value, amount.value


def copy(nbytes=1 << 30, reps=5):
    """Device copy: (bytes read + written per second, bytes per launch)."""
    return _run(lib.rtmi_peak_copy, int(nbytes), int(reps))


def gather(footprint, iters=64, reps=5):
    """Random whole 64-byte line reads over `footprint` bytes: (bytes/s, bytes per launch)."""
    return _run(lib.rtmi_peak_gather, int(footprint), int(iters), int(reps))


LDS_KINDS = {"f64": 0, "u64": 1, "f32": 2, "f64_random": 3, "u64_random": 4,
             "f64_random_half": 5, "f64_random_quarter": 6, "f64_random_eighth": 7}


def lds_atomic(kind="f64", iters=1200, reps=5):
    """LDS atomic adds (kinds: f64, u64, f32 on consecutive slots; f64_random, u64_random
    on random slots; f64_random_half/_quarter/_eighth with one lane in 2/4/8 adding):
    (adds/s of the adding lanes, adds per launch)."""
    return _run(lib.rtmi_peak_lds_atomic, LDS_KINDS[kind], int(iters), int(reps))


def global_atomic(footprint=64 << 20, scattered=False, iters=64, reps=5):
    """Global binary32 atomic adds: (adds/s, adds per launch)."""
    return _run(lib.rtmi_peak_global_atomic, int(footprint), 1 if scattered else 0, int(iters), int(reps))


def measure_all():
    """The peaks the march's rooflines use, measured now on the current device."""
    out = {}
    out["copy_Bps"] = copy()[0]
    out["gather_l2_Bps"] = gather(2 << 20)[0]          # fits every XCD's 4 MB L2
    out["gather_mall_Bps"] = gather(128 << 20)[0]      # beyond L2, inside the 256 MB Infinity Cache
    out["gather_hbm_Bps"] = gather(4 << 30, iters=16)[0]   # beyond the Infinity Cache
    out["lds_add_f64_per_s"] = lds_atomic("f64")[0]
    out["lds_add_u64_per_s"] = lds_atomic("u64")[0]
    out["lds_add_f32_per_s"] = lds_atomic("f32")[0]
    out["lds_add_f64_random_per_s"] = lds_atomic("f64_random")[0]
    out["lds_add_u64_random_per_s"] = lds_atomic("u64_random")[0]
    out["lds_add_f64_random_half_lanes_per_s"] = lds_atomic("f64_random_half")[0]
    out["lds_add_f64_random_quarter_lanes_per_s"] = lds_atomic("f64_random_quarter")[0]
    out["global_atomic_f32_coalesced_per_s"] = global_atomic(scattered=False)[0]
    out["global_atomic_f32_scattered_per_s"] = global_atomic(scattered=True)[0]
    return out
