"""Host-side tests of librtmi (no GPU): exports, host logic and argument validation."""

import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rtmi.h")
LIB = os.path.join(ROOT, "paper_2511_09389_amd", "librtmi.so")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("librtmi.so is not built (run __graft_entry__.build())")
    from paper_2511_09389_amd import rtmi
    return rtmi.lib


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rtmi_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared_functions()
    for want in ("rtmi_trace_single", "rtmi_trace_multi", "rtmi_trace_bins", "rtmi_num_substeps",
                 "rtmi_fibonacci_directions", "rtmi_debug_rays", "rtmi_last_error", "rtmi_prepare"):
        assert want in names


def test_library_exports_every_declared_symbol(lib):
    raw = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(raw, name), name


def test_peaks_library_exports_every_declared_symbol():
    path = os.path.join(ROOT, "paper_2511_09389_amd", "librtmi_peaks.so")
    if not os.path.exists(path):
        pytest.fail("librtmi_peaks.so is not built (run __graft_entry__.build())")
    text = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "rtmi_peaks.h")).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(rtmi_peak_[a-z0-9_]+)\s*\(", text)))
    assert len(names) == 4
    import torch  # noqa: F401  (its HIP runtime first, as the binding does)
    raw = ctypes.CDLL(path)
    for name in names:
        assert hasattr(raw, name), name
    # argument checks run before any device call
    rate = ctypes.c_double(0.0)
    raw.rtmi_peak_copy.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    assert raw.rtmi_peak_copy(16, 1, ctypes.byref(rate), None) == -1


def test_fibonacci_table_is_bitwise_the_oracle_table(lib):
    from paper_2511_09389_amd import rtmi
    for n in (1, 2, 3, 64, 255, 256, 1000, 4096, 16384):
        got = rtmi.fibonacci_directions(n)
        want = oracle.fibonacci_directions(n).astype(np.float32)
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), n


@pytest.mark.parametrize("ds,c,dt,cap", [(0.5, 16.0, 1.0, 0), (0.5, 128.0, 1.0, 0), (0.5, 256.0, 1.0, 100),
                                          (0.5, 10.0, 0.3, 0), (0.25, 1.0, 1.1, 0), (0.3, 7.0, 0.9, 3),
                                          (0.5, 0.0, 1.0, 0), (0.7, 3.0, 0.0, 5), (1e-3, 1.0, 1.0, 0)])
def test_num_substeps_matches_oracle(lib, ds, c, dt, cap):
    from paper_2511_09389_amd import rtmi
    assert rtmi.num_substeps(ds, c, dt, cap) == oracle.num_substeps(ds, c, dt, cap)


def test_num_substeps_errors(lib):
    assert lib.rtmi_num_substeps(0.0, 1.0, 1.0, 0) == -1
    assert lib.rtmi_num_substeps(0.5, -1.0, 1.0, 0) == -1
    assert lib.rtmi_num_substeps(0.5, 1.0, -1.0, 0) == -1
    assert lib.rtmi_num_substeps(float("nan"), 1.0, 1.0, 0) == -3
    assert lib.rtmi_num_substeps(0.5, float("inf"), 1.0, 0) == -3
    assert lib.rtmi_num_substeps(1e-6, 1e3, 1e3, 0) == -6          # N_s > 2^24
    assert "2^24" in lib.rtmi_last_error().decode()
    assert lib.rtmi_num_substeps(1e-6, 1e3, 1e3, 10) == 10         # the cap keeps it in range


def _call_single(lib, j=1, k=1, n=(4, 4, 4), src=(1.0, 1.0, 1.0), rays=8, ds=0.5, c=2.0, dt=1.0, out=1):
    s = (ctypes.c_float * 3)(*src)
    return lib.rtmi_trace_single(ctypes.c_void_p(j), ctypes.c_void_p(k), n[0], n[1], n[2], s, rays,
                                 ds, c, dt, ctypes.c_void_p(out), None)


@pytest.mark.parametrize("kw,code", [
    (dict(j=0), -1), (dict(k=0), -1), (dict(out=0), -1),
    (dict(n=(0, 4, 4)), -2), (dict(n=(4, -1, 4)), -2), (dict(n=(2048, 2048, 1024)), -2),
    (dict(src=(float("nan"), 0.0, 0.0)), -3), (dict(src=(0.0, float("inf"), 0.0)), -3),
    (dict(ds=0.0), -1), (dict(ds=-0.5), -1), (dict(c=-1.0), -1), (dict(dt=-1.0), -1),
    (dict(ds=float("nan")), -3), (dict(rays=0), -1), (dict(rays=(1 << 24) + 1), -6),
    (dict(ds=1e-6, c=1e3, dt=1e3), -6),
])
def test_validation_rejects_before_any_device_work(lib, kw, code):
    """Invalid arguments are rejected on the host; the bogus pointers are never touched."""
    assert _call_single(lib, **kw) == code
    assert lib.rtmi_last_error().decode() != ""


def test_multi_and_bins_validation(lib):
    src = (ctypes.c_float * 6)(1, 1, 1, 2, 2, 2)
    nr = (ctypes.c_int32 * 2)(8, 0)
    assert lib.rtmi_trace_multi(ctypes.c_void_p(1), ctypes.c_void_p(1), 4, 4, 4, 2, src, nr, None,
                                0.5, 2.0, 1.0, ctypes.c_void_p(1), None) == -1
    nr2 = (ctypes.c_int32 * 2)(8, 8)
    assert lib.rtmi_trace_multi(ctypes.c_void_p(1), ctypes.c_void_p(1), 4, 4, 4, 0, src, nr2, None,
                                0.5, 2.0, 1.0, ctypes.c_void_p(1), None) == -1
    assert lib.rtmi_trace_multi(ctypes.c_void_p(1), ctypes.c_void_p(1), 4, 4, 4, 2, None, nr2, None,
                                0.5, 2.0, 1.0, ctypes.c_void_p(1), None) == -1
    from paper_2511_09389_amd.rtmi import Options
    bad_scale = (ctypes.c_float * 2)(1.0, float("nan"))
    assert lib.rtmi_trace_bins(ctypes.c_void_p(1), 0, ctypes.c_void_p(1), 0, bad_scale, 2, 4, 4, 4, 2,
                               src, nr2, None, 0.5, 2.0, 1.0, ctypes.c_void_p(1), None, None) == -3
    # a per-bin stride shorter than one grid
    assert lib.rtmi_trace_bins(ctypes.c_void_p(1), 10, ctypes.c_void_p(1), 0, None, 2, 4, 4, 4, 2,
                               src, nr2, None, 0.5, 2.0, 1.0, ctypes.c_void_p(1), None, None) == -1
    opts = Options(7, None, 0.0, 0)
    assert lib.rtmi_trace_bins(ctypes.c_void_p(1), 0, ctypes.c_void_p(1), 0, None, 1, 4, 4, 4, 2,
                               src, nr2, None, 0.5, 2.0, 1.0, ctypes.c_void_p(1), ctypes.byref(opts), None) == -1
    nr3 = (ctypes.c_int32 * 2)(8, 9)
    dirs = (ctypes.c_float * 27)(*([1.0, 0.0, 0.0] * 9))
    opts = Options(0, ctypes.cast(dirs, ctypes.c_void_p).value, 0.0, 0)
    assert lib.rtmi_trace_bins(ctypes.c_void_p(1), 0, ctypes.c_void_p(1), 0, None, 1, 4, 4, 4, 2,
                               src, nr3, None, 0.5, 2.0, 1.0, ctypes.c_void_p(1), ctypes.byref(opts), None) == -1


def test_debug_rays_validation(lib):
    src = (ctypes.c_float * 3)(1, 1, 1)
    assert lib.rtmi_debug_rays(ctypes.c_void_p(1), ctypes.c_void_p(1), 4, 4, 4, src, 0, 0.5, 2.0, 1.0, 0,
                               ctypes.c_void_p(1), None, None) == -1
    assert lib.rtmi_debug_rays(ctypes.c_void_p(1), ctypes.c_void_p(1), 4, 4, 4, src, 8, 0.5, 2.0, 1.0, 0,
                               None, None, None) == -1


def test_version(lib):
    assert lib.rtmi_version() >= 100


def test_deterministic_mode_refuses_negative_kappa_scale(lib):
    """The fixed-point bound assumes non-negative bin scales; the call is refused on the
    host (the bogus device pointers are never touched)."""
    from paper_2511_09389_amd.rtmi import Options
    src = (ctypes.c_float * 3)(1, 1, 1)
    nr = (ctypes.c_int32 * 1)(8)
    scale = (ctypes.c_float * 2)(1.0, -0.5)
    opts = Options(1, None, 0.0, 0, 0)
    assert lib.rtmi_trace_bins(ctypes.c_void_p(1), 0, ctypes.c_void_p(1), 0, scale, 2, 4, 4, 4, 1,
                               src, nr, None, 0.5, 2.0, 1.0, ctypes.c_void_p(1), ctypes.byref(opts),
                               None) == -1
    assert "kappa_scale" in lib.rtmi_last_error().decode()
