"""The rocprofv3 counter reducer (host logic, no GPU): per-dispatch sums over the rows of a
dispatch, averages over dispatches, the copy-kernel calibration of HBM bytes, and the
source hash that tells the benchmark whether a committed summary still describes the
kernels."""

import csv
import os

import pytest

from paper_2511_09389_amd import counters


def write_pass(directory, rows):
    os.makedirs(directory, exist_ok=True)
    with open(os.path.join(directory, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for d, k, c, v in rows:
            w.writerow({"Dispatch_Id": d, "Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})


COPY = "void (anonymous namespace)::copy_kernel(float4 const*, float4*, long)"
TILE = "void rtmi::(anonymous namespace)::tile_kernel<false, false>(rtmi::TileArgs)"


def test_reduce_sums_rows_averages_dispatches_and_calibrates(tmp_path):
    p1, p2 = str(tmp_path / "p1"), str(tmp_path / "p2")
    mib = 1 << 20
    # pass 1: FETCH_SIZE in KiB, a dispatch's value split over two rows (e.g. two XCDs)
    write_pass(p1, [(1, COPY, "FETCH_SIZE", 64 * 1024), (1, COPY, "FETCH_SIZE", 64 * 1024),
                    (2, COPY, "FETCH_SIZE", 128 * 1024),
                    (3, TILE, "FETCH_SIZE", 300.0), (3, TILE, "FETCH_SIZE", 200.0),
                    (4, TILE, "FETCH_SIZE", 700.0),
                    (5, "some_other_kernel", "FETCH_SIZE", 1e9)])
    # pass 2: WRITE_SIZE and the L2 hit counters
    write_pass(p2, [(1, COPY, "WRITE_SIZE", 256 * 1024),
                    (2, TILE, "WRITE_SIZE", 10.0), (2, TILE, "TCC_HIT_sum", 30.0), (2, TILE, "TCC_MISS_sum", 10.0)])
    known = {"copy_read_bytes": 256 * mib, "copy_write_bytes": 256 * mib, "gather_bytes": 1}
    kernels, cal = counters.reduce([p1, p2], known)
    # the copy reads 256 MiB while FETCH_SIZE reports 128 MiB per dispatch: factor 2
    assert cal["fetch_factor"] == pytest.approx(2.0)
    assert cal["write_factor"] == pytest.approx(1.0)
    tile = kernels["tile"]
    assert tile["counters"]["FETCH_SIZE"] == pytest.approx(600.0)   # (300 + 200 + 700) / 2 dispatches
    assert tile["hbm_read_bytes"] == pytest.approx(600.0 * 1024 * 2.0)
    assert tile["hbm_write_bytes"] == pytest.approx(10.0 * 1024)
    assert tile["l2_hit_rate"] == pytest.approx(0.75)
    assert tile["dispatches"] == 2
    assert set(kernels) == {"copy", "tile"}   # kernels outside the march are left out


def test_source_hash_ignores_comments_and_blank_space(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    monkeypatch.setattr(counters, "ROOT", str(tmp_path))
    monkeypatch.setattr(counters, "KERNEL_SOURCES", ["k.hip"])
    src.write_text("int f(int a) {\n  return a + 1;\n}\n")
    h0 = counters.kernel_source_hash()
    src.write_text("// a comment\nint f(int a) {   /* another\n spanning lines */\n\n  return a + 1;  // why\n}\n")
    assert counters.kernel_source_hash() == h0
    src.write_text("int f(int a) {\n  return a + 2;\n}\n")
    assert counters.kernel_source_hash() != h0
