"""Host logic of the benchmark script (no GPU): the committed traffic records are used only
on the kernel sources they were taken on, their byte counts follow from the counters and
the copy-probe calibration they carry, and a request for more than one GPU is refused."""
import json
import os
import subprocess
import sys

import bench

WORKLOADS = ("disc10", "outflow5")


def _record(wl):
    return json.load(open(os.path.join(bench.ROOT, "profiles", f"formal_solve_{wl}_fp64_traffic.json")))


def test_traffic_record_is_gated_by_the_kernel_source_hash(monkeypatch):
    for wl in WORKLOADS:
        d = _record(wl)
        monkeypatch.setattr(bench, "kernel_source_hash", lambda: d["kernel_sha"])
        assert bench.traffic_from_profile(wl, "fp64", None) == d["hbm_bytes_per_launch"]
        monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
        assert bench.traffic_from_profile(wl, "fp64", None) is None
    assert bench.traffic_from_profile("no_such_workload", "fp64", None) is None


def test_traffic_records_follow_from_counters_and_copy_probe():
    for wl in WORKLOADS:
        d = _record(wl)
        cp = d["copy_probe"]
        # the probe's factors: bytes a plain copy moved over what the counter read for it
        assert abs(cp["fetch_factor"] - cp["bytes_read"] / (cp["fetch_size_kib"] * 1024)) < 1e-12
        assert abs(cp["write_factor"] - cp["bytes_written"] / (cp["write_size_kib"] * 1024)) < 1e-12
        read = d["fetch_size_kib"] * 1024 * cp["fetch_factor"]
        write = d["write_size_kib"] * 1024 * cp["write_factor"]
        assert abs(d["hbm_read_bytes_per_launch"] - read) <= 1e-9 * read
        assert abs(d["hbm_write_bytes_per_launch"] - write) <= 1e-9 * write
        assert abs(d["hbm_bytes_per_launch"] - (read + write)) <= 1e-9 * (read + write)
        assert d["workload"] == wl and d["precision"] == "fp64"


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""
