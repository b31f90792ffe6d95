"""CPU checks of bench.py's contract: one GPU only, the roofline arithmetic
over timing records, and traffic reported only for the profiled sources."""

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def rec(pass_, bucket, ms, probes=0, staged=0, edges=0, triangles=0, tile=64):
    return {"pass": pass_, "bucket": bucket, "arm": 0, "tile": tile, "edges": edges,
            "probes": probes, "staged": staged, "triangles": triangles, "ms": ms}


def test_launch_bytes_follow_the_per_unit_figures():
    count = rec(0, 20, 1.0, probes=1000, staged=100, edges=10, triangles=7)
    write = rec(1, 20, 1.0, probes=1000, staged=100, edges=10, triangles=7)
    assert bench.launch_bytes(count) == 4 * 1000 + 4 * 100 + 8 * 10
    # write: + per edge its two offsets and one original id, + per triangle
    # the third vertex's original id and the 12 bytes written
    assert bench.launch_bytes(write) == 4 * 1000 + 4 * 100 + 8 * 10 + 12 * 10 + 16 * 7
    # the look-ups a launch made, where the record has them, replace its probes
    made = dict(count, lookups=700)
    assert bench.launch_bytes(made) == 4 * 700 + 4 * 100 + 8 * 10


def test_roofline_takes_the_kernel_with_the_most_time():
    recs = [rec(0, 20, 2.0, probes=10**9, edges=10**6),          # heavy count: 2 ms
            rec(1, 20, 3.0, probes=10**9, edges=10**6, triangles=10**8),   # heavy write: 3 ms
            rec(1, 21, 1.0, probes=10**8, edges=10**5, triangles=10**7),
            rec(0, 3, 0.5, probes=10**6, edges=10**5, tile=8)]
    r = bench.roofline(recs, "no-such-workload")
    assert r["kernel"] == "k_heavy<write>" and r["launches"] == 2
    want = (bench.launch_bytes(recs[1]) + bench.launch_bytes(recs[2])) / 4.0e-3 / 1e9
    assert r["achieved"] == pytest.approx(want)
    assert r["frac"] == pytest.approx(want / 8000.0) and r["peak"] == 8000.0
    assert r["traffic"] is None               # nothing profiled for this workload


def test_windowed_write_bytes_come_from_the_whole_buckets():
    # a heavy bucket's write split over two windows: each write record carries
    # the whole bucket (its probes are the hit-span look-ups of the write
    # pass), counted once, over both launches' time
    recs = [rec(0, 20, 2.0, probes=10**9, edges=10**6, triangles=10**8),
            rec(1, 20, 2.0, probes=6 * 10**8, edges=10**6, triangles=10**8),
            rec(1, 20, 2.0, probes=6 * 10**8, edges=10**6, triangles=10**8)]
    r = bench.roofline(recs, "no-such-workload", windowed=True)
    assert r["kernel"] == "k_heavy<write>" and r["launches"] == 2
    assert r["achieved"] == pytest.approx(bench.launch_bytes(recs[1]) / 4.0e-3 / 1e9)
    # a light bin's partial write launches (probes -1) take the count record's
    # figures as a write pass
    recs = [rec(0, 5, 1.0, probes=10**9, edges=10**7, triangles=10**8, tile=32),
            rec(1, 5, 3.0, probes=-1, edges=10**6, triangles=-1, tile=32),
            rec(1, 5, 3.0, probes=-1, edges=10**6, triangles=-1, tile=32)]
    r = bench.roofline(recs, "no-such-workload", windowed=True)
    assert r["kernel"] == "k_light<32><write>" and r["launches"] == 2
    whole = bench.launch_bytes(dict(recs[0], **{"pass": 1}))
    assert r["achieved"] == pytest.approx(whole / 6.0e-3 / 1e9)


@pytest.mark.parametrize("workload", ["rmat20", "chunglu4m", "rmat26"])
def test_traffic_only_for_the_profiled_sources(workload, monkeypatch):
    prof = os.path.join(ROOT, "profiles", f"k_heavy_write_{workload}_traffic.json")
    with open(prof) as f:
        stored = json.load(f)
    assert stored["workload"] == workload
    if stored["source_hash"] == bench.kernel_source_hash():
        # a pass's bytes spread over the launches of this run's pass
        assert bench.profiled_traffic("k_heavy<write>", workload, 4) == \
            pytest.approx(stored["traffic_bytes_per_pass"] / 4)
    # no profile for another workload
    assert bench.profiled_traffic("k_heavy<write>", "rmat18", 4) is None
    # a different kernel source: no traffic
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.profiled_traffic("k_heavy<write>", workload, 4) is None
    assert bench.profiled_traffic("k_light<64><write>", workload, 4) is None
