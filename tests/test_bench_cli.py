"""bench.py's contract on the CPU (no GPU is touched): a request for more than one GPU
or an intercommutation probability outside (0, 1] exits with status 2 and a message;
the per-unit byte counts behind the roofline are the documented ones; the HBM traffic
comes from the committed counter summary only for the kernel source and launch
configuration it was taken with."""
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = run("--gpus", "2")
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_probability_out_of_range_is_refused():
    for p in ("0", "1.5", "-0.2"):
        r = run("--p", p)
        assert r.returncode == 2 and "outside (0, 1]" in r.stderr


def test_byte_model():
    # evolve: X[n], X[n-1] (64), next (4), X[n+1] (32), box (32 or 64), cell + slot (8),
    # bucket counter read-modify-write (8); bounded regions: stop step + sub-region (8)
    assert bench.evolve_bytes_per_point(True, False) == 148
    assert bench.evolve_bytes_per_point(True, True) == 156
    assert bench.evolve_bytes_per_point(False, False) == 180
    # screen: the packed FP32 entry; FP64: (cell, slot) + FP64 box
    assert bench.screen_bytes_per_element(True) == 32
    assert bench.screen_bytes_per_element(False) == 72


def profiled(key):
    with open(os.path.join(ROOT, "profiles", "batched512_hbm_counters.txt")) as f:
        for line in f:
            if line.startswith("traffic-per-launch:"):
                return dict(t.split("=", 1) for t in line.split()[1:])[key]
    return None


def test_traffic_only_for_the_profiled_source_and_configuration():
    cfg = profiled("config")
    assert cfg and cfg.startswith("eager-1lane-")
    for k in ("k_screen", "k_evolve"):
        assert bench.counted_traffic(k, "eager-1lane-bp1-split5-sync64-f64") is None
    assert bench.counted_traffic("k_confirm", cfg) is None
    if profiled("source") != bench.kernel_source_hash():
        pytest.skip("the committed counter summary is for another kernel source: traffic is "
                    "reported as null until the kernels are profiled again")
    for k in ("k_screen", "k_evolve"):
        t = bench.counted_traffic(k, cfg)
        assert t is not None and t > 0
