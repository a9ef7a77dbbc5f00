"""Host logic of bench.py (CPU): the one-GPU guard, the level schedule and
algorithmic model behind the roofline fields, the bound selection, and the
hash guard on the committed traffic summaries."""
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("N", [1, 2, 3, 7, 64, 777, 65536])
def test_levels_eliminate_every_block_once(N):
    """One-sided CR eliminates each block row exactly once over the levels
    (the last level factors its single block); kept blocks halve."""
    L = list(bench.levels(N))
    assert sum(lv[1] for lv in L) == N
    n = N
    for (nl, ne, nk, *_rest) in L:
        assert nl == n and ne + nk == n and ne == (n + 1) // 2
        n = nk
    assert n == 0


def test_step_model_totals():
    """N=65536, m=32, k=16, FP64: 18.9 GB and 97.3 GFLOP per fused step (the
    figures the roofline fraction of the default line is quoted against)."""
    t = bench.step_model("fp64", 65536, 32, 16)
    assert set(t) == {"k_elim", "k_reduce", "k_back"}
    assert abs(sum(v[0] for v in t.values()) / 18.87e9 - 1) < 1e-3
    assert abs(sum(v[1] for v in t.values()) / 97.34e9 - 1) < 1e-3


def test_roofline_bound_and_fraction():
    # 17 launches of 2 ms with 1.6 GB and 1 GFLOP in all: HBM-bound
    r = bench.roofline({"k_elim": (17.0, 34.0)}, {"k_elim": [1.6e9, 1e9]}, True)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["kernel"] == "k_elim"
    assert abs(r["achieved"] - 1.6e9 / 17 / 2e-3 / 1e9) < 1e-9
    assert abs(r["frac"] - r["achieved"] / 8000.0) < 1e-12
    # the same time with 100 TFLOP: matrix-bound, FP64 or FP32 peak
    r64 = bench.roofline({"k_reduce": (10.0, 20.0)}, {"k_reduce": [1e9, 1e14]}, True)
    r32 = bench.roofline({"k_reduce": (10.0, 20.0)}, {"k_reduce": [1e9, 1e14]}, False)
    assert r64["bound"] == r32["bound"] == "mfma"
    assert r64["peak"] == 78.6 and r32["peak"] == 157.3
    assert abs(r64["achieved"] - 1e13 / 2e-3 / 1e12) < 1e-9


def test_traffic_summary_guarded_by_source_hash(monkeypatch):
    path = os.path.join(ROOT, "profiles", "hbm_traffic_fp64_N65536_m32_k16.json")
    rec = json.load(open(path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: rec["kernel_source_sha256_16"])
    t = bench.measured_traffic("fp64", "k_elim")
    assert t == rec["kernels"]["k_elim"]["traffic_bytes_per_launch"] and t > 0
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.measured_traffic("fp64", "k_elim") is None
