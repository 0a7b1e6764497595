"""Host-side checks of bench.py's contract (no GPU calls)."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_is_reported_only_for_the_profiled_sources():
    b = _bench()
    h = b.kernel_source_hash("pm1")
    path = os.path.join(ROOT, "profiles", "traffic_pm_kernel_spw1_ea_l8_r32_x64.json")
    d = json.load(open(path))
    want = d["hbm_bytes_per_launch"] if d["kernel_source_sha256"] == h else None
    assert b.traffic_from_profiles(d["sweeps_per_launch"], h, "pm1") == want
    # another launch length or other sources: no figure
    assert b.traffic_from_profiles(d["sweeps_per_launch"] + 1, h, "pm1") is None
    assert b.traffic_from_profiles(d["sweeps_per_launch"], "0" * 64, "pm1") is None


def test_kernel_hash_follows_the_sources():
    b = _bench()
    assert b.kernel_source_hash("pm1") != b.kernel_source_hash("block")
    assert len(b.kernel_source_hash("pm1")) == 64
