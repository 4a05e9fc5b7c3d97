"""The benchmark's contract: one JSON line with the agreed fields, one GPU only.
The CPU tests check the host logic; the GPU test runs a short benchmark."""
import argparse
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_trace_bytes_counts_spheres_nodes_and_pixels():
    # N (16 + colour) + (N - 1) 56 + 20 P
    assert bench.trace_bytes(1, 1, True) == 24 + 0 + 20
    assert bench.trace_bytes(10, 100, False) == 10 * 32 + 9 * 56 + 2000
    assert bench.trace_bytes(735159, 1920 * 1080, True) == 100284664


def test_profile_figures_only_for_the_profiled_configuration():
    base = dict(kbuf=6, tile="8x8", scale=1.0, walk=2, schedule=2)
    for change in ({"kbuf": 8}, {"tile": "16x4"}, {"scale": 2.0}, {"walk": 0}, {"schedule": 0}):
        a = argparse.Namespace(**dict(base, **change))
        assert bench.measured_traffic(a) is None
        assert bench.valu_issue(a, 0.3) is None


@pytest.mark.gpu
def test_short_benchmark_prints_the_contract_line():
    r = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--steps", "2", "--warmup", "1",
                        "--no-cpu", "--no-bwd", "--batch-frames", "0", "--no-extra"],
                       capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 2 and d["warmup"] == 1 and d["higher_is_better"] is True
    assert d["value"] > 0 and d["ms_per_step"] > 0 and "workload" in d["config"]
    ro = d["roofline"]
    assert ro["bound"] == "hbm" and ro["unit"] == "GB/s" and ro["peak"] == 8000.0
    assert abs(ro["frac"] - ro["achieved"] / ro["peak"]) < 1e-3
    assert "cpu_baseline" not in d
