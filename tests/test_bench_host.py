"""Host logic of the benchmark script (no GPU): the layout procedure's
choice of order, the guard that keeps counter traffic from a stale profile
out of the result line, and the single-GPU contract."""
import hashlib
import os
import subprocess
import sys
from pathlib import Path

import numpy as np

import bench

ROOT = Path(__file__).resolve().parent.parent


class _FakeSearch:
    """Stands in for the library's order search: a fixed cost per (seed,
    start) and a record of the calls."""

    def __init__(self, costs):
        self.costs = costs
        self.calls = []

    def order_search(self, ctx, text, seed, budget, start=None):
        key = (seed, None if start is None else int(start[0]))
        self.calls.append((seed, budget, key[1]))
        c = self.costs[key]
        return np.array([seed & 0xFF, 1, 2], dtype=np.int32), 100.0, c


def test_benchmark_layout_keeps_the_cheapest_start_and_only_improvements():
    s = 0x100
    costs = {(s, None): 90.0, (s + 1, None): 70.0, (s + 2, None): 80.0,
             # refinement rounds start from the best order so far, whose
             # first entry is the low byte of the seed that found it
             (s + 16, 0x01): 75.0,          # worse: kept out
             (s + 17, 0x01): 60.0,          # better: taken
             (s + 18, 0x11): 65.0}          # worse than 60: kept out
    fake = _FakeSearch(costs)
    order, info = bench.benchmark_layout(fake, None, "text", seed=s, budget=7, starts=3, refine=3)
    assert [c[0] for c in fake.calls] == [s, s + 1, s + 2, s + 16, s + 17, s + 18]
    assert all(c[1] == 7 for c in fake.calls)
    assert [c[2] for c in fake.calls] == [None, None, None, 0x01, 0x01, 0x11]
    assert int(order[0]) == 0x11
    assert info["searched_cost"] == 60.0 and info["snake_cost"] == 100.0
    assert info["costs_of_starts"] == [90.0, 70.0, 80.0]
    assert info["costs_after_refine"] == [70.0, 60.0, 60.0]
    assert info["best_start_seed"] == hex(s + 1)
    assert info["ratio"] == 0.6


def test_measured_traffic_requires_matching_kernel_and_layout(tmp_path, monkeypatch):
    src = tmp_path / "paper_2609_19116_amd" / "csrc" / "kernels" / "mps.hip"
    src.parent.mkdir(parents=True)
    src.write_bytes(b"kernel source v1")
    sha = hashlib.sha256(b"kernel source v1").hexdigest()[:16]
    (tmp_path / "profiles").mkdir()
    lay = "search 3x128 +4 from 0x5eed0081"
    for name, val in (("mps_kernel", "1.5e+08"), ("mps_wave_kernel", "2.5e+08")):
        (tmp_path / "profiles" / f"{name}_c3_hbm_counters.md").write_text(
            f"header\n\ntraffic_bytes_per_launch: {val}\nkernel_sha256_16: {sha}\n"
            f"layout: {lay}\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # each shot kernel reads its own summary
    assert bench.measured_traffic(lay, "mps_kernel<float,32>") == 1.5e8
    assert bench.measured_traffic(lay, "mps_wave_kernel<float>") == 2.5e8
    assert bench.measured_traffic("snake", "mps_wave_kernel<float>") is None
    src.write_bytes(b"kernel source v2")
    assert bench.measured_traffic(lay, "mps_kernel<float,32>") is None
    assert bench.measured_traffic(lay, "mps_wave_kernel<float>") is None
    (tmp_path / "profiles" / "mps_kernel_c3_hbm_counters.md").unlink()
    assert bench.measured_traffic(lay, "mps_kernel<float,32>") is None


def test_bench_refuses_more_than_one_gpu():
    env = dict(os.environ)
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""
