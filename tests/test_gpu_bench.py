"""The benchmark on an MI355X: a short default run (10^6 particles,
Gauss-Hermite kinematics, 20 timed steps) in a child process prints one JSON
line whose fields follow the benchmark's output contract."""

import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_prints_one_json_line_with_roofline():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("[gpu-test] bench.py --steps 20 --warmup 2", file=sys.stderr, flush=True)
    r = subprocess.run([sys.executable, "-u", "bench.py", "--steps", "20", "--warmup", "2",
                        "--no-cpu-baseline"], cwd=ROOT, capture_output=True, text=True, timeout=110)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
    assert len(lines) == 1, r.stdout[-2000:]
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config", "roofline",
              "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 20 and d["warmup"] == 2
    assert d["unit"] == "particle-steps/s" and d["dtype"] == "f32" and d["data"] == "synthetic"
    assert d["config"]["workload"] == "hernquist_gh_n1m" and d["config"]["particles"] == 1_000_000
    # whole-step throughput: N particles per step over the measured time per step
    assert d["value"] == pytest.approx(1_000_000 / (d["ms_per_step"] * 1e-3), rel=1e-9)
    roof = d["roofline"]
    assert roof["bound"] == "hbm" and roof["unit"] == "GB/s" and roof["peak"] == 8000.0
    assert 0.0 < roof["frac"] <= 1.0
    assert roof["frac"] == pytest.approx(roof["achieved"] / roof["peak"], rel=1e-9)
    # achieved: 60 B per particle-step over the step kernel's own duration,
    # which is shorter than the whole step
    assert roof["achieved"] == pytest.approx(60 * 1_000_000 / (roof["kernel_ms"] * 1e-3) / 1e9,
                                             rel=1e-9)
    assert 0.0 < roof["kernel_ms"] < d["ms_per_step"]
