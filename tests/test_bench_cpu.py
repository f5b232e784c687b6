"""Host-side parts of the benchmark (no GPU): the one-GPU rule, the use of the
committed HBM counters only for the kernel they were taken on, and the shape
of the CPU baseline."""

import json

import pytest

import bench
from workloads import workload


def test_more_than_one_gpu_is_refused_before_any_device_work(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    assert "one GPU" in capsys.readouterr().err


def test_traffic_is_used_only_for_the_kernel_it_was_measured_on(tmp_path, monkeypatch):
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps({"w": {"kernel_hash": bench.kernel_hash(), "bytes_per_launch": 6.1e7,
                                   "algorithmic_bytes_per_launch": 6.0e7}}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("w", 1_000_000) == pytest.approx(61.0)
    assert bench.measured_traffic("other", 1_000_000) is None
    f.write_text(json.dumps({"w": {"kernel_hash": "0" * 16, "bytes_per_launch": 6.1e7}}))
    assert bench.measured_traffic("w", 1_000_000) is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.measured_traffic("w", 1_000_000) is None


def test_kernel_hash_covers_every_source_of_the_step_kernel():
    """The traffic record is kept only while the step kernel is unchanged: the
    hash covers the units that instantiate it and every file they include
    (the finalize kernels in m2m_kernels.hip are not part of it)."""
    import os
    import re
    srcs = set(bench.KERNEL_SOURCES)
    csrc = os.path.join(bench.ROOT, "paper_1202_2355_amd", "csrc")
    todo = [n for n in os.listdir(csrc) if n.startswith("m2m_step") and n.endswith(".hip")]
    assert len(todo) == 3
    seen = set()
    while todo:
        name = todo.pop()
        if name in seen:
            continue
        seen.add(name)
        assert f"paper_1202_2355_amd/csrc/{name}" in srcs, name
        with open(os.path.join(csrc, name)) as fh:
            todo += [m for m in re.findall(r'#include "([^"]+)"', fh.read())
                     if os.path.exists(os.path.join(csrc, m))]


def test_cpu_baseline_reports_all_cores_and_one_thread():
    r = bench.cpu_baseline(workload(1), 0.5)
    assert r["kind"] == "oracle" and r["unit"] == "particle-steps/s"
    assert r["cores"] >= 1 and r["value"] > 0 and r["value_1_thread"] > 0
    assert "one thread" in r["sample_1_thread"]


def test_cpu_baseline_of_the_batch_runs_its_own_fits():
    from workloads.configs import batch_fits
    r = bench.cpu_baseline_batch(batch_fits(n_fits=3), 0.5, n_cap=4096)
    assert r["kind"] == "oracle" and r["unit"] == "particle-steps/s"
    assert r["cores"] >= 1 and r["value"] > 0
    assert "fits of the batch" in r["sample"]


def test_default_workload_is_the_batch():
    args = bench.parser().parse_args([])
    assert args.workload == 4 and args.fits == 64 and args.gpus == 1
