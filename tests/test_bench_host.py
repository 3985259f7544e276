"""Host logic of the benchmark script (no GPU): argument handling, the
workload table, the roofline record and the use of the committed traffic
summary only while it matches the kernel sources."""
from __future__ import annotations

import os
import subprocess
import sys
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_workload_table():
    envs, desc = bench.build_workload("batch60")
    assert len(envs) == 60 and "60 mixed pads" in desc
    words = {"slide": "friction off", "friction": "friction 0.5", "layers": "two layers", "mesh": "triangle meshes"}
    for kind, w in words.items():
        envs, desc = bench.build_workload(f"batch60-{kind}")
        assert len(envs) == 60 and w in desc
    envs, _ = bench.build_workload("single1944")
    assert len(envs) == 1 and envs[0].pad.tets.shape[0] == 1944
    with pytest.raises(SystemExit):
        bench.build_workload("batch61")


def _fake_ctx(timers):
    return types.SimpleNamespace(timing=lambda: timers)


def test_roofline_record_takes_the_dominant_kernel():
    args = types.SimpleNamespace(workload="batch60", sequential=False, timing_stride=29)
    # cg_spmv: 0.02 ms x 1000 launches = 20 ms in total; element 0.2 ms x 50 = 10 ms
    timers = {"cg_spmv": (0.02, 1000, 40e6), "element": (0.2, 50, 1e9)}
    r = bench.roofline(_fake_ctx(timers), args)
    assert r["kernel"] == "cg_spmv" and r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx(40e6 / 0.02e-3 / 1e9, rel=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0, rel=1e-3)
    assert bench.roofline(_fake_ctx({}), args) is None


def test_traffic_only_from_a_matching_summary(tmp_path, monkeypatch):
    from paper_2606_20426_amd.profiling import kernel_sources_hash
    h = kernel_sources_hash()
    f = tmp_path / "pmc.md"

    def write(workload, kernel, sha):
        f.write_text(f"# x\n\n- workload: `{workload}`\n- kernel: `{kernel}`\n- kernel_sources_sha256: `{sha}`\n"
                     f"- traffic_bytes_per_launch: 12345\n")
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(f))
    write("batch60", "cg_spmv", h)
    assert bench.measured_traffic("batch60", "cg_spmv") == 12345.0
    assert bench.measured_traffic("batch60", "element") is None
    assert bench.measured_traffic("batch60-mesh", "cg_spmv") is None
    write("batch60", "cg_spmv", "0" * 64)                 # kernels changed since the counters
    assert bench.measured_traffic("batch60", "cg_spmv") is None
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(tmp_path / "missing.md"))
    assert bench.measured_traffic("batch60", "cg_spmv") is None
