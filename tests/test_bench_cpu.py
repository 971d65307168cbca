"""The benchmark's host-side contract (no GPU): the multi-GPU refusal, the per-attempt
work model of the roofline, the traffic record gated on the kernel source hash, and the
oracle baseline's report."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
import workloads as W  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and p.stdout == ""


def test_tau_corr_with_packed_spins_is_refused_with_a_message():
    # the correlations are taken from byte spins; --tau-corr alone picks that encoding
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--tau-corr",
                        "--encoding", "bitpack"], capture_output=True, text=True, timeout=60)
    assert p.returncode == 2
    assert "--encoding int8" in p.stderr and p.stdout == ""


def test_work_model():
    # Philox share 10, field d/2, time field 0.5, index 1.25, decision 3, update 0.25
    assert bench.ops_per_flip(6) == pytest.approx(18.0)
    assert bench.ops_per_flip(4) == pytest.approx(17.0)
    assert bench.PEAK_INT_OPS == pytest.approx(256 * 64 * 2.4e9)


def test_traffic_record_follows_the_kernel_source(tmp_path, monkeypatch):
    rec = tmp_path / "rec.json"
    src = tmp_path / "k.hip"
    src.write_bytes(b"kernel v1")
    import hashlib
    rec.write_text(json.dumps({"source_sha256": hashlib.sha256(b"kernel v1").hexdigest(),
                               "hbm_bytes_per_launch": 123.0}))
    monkeypatch.setattr(bench, "TRAFFIC_RECORDS", {("k", 3): (str(rec), str(src))})
    assert bench.traffic_per_launch("k", 3) == 123.0
    assert bench.traffic_per_launch("k", 4) is None
    src.write_bytes(b"kernel v2")
    assert bench.traffic_per_launch("k", 3) is None


@pytest.mark.parametrize("kernel", ["sweep_fast_kernel", "oct_tile_kernel"])
def test_committed_traffic_record_matches_the_source(kernel):
    """The committed HBM-traffic records of the config-3 kernels were measured on the
    kernel sources as they stand."""
    assert bench.traffic_per_launch(kernel, 3) is not None


def test_cpu_baseline_report():
    insts = [W.config1(), W.config1()]
    out = bench.cpu_baseline(insts, W.sampler_seed(1), 1, budget_s=0.2, max_threads=2)
    assert out["kind"] == "oracle" and out["unit"] == "spin-flip attempts/s"
    assert 1 <= out["cores"] <= 2 and out["value"] > 0
    assert "instances 0.." in out["sample"]
