"""Host-side checks of bench.py (no GPU): the one-GPU refusal, the counter
traffic tied to the stage-kernel source it was measured on and to the
profile summary that records it, and the host description of the CPU
baseline."""
import hashlib
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILE = os.path.join(ROOT, "profiles", "rk4_stage_kernels_n922_n4096.md")


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test",
                                                  os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""  # no JSON line


def test_counter_traffic_belongs_to_the_current_stage_kernels(monkeypatch):
    b = _bench()
    path, prefix = b.COUNTERS_SRC
    with open(os.path.join(ROOT, path), "rb") as fh:
        digest = hashlib.sha256(fh.read()).hexdigest()
    assert digest.startswith(prefix), (
        "the stage kernels changed since the HBM counters were taken: take them again "
        "(the commands are in the profile summary) and update COUNTERS_SRC and TRAFFIC_N922")
    for kernel in ("fused", "epilogue", "spmm"):
        assert b.measured_traffic(kernel) == b.TRAFFIC_N922[kernel]
    monkeypatch.setattr(b, "COUNTERS_SRC", (path, "0" * 16))
    assert b.measured_traffic("fused") is None


def test_counter_figures_match_the_profile_summary():
    b = _bench()
    with open(PROFILE) as fh:
        text = fh.read()
    assert b.COUNTERS_SRC[1] in text
    heads = {"fused": "fused FP64 | 922", "epilogue": "epilogue FP64 | 922",
             "spmm": "sparse product FP64 (`k_spmm`) | 922"}
    for kernel, head in heads.items():
        line = next(l for l in text.splitlines() if l.startswith("| " + head + " |"))
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        fetch_kib = float(cells[2].replace(",", ""))
        write_kib = float(cells[4].replace(",", ""))
        # FETCH_SIZE x 2.00 and WRITE_SIZE x 1.00, the copy-kernel calibration
        assert b.TRAFFIC_N922[kernel] == pytest.approx((2.0 * fetch_kib + write_kib) * 1024.0,
                                                       rel=1e-12)


def test_cpu_baseline_states_its_host():
    h = _bench().host_cpu()
    assert h["cpu_count"] == os.cpu_count()
    assert isinstance(h["cpu_model"], str) and h["cpu_model"]
    assert h["blas_threads"] >= 1
