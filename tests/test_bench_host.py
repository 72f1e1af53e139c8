"""Host-side checks of bench.py (no GPU): the one-GPU guard, the argument
surface, and the counted-traffic record that is reported only for the kernel
sources it was counted on."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench_module():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_defaults_and_options(monkeypatch):
    b = _bench_module()
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    a = b.parse()
    assert (a.gpus, a.steps, a.warmup, a.workload, a.precision, a.law, a.damping) == \
        (1, 3, 1, "d6-hcmax16-allen-cahn", "f64", "logistic", 0.0)
    monkeypatch.setattr(sys, "argv", ["bench.py", "--law", "cauchy", "--damping", "2", "--precision", "bf16"])
    a = b.parse()
    assert (a.law, a.damping, a.precision) == ("cauchy", 2.0, "bf16")


def test_counted_traffic_only_for_its_sources(monkeypatch):
    b = _bench_module()
    # unknown workloads or sizes carry no counted traffic
    assert b.counted_traffic("d6-hcmax16-allen-cahn", "f64", 1 << 18) == (None, None)
    assert b.counted_traffic("d6-hcmax16-allen-cahn", "bf16", 1 << 20) == (None, None)
    # a recorded figure is reported only while the sources hash to its value
    key = ("d6-hcmax16-allen-cahn", "f64", 1 << 20)
    rd, wr, sha = b.COUNTED_TRAFFIC[key]
    monkeypatch.setattr(b, "kernel_sources_sha256", lambda: sha)
    total, detail = b.counted_traffic(*key)
    assert total == rd + wr and detail["read_bytes"] == rd and detail["written_bytes"] == wr
    monkeypatch.setattr(b, "kernel_sources_sha256", lambda: "0" * 64)
    assert b.counted_traffic(*key) == (None, None)
