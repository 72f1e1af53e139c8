"""Host-side checks of bench.py (no GPU): the one-GPU guard, the argument
surface, and the counted-traffic record that is reported only for the kernel
sources it was counted on."""
import importlib.util
import json
import math
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
    assert (a.gpus, a.steps, a.warmup, a.workload, a.precision, a.prec_kernel, a.law, a.damping) == \
        (1, 3, 1, "d6-hcmax16-allen-cahn", "bf16", "auto", "logistic", 0.0)
    monkeypatch.setattr(sys, "argv", ["bench.py", "--law", "cauchy", "--damping", "2", "--precision", "f64"])
    a = b.parse()
    assert (a.law, a.damping, a.precision) == ("cauchy", 2.0, "f64")


def test_projection_floor_of_the_workloads():
    """The projection floor used in the error split: relative squared
    distance of u(0, .) to the span of the basis.  Against values computed
    independently when the workloads were planned (0.169 for the d = 2
    tensor set, 0.194 for the d = 6 hyperbolic cross), ||u||^2 in closed form
    (E cos^2 through the logistic characteristic function pi t / sinh(pi t)),
    and the floor falling strictly with the level of nested sets."""
    import workloads as W
    import oracle as O
    b = _bench_module()
    f2, u2 = b.projection_floor(W.D2_TENSOR4, O.reps_for(W.D2_TENSOR4))
    assert abs(f2 - 0.169) < 1e-3
    assert abs(u2 - 0.5 * math.exp(-2.0) * (1.0 + (2 * math.pi / math.sinh(2 * math.pi)) ** 2)) < 1e-12
    f6, _ = b.projection_floor(W.D6_HCMAX16, O.reps_for(W.D6_HCMAX16))
    assert abs(f6 - 0.194) < 1e-3
    floors = [b.projection_floor(W.D2_TENSOR4.with_(level=k), O.reps_for(W.D2_TENSOR4.with_(level=k)))[0]
              for k in (1, 2, 4, 8)]
    assert all(0.0 <= f <= 1.0 for f in floors)
    assert all(x > y for x, y in zip(floors, floors[1:]))


def test_counted_traffic_only_for_its_sources(monkeypatch):
    b = _bench_module()
    # unknown workloads or sizes carry no counted traffic
    assert b.counted_traffic("d6-hcmax16-allen-cahn", "f64", 1 << 18) == (None, None)
    assert b.counted_traffic("d2-tensor4", "bf16", 1 << 20) == (None, None)
    # a recorded figure is reported only while the sources of its kernel hash to its value
    for key, kind in ((("d6-hcmax16-allen-cahn", "f64", 1 << 20), "f64"),
                      (("d6-hcmax16-allen-cahn", "bf16", 1 << 20), "factored")):
        sha = b.kernel_sources_sha256(kind)
        monkeypatch.setitem(b.COUNTED_TRAFFIC, key, (1000, 300, sha))
        total, detail = b.counted_traffic(*key)
        assert total == 1300 and detail["read_bytes"] == 1000 and detail["written_bytes"] == 300
        monkeypatch.setattr(b, "kernel_sources_sha256", lambda kind="f64": "0" * 64)
        assert b.counted_traffic(*key) == (None, None)
        monkeypatch.undo()
    # the two kernels hash different sources
    assert b.kernel_sources_sha256("f64") != b.kernel_sources_sha256("factored")


def test_paper_workloads_are_the_printed_rows():
    """The paper-variant legs are rows of Tables d1_mse / d2_mse: N = 1/Delta,
    the printed cardinalities of the sets over N^d, and the printed M."""
    import workloads as W
    import oracle as O
    b = _bench_module()
    want = {"paper-d1-tensor100": (20, 101, 20_000), "paper-d1-tensor150": (50, 151, 200_000),
            "paper-d1-tensor200": (100, 201, 2_000_000),
            "paper-d2-total20": (20, 231, 20_000), "paper-d2-hc_max19": (20, 99, 20_000),
            "paper-d2-total25": (50, 351, 200_000), "paper-d2-hc_max24": (50, 133, 200_000),
            "paper-d2-total31": (100, 528, 2_000_000), "paper-d2-hc_max30": (100, 172, 2_000_000)}
    for name, (N, card, M) in want.items():
        w = W.ALL[name]
        assert (w.N, O.reps_for(w).shape[0], w.M) == (N, card, M)
        assert w.basis == "cosine" and w.law == "student2" and w.driver == "paper"
        assert name in b.PAPER_CONTEXT
