#!/usr/bin/env python3
"""Benchmark: full-solve time and basis-evals/s of the QRMC solve on one MI355X,
the chosen (reduced-precision, factored) form against the plain FP64 path at
equal L2 error.

Workload (default): d=6, N=20, sigma=0.4 I, b(x)=-0.1 x, standard-logistic
sampling law, hyperbolic cross prod max(1,|k_l|) <= 16 over Z^6
(169,209 basis functions), M=2^20 paths per step, Allen-Cahn driver
y - y^3 + h with u(t,x) = exp(-(T-t)) cos(sum x)/2, T=1, clamp 1, seed 0.

A step is one full backward induction (Algorithm 1, i = N-1..0) in the
chosen form (default bfloat16: the expansion along the paths and the
projection as products of the staircase coefficient matrix with the paths'
basis factors on the matrix cores).  One solve evaluates M |Gamma| N(N+1)/2
basis functions (expansions along the paths plus the projections); value =
that count times the timed solves over the timed wall time, with everything
resident on the GPU.  The plain FP64 solve of the same workload is timed in
the same run; both relative L2 errors at t_0 (closed-form u on 2^16
stream-1 points) are reported with the speed-up, and the FP64 error is split
into the projection floor of the index set and the Monte-Carlo variance of
the coefficients (Lemma 3.1).  The dominant kernel is timed with HIP events
recorded on its launch stream.  The CPU oracle is timed on a bounded sample
of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
FP32_VECTOR_PEAK_TFLOPS = 157.3  # published; packed FP32 (the second half) is not used here
MFMA_16BIT_PEAK_TFLOPS = 2500.0  # dense bf16 / fp16

# HBM bytes per launch of the dominant kernel (mean over the launches of one
# solve), from rocprofv3 FETCH_SIZE and WRITE_SIZE counter runs of
# `bench.py --steps 1 --warmup 0 --no-cpu-baseline --copy-calibration-mib 256`
# (with --precision f64 for the plain path), scaled by what the same counters
# read for the plain 256 MiB device copy in that run (FETCH_SIZE x 2.0,
# WRITE_SIZE x 1.0).  A figure holds only for the kernel sources it was
# counted on (their SHA-256); after any change to them the bench reports null
# until the counters are taken again.
_CSRC = "paper_2407_21084_amd/csrc/"
KERNEL_SOURCES = {
    "f64": tuple(_CSRC + f for f in ("qrmc_common.h", "qrmc_device.h", "qrmc_kernels.h", "qrmc_kernels.hip")),
    "factored": tuple(_CSRC + f for f in ("qrmc_common.h", "qrmc_device.h", "qrmc_factored.h",
                                          "qrmc_factored.hip")),
}
COUNTED_TRAFFIC = {
    # (workload, precision, M): read bytes, written bytes, sources counted on
    ("d6-hcmax16-allen-cahn", "bf16", 1 << 20): (1604766688, 260522874,
        "421db16bd2f4b9a7ce77163205370f4ba374ecddd38720fabf6a11b8318df413"),
    ("d6-hcmax16-allen-cahn", "f64", 1 << 20): (2354062624, 1137811482,
        "6620aabad9b3a9b9dedd5b453d760910011e1eaeeb5275747ec162e91acd51bb"),
}


def kernel_sources_sha256(kind: str = "f64") -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kind]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counted_traffic(workload: str, precision: str, M: int):
    """(read + written bytes per launch, detail) if counted on these sources, else (None, None)."""
    rec = COUNTED_TRAFFIC.get((workload, precision, M))
    if rec is None or rec[2] != kernel_sources_sha256("f64" if precision == "f64" else "factored"):
        return None, None
    return float(rec[0] + rec[1]), {"read_bytes": rec[0], "written_bytes": rec[1],
                                    "scaling": "FETCH_SIZE x2.0, WRITE_SIZE x1.0 (256 MiB copy)"}


# The paper's own figures for its Tables d1_mse / d2_mse rows (Sec. 5): GPU
# full-solve seconds on one GeForce GTX TITAN Black in single precision, and
# (MSE_max, MSE_av) of eq (mse) (natural logs) per damping exponent q.
# Context only: other hardware, other precision, other random numbers, and
# the paper averages its indicators over 10^3 independent runs.
PAPER_CONTEXT = {
    "paper-d1-tensor100": {"gpu_s": 0.09, "table": "d1_mse", "mse": {0.0: (-3.658, -3.868), 2.1: (-4.615, -4.874),
                                                                      5.1: (-4.517, -5.130), 8.1: (-4.781, -5.319)}},
    "paper-d1-tensor150": {"gpu_s": 7.37, "table": "d1_mse", "mse": {0.0: (-4.427, -4.900), 2.1: (-6.450, -6.740),
                                                                      5.1: (-6.685, -7.094), 8.1: (-6.740, -7.221)}},
    "paper-d1-tensor200": {"gpu_s": 414.44, "table": "d1_mse", "mse": {0.0: (-4.704, -5.524), 2.1: (-8.465, -8.729),
                                                                        5.1: (-8.717, -9.096), 8.1: (-8.830, -9.301)}},
    "paper-d2-total20": {"gpu_s": 0.33, "table": "d2_mse", "mse": {0.0: (-2.322, -2.773), 5.1: (-4.646, -5.239)}},
    "paper-d2-hc_max19": {"gpu_s": 0.16, "table": "d2_mse", "mse": {0.0: (-2.526, -3.062), 5.1: (-5.588, -6.196)}},
    "paper-d2-total25": {"gpu_s": 35.51, "table": "d2_mse", "mse": {0.0: (-2.869, -3.688), 5.1: (-6.761, -7.186)}},
    "paper-d2-hc_max24": {"gpu_s": 12.38, "table": "d2_mse", "mse": {0.0: (-2.745, -3.550), 5.1: (-7.487, -8.191)}},
    "paper-d2-total31": {"gpu_s": 2243.06, "table": "d2_mse", "mse": {0.0: (-2.978, -3.966), 5.1: (-8.793, -9.107)}},
    "paper-d2-hc_max30": {"gpu_s": 662.54, "table": "d2_mse", "mse": {0.0: (-2.898, -3.770), 5.1: (-9.389, -10.137)}},
}


def paper_indicators(ctx, basis, w, alpha, torch, dev, stream, n=1 << 14):
    """MSE_max and MSE_av of eq (mse) (natural logs) on n stream-1 points of
    the law per time index, and ybar_0 at the origin.  With damping q > 0 the
    paper's indicators compare the damped quantities y_i / D = u(t_i, .) / D
    with the expansion ybar_i (the "_damped" keys); the undamped keys compare
    u with ybar_i D, as the oracle's error indicators do."""
    xt = torch.empty((w.d, n), dtype=torch.float64, device=dev)
    yt = torch.empty(n, dtype=torch.float64, device=dev)
    wv = torch.tensor(w.sol_w, dtype=torch.float64, device=dev)
    per, per_d = [], []
    for i in range(w.N):
        ctx.sample_points(w.d, w.seed, 1, i, n, xt, stream=stream, law=w.law)
        ctx.eval(basis, alpha[i].contiguous(), xt, yt, stream=stream)
        D = (1.0 + (xt * xt).sum(dim=0)) ** (0.5 * w.damping_q) if w.damping_q else None
        t = i * w.T / w.N
        u = w.sol_B + w.sol_A * math.exp(-w.sol_c * (w.T - t)) * torch.cos(wv @ xt + w.sol_p)
        per.append(float(((yt * D - u if D is not None else yt - u) ** 2).mean()))
        if D is not None:
            per_d.append(float(((yt - u / D) ** 2).mean()))
    x0 = torch.zeros((w.d, 1), dtype=torch.float64, device=dev)
    y0 = torch.empty(1, dtype=torch.float64, device=dev)
    ctx.eval(basis, alpha[0].contiguous(), x0, y0, stream=stream)
    torch.cuda.synchronize()
    out = {"mse_max": math.log(max(per)), "mse_av": math.log(sum(per) / len(per)),
           "ybar0_at_0": float(y0[0]), "u0_at_0": w.sol_B + w.sol_A * math.exp(-w.sol_c * w.T) * math.cos(w.sol_p),
           "test_points_per_step": n}
    if per_d:
        out["mse_max_damped"] = math.log(max(per_d))
        out["mse_av_damped"] = math.log(sum(per_d) / len(per_d))
    return out


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="d6-hcmax16-allen-cahn")
    ap.add_argument("--M", type=int, default=None, help="override paths per step")
    ap.add_argument("--precision", default="bf16", choices=["f64", "bf16", "f16"],
                    help="arithmetic of the chosen form (f64: the plain path alone)")
    ap.add_argument("--prec-kernel", default="auto", choices=["auto", "walk", "factored"],
                    help="kernel of the reduced-precision form")
    ap.add_argument("--law", default="logistic", choices=["logistic", "student2", "cauchy"],
                    help="sampling law nu of the basis and of the start draws")
    ap.add_argument("--damping", type=float, default=0.0,
                    help="damping exponent q of the plain FP64 solve")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=30.0)
    ap.add_argument("--cpu-plan", action="store_true",
                    help="time the CPU oracle on every configuration (no GPU work) and exit")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one plain device copy of this size (for counter scaling)")
    return ap.parse_args()


def cpu_baseline(w, target_s: float):
    """The oracle, as it stands, on one backward step of the same workload
    with a reduced cloud; evals counted as on the GPU (M' |Gamma| (N - i))."""
    import numpy as np
    import oracle as O
    reps = O.reps_for(w)
    nf = O.nfuncs(reps)
    alpha = np.zeros((w.N, nf))
    rng = np.random.default_rng(0)
    alpha[w.N - 1] = rng.standard_normal(nf) * 1e-3
    i = w.N - 2
    M1 = 256
    t0 = time.perf_counter()
    O.backward_step(w, reps, i, M1, w.seed, alpha.copy())
    t1 = time.perf_counter() - t0
    M2 = max(M1, int(M1 * target_s / max(t1, 1e-3)))
    t0 = time.perf_counter()
    O.backward_step(w, reps, i, M2, w.seed, alpha.copy())
    dt = time.perf_counter() - t0
    evals = M2 * nf * (w.N - i)
    rate = evals / dt
    full = w.M * nf * w.N * (w.N + 1) / 2
    return {"value": rate, "unit": "basis-evals/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"one backward step i=N-2 with M'={M2} paths (full |Gamma|={nf}); "
                      f"{dt:.1f} s", "seconds": dt, "cpu_model": cpu_model(),
            "full_solve_s_extrapolated": full / rate,
            "extrapolation": "linear in M |Gamma| N(N+1)/2 basis-evals at the sampled rate"}


def cpu_plan(seconds: float):
    """The oracle on the host cores for every configuration: the d = 2
    workload's full solve as it stands, and one backward step (i = N-2) of
    each larger one on a cloud sized to about `seconds`, with the full solve
    extrapolated linearly in M |Gamma| N(N+1)/2 basis-evals."""
    import numpy as np
    import oracle as O
    import workloads as W
    legs = []
    w = W.D2_TENSOR4
    reps = O.reps_for(w)
    t0 = time.perf_counter()
    O.solve(w, reps)
    dt = time.perf_counter() - t0
    evals = w.M * O.nfuncs(reps) * w.N * (w.N + 1) / 2
    legs.append({"workload": w.name, "kind": "full solve", "M": w.M, "seconds": dt, "basis_evals_per_s": evals / dt})
    print(f"[bench] cpu plan: {w.name} full solve {dt:.2f} s", file=sys.stderr, flush=True)
    for w in (W.D6_HCMAX16, W.D10_HC1P32_ZRAT, W.D16_HC1P32):
        r = cpu_baseline(w, seconds)
        legs.append({"workload": w.name, "kind": "one step i=N-2", "sample": r["sample"], "seconds": r["seconds"],
                     "basis_evals_per_s": r["value"], "full_solve_s_extrapolated": r["full_solve_s_extrapolated"]})
        print(f"[bench] cpu plan: {w.name} {r['seconds']:.1f} s", file=sys.stderr, flush=True)
    return {"metric": "CPU oracle timing plan", "cores": O.num_threads(), "cpu_model": cpu_model(),
            "kind": "oracle", "legs": legs,
            "extrapolation": "linear in M |Gamma| N(N+1)/2 basis-evals at the sampled rate"}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# ---------------------------------------------------------------------------
# Error split of the FP64 solve at t_0 (Lemma 3.1 / Thm 3.2): the
# projection floor of the index set, ||u - P_Gamma u||^2 / ||u||^2 for the
# closed-form u(0, .), and the Monte-Carlo variance of the coefficients,
# sum_k Var(alpha_0,k) / ||u||^2.  With the orthonormal real basis,
# sum_k phi_k(x)^2 = |Gamma| at every x, so sum_k E[(S phi_k)^2] = |Gamma| E[S^2]
# and the variance sum is estimated by (|Gamma| mean(S^2) - ||alpha_0||^2) / M.
# ---------------------------------------------------------------------------
def _logistic_1d(a, mmax):
    """c_m(a) = E[e^{i a X} e^{-2 pi i m F(X)}] for standard logistic X,
    m = -mmax..mmax, by the trapezoid rule on [-60, 60]."""
    import numpy as np
    x = np.linspace(-60.0, 60.0, 240001)
    F = 0.5 * (1.0 + np.tanh(0.5 * x))
    dens = F * (1.0 - F)
    m = np.arange(-mmax, mmax + 1)[:, None]
    vals = np.exp(1j * a * x)[None, :] * np.exp(-2j * np.pi * m * F[None, :]) * dens[None, :]
    return np.trapezoid(vals, x, axis=1)


def projection_floor(w, reps) -> float:
    """Relative squared L2(nu) distance of u(0, .) to the span of the basis
    (standard logistic law, manufactured solution A e^{-c T} cos(w.x + p))."""
    import numpy as np
    A = w.sol_A * math.exp(-w.sol_c * w.T)
    full = np.concatenate([reps, -reps[1:]], axis=0)
    mmax = int(np.abs(full).max())
    uhat = np.zeros(full.shape[0], dtype=complex)
    for sgn in (1.0, -1.0):
        prod = np.ones(full.shape[0], dtype=complex)
        cache = {}
        for l in range(w.d):
            a = sgn * w.sol_w[l]
            if a not in cache:
                cache[a] = _logistic_1d(a, mmax)
            prod *= cache[a][full[:, l] + mmax]
        uhat += 0.5 * A * np.exp(1j * sgn * w.sol_p) * prod
    proj2 = float(np.sum(np.abs(uhat) ** 2))
    phi2 = 1.0
    for l in range(w.d):
        t = 2.0 * w.sol_w[l]
        phi2 *= 1.0 if t == 0.0 else math.pi * t / math.sinh(math.pi * t)
    u2 = 0.5 * A * A * (1.0 + math.cos(2.0 * w.sol_p) * phi2)
    return max(0.0, 1.0 - proj2 / u2), u2


BATCHED = "batched-256"
LEARNED = "learned-d16"


def run_learned(args, torch, W, Q):
    """The learned form on the d=16 workload (prod(1+|k_l|) <= 32, 599,969
    functions, Allen-Cahn driver) at a reduced cloud (--M, default 2^16):
    the plain FP64 solve, the learned solve (surrogate per time index,
    gate 1e-3), and the cost of one evaluation of ybar by the expansion and
    by the network on 2^20 points."""
    dev = torch.device("cuda:0")
    w = W.D16_HC1P32.with_(M=args.M or (1 << 16))
    ctx = Q.Context(0)
    b = Q.Basis(w.d, w.set_kind, w.level)
    prob = Q.problem_from(w)
    stream = torch.cuda.current_stream()
    n_test = 1 << 16
    xt = torch.empty((w.d, n_test), dtype=torch.float64, device=dev)
    ctx.sample_points(w.d, w.seed, 1, 0, n_test, xt, stream=stream)
    wv = torch.tensor(w.sol_w, dtype=torch.float64, device=dev)
    u0 = w.sol_B + w.sol_A * math.exp(-w.sol_c * w.T) * torch.cos(wv @ xt + w.sol_p)

    def rel_err(a):
        yt = torch.empty(n_test, dtype=torch.float64, device=dev)
        ctx.eval(b, a[0].contiguous(), xt, yt, stream=stream)
        return float(torch.linalg.norm(yt - u0) / torch.linalg.norm(u0))

    a64 = torch.zeros((w.N, b.n_funcs), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.solve(prob, b, w.M, w.seed, a64, stream)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    print(f"[bench] plain solve {t_plain:.1f} s", file=sys.stderr, flush=True)
    al = torch.zeros_like(a64)
    t0 = time.perf_counter()
    rep = ctx.solve_learned(prob, b, w.M, w.seed, al, stream=stream, reject=0.5)
    torch.cuda.synchronize()
    t_learned = time.perf_counter() - t0
    print(f"[bench] learned solve {t_learned:.1f} s", file=sys.stderr, flush=True)
    # the same without the screen: every time index runs the full fit
    af = torch.zeros_like(a64)
    t0 = time.perf_counter()
    rep_full = ctx.solve_learned(prob, b, w.M, w.seed, af, stream=stream, reject=0.0)
    torch.cuda.synchronize()
    t_full = time.perf_counter() - t0
    print(f"[bench] learned solve without the screen {t_full:.1f} s", file=sys.stderr, flush=True)
    # cost of one evaluation of ybar_j at 2^20 points: expansion vs network
    n = 1 << 20
    x = torch.empty((w.d, n), dtype=torch.float64, device=dev)
    ctx.sample_points(w.d, w.seed, 1, 1, n, x, stream=stream)
    y = torch.empty(n, dtype=torch.float64, device=dev)
    feat = torch.empty((n, 16), dtype=torch.float32, device=dev)
    y32 = torch.empty(n, dtype=torch.float32, device=dev)
    th = torch.empty(Q.MLP_NPARAMS, dtype=torch.float32, device=dev)
    ctx.mlp_init(th, 1, stream=stream)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ctx.eval(b, a64[1].contiguous(), x, y, stream=stream)            # warm
    ctx.mlp_features(w.d, x, feat, stream=stream)
    ctx.mlp_forward(th, feat, y32, stream=stream)
    ev[0].record(stream)
    ctx.eval(b, a64[1].contiguous(), x, y, stream=stream)
    ev[1].record(stream)
    ctx.mlp_features(w.d, x, feat, stream=stream)
    ctx.mlp_forward(th, feat, y32, stream=stream)
    ev[2].record(stream)
    torch.cuda.synchronize()
    t_exp, t_net = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
    line = {
        "metric": "full-solve time, learned form vs plain FP64 (d=16, reduced cloud)",
        "value": t_learned, "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": t_learned * 1e3, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64+bf16", "data": "synthetic",
        "config": {"workload": LEARNED, "d": w.d, "N": w.N, "n_funcs": b.n_funcs, "M": w.M,
                   "train_points": 1 << 18, "heldout_points": 1 << 16, "epochs": 8, "gate": 1e-3,
                   "reject": 0.5},
        "plain_solve_s": t_plain, "learned_solve_s": t_learned,
        "rel_l2_t0": {"plain": rel_err(a64), "learned": rel_err(al)},
        "surrogates_used": sum(r["used"] for r in rep),
        "epochs_run": [r["epochs_run"] for r in rep[1:]],
        "learned_equals_plain": bool(torch.equal(al, a64)),
        "overhead_vs_plain": t_learned / t_plain - 1.0,
        "without_screen": {"learned_solve_s": t_full, "overhead_vs_plain": t_full / t_plain - 1.0,
                           "surrogates_used": sum(r["used"] for r in rep_full),
                           "equals_plain": bool(torch.equal(af, a64)),
                           "heldout_rel_l2": {"min": min(r["heldout_rel_l2"] for r in rep_full[1:]),
                                              "max": max(r["heldout_rel_l2"] for r in rep_full[1:])}},
        "heldout_rel_l2": {"min": min(r["heldout_rel_l2"] for r in rep[1:]),
                           "max": max(r["heldout_rel_l2"] for r in rep[1:])},
        "eval_2p20_points_ms": {"expansion": t_exp, "network": t_net, "ratio": t_exp / t_net},
    }
    print(json.dumps(line), flush=True)
    ctx.close()


ZREG = "z-d6"


def run_z(args, torch, W, Q):
    """The gradient component on the d=6 workload (hyperbolic cross 16,
    169,209 functions, Allen-Cahn, M = 2^20 unless --M): the plain FP64
    solve, then the solve with the Z regression of eq (MDP:intro:0a), and
    the relative L2 errors of Y_0 and Z_0 against u(t_0) and sigma^T grad u(t_0)."""
    dev = torch.device("cuda:0")
    w = W.D6_HCMAX16.with_(M=args.M or W.D6_HCMAX16.M)
    ctx = Q.Context(0)
    b = Q.Basis(w.d, w.set_kind, w.level)
    prob = Q.problem_from(w)
    stream = torch.cuda.current_stream()
    n_test = 1 << 16
    xt = torch.empty((w.d, n_test), dtype=torch.float64, device=dev)
    ctx.sample_points(w.d, w.seed, 1, 0, n_test, xt, stream=stream)
    wv = torch.tensor(w.sol_w, dtype=torch.float64, device=dev)
    sig = torch.tensor(w.sigma, dtype=torch.float64, device=dev)
    e0 = math.exp(-w.sol_c * w.T)
    u0 = w.sol_B + w.sol_A * e0 * torch.cos(wv @ xt + w.sol_p)
    z0 = sig.T @ (-w.sol_A * e0 * torch.sin(wv @ xt + w.sol_p)[None, :] * wv[:, None])  # [nbm][n]

    def timed_solve(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    a64 = torch.zeros((w.N, b.n_funcs), dtype=torch.float64, device=dev)
    t_plain = timed_solve(lambda: ctx.solve(prob, b, w.M, w.seed, a64, stream))
    print(f"[bench] plain solve {t_plain:.2f} s", file=sys.stderr, flush=True)
    runs = {}
    for scheme in ("multistep", "onestep"):
        az = torch.zeros((w.N, w.nbm, b.n_funcs), dtype=torch.float64, device=dev)
        ay = torch.zeros_like(a64)
        ctx.set_timing(True)
        ctx.reset_timing()
        t_z = timed_solve(lambda: ctx.solve_z(prob, b, w.M, w.seed, ay, az, scheme=scheme, stream=stream))
        ktime = {name: ctx.kernel_time(k)[0] for k, name in enumerate(("path", "projection", "reduction"))}
        ctx.set_timing(False)
        print(f"[bench] solve with Z ({scheme}) {t_z:.2f} s", file=sys.stderr, flush=True)
        y = torch.empty(n_test, dtype=torch.float64, device=dev)
        ctx.eval(b, ay[0].contiguous(), xt, y, stream=stream)
        ez = torch.empty((w.nbm, n_test), dtype=torch.float64, device=dev)
        for k in range(w.nbm):
            ctx.eval(b, az[0, k].contiguous(), xt, ez[k], stream=stream)
        torch.cuda.synchronize()
        runs[scheme] = {"z_solve_s": t_z, "overhead_vs_plain": t_z / t_plain - 1.0, "kernel_ms": ktime,
                        "y_equals_plain": bool(torch.equal(ay, a64)),
                        "rel_l2_t0": {"y": float(torch.linalg.norm(y - u0) / torch.linalg.norm(u0)),
                                      "z": float(torch.linalg.norm(ez - z0) / torch.linalg.norm(z0))}}
    t_z = runs["multistep"]["z_solve_s"]
    line = {
        "metric": "full-solve time with the Z regression (multistep scheme) vs plain FP64 (d=6)",
        "value": t_z, "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": t_z * 1e3, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": ZREG, "d": w.d, "nbm": w.nbm, "N": w.N, "n_funcs": b.n_funcs, "M": w.M},
        "plain_solve_s": t_plain, "schemes": runs,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


def run_batched(args, torch, W, Q):
    """The batched form: 256 instances (d ~ U{2..12}, M in {2^14..2^20},
    level in {8,16,32}, hyperbolic cross prod(1+|k_l|), sin driver with
    per-instance c_j) in groups of 64 sharing one cloud.  A step solves all
    groups; evals are counted per instance (M_r |Gamma_r| N(N+1)/2)."""
    import numpy as np
    dev = torch.device("cuda:0")
    insts = W.batched_instances()
    groups = W.batched_group(insts)
    ctx = Q.Context(0)
    stream = torch.cuda.current_stream()
    runs = []
    evals = 0.0
    path_evals_step = 0.0
    for gw, inst, _ in groups:
        b = Q.Basis(gw.d, gw.set_kind, gw.level)
        a = torch.zeros((len(inst), gw.N, b.n_funcs), dtype=torch.float64, device=dev)
        runs.append((gw, inst, b, a))
        for (_, d, L, M) in inst:
            nf = Q.Basis(d, gw.set_kind, L).n_funcs
            evals += M * nf * gw.N * (gw.N + 1) / 2
            path_evals_step += M * nf * gw.N * (gw.N - 1) / 2

    def step():
        for gw, inst, b, a in runs:
            ctx.solve_batched(Q.problem_from(gw), b, inst, gw.seed, a, stream)

    for k in range(args.warmup):
        step()
        torch.cuda.synchronize()
        print(f"[bench] warmup step {k + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    ctx.reset_timing()
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.set_timing(False)
    path_ms, path_n = ctx.kernel_time(Q.K_PATH)
    proj_ms, proj_n = ctx.kernel_time(Q.K_PROJECT)
    red_ms, _ = ctx.kernel_time(Q.K_REDUCE)
    path_evals = path_evals_step * args.steps
    print(f"[bench] timed region {elapsed:.2f} s", file=sys.stderr, flush=True)

    # accuracy of every instance at t_0 against its closed form (stream-1 points)
    n_test = 1 << 14
    rels = []
    for gw, inst, b, a in runs:
        xt = torch.empty((gw.d, n_test), dtype=torch.float64, device=dev)
        ctx.sample_points(gw.d, gw.seed, 1, 0, n_test, xt, stream=stream)
        u0 = math.exp(-1.0) * torch.cos(xt[0] + xt[1])
        yt = torch.empty(n_test, dtype=torch.float64, device=dev)
        for r in range(len(inst)):
            ctx.eval(b, a[r, 0].contiguous(), xt, yt, stream=stream)
            rels.append(float(torch.linalg.norm(yt - u0) / torch.linalg.norm(u0)))
    torch.cuda.synchronize()
    # the same instances solved one by one with qr_solve (each on its own
    # cloud and basis), on a sample of every 16th: time and error
    sample = list(range(0, len(insts), 16))
    t_plain = 0.0
    rel_plain, rel_batched = [], []
    for k in sample:
        w = insts[k]
        b = Q.Basis(w.d, w.set_kind, w.level)
        a = torch.zeros((w.N, b.n_funcs), dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ctx.solve(Q.problem_from(w), b, w.M, w.seed, a, stream)
        torch.cuda.synchronize()
        t_plain += time.perf_counter() - t1
        xt = torch.empty((w.d, n_test), dtype=torch.float64, device=dev)
        ctx.sample_points(w.d, w.seed, 1, 0, n_test, xt, stream=stream)
        u0 = math.exp(-1.0) * torch.cos(xt[0] + xt[1])
        yt = torch.empty(n_test, dtype=torch.float64, device=dev)
        ctx.eval(b, a[0].contiguous(), xt, yt, stream=stream)
        torch.cuda.synchronize()
        rel_plain.append(float(torch.linalg.norm(yt - u0) / torch.linalg.norm(u0)))
        rel_batched.append(rels[k])
    print(f"[bench] plain solves of {len(sample)} sampled instances {t_plain:.1f} s", file=sys.stderr, flush=True)
    line = {
        "metric": "basis-evals/s (batched form, 256 instances, FP64)",
        "value": evals * args.steps / elapsed,
        "unit": "basis-evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": BATCHED, "instances": len(insts), "groups": len(groups),
                   "evals_per_step": evals},
        "full_solve_s": elapsed / args.steps,
        "rel_l2_t0": {"median": float(np.median(rels)), "max": float(np.max(rels))},
        "vs_plain_solves": {"sample": f"every 16th instance ({len(sample)} of {len(insts)}), each by qr_solve "
                                      "on its own basis and cloud",
                            "plain_s_sample": t_plain,
                            "plain_s_extrapolated": t_plain * len(insts) / len(sample),
                            "batched_s": elapsed / args.steps,
                            "speedup_extrapolated": t_plain * len(insts) / len(sample) / (elapsed / args.steps),
                            "rel_l2_t0_sample": {"plain_median": float(np.median(rel_plain)),
                                                 "batched_median": float(np.median(rel_batched)),
                                                 "plain_max": float(np.max(rel_plain)),
                                                 "batched_max": float(np.max(rel_batched))}},
        "kernels_ms_per_solve": {"path": path_ms / args.steps, "project": proj_ms / args.steps,
                                 "reduce": red_ms / args.steps},
        "launches_per_step": {"path": path_n // max(1, args.steps), "project": proj_n // max(1, args.steps)},
        # algorithmic rate of the walks: 5 flops per instance basis function
        # along the paths (useful work; passes also walk their members'
        # envelopes)
        "roofline": {"bound": "alu", "achieved": path_evals * 5.0 / (path_ms * 1e-3) / 1e12 if path_ms > 0 else 0.0,
                     "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": path_evals * 5.0 / (path_ms * 1e-3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS if path_ms > 0 else 0.0,
                     "traffic": None, "kernel": "batched_path_kernel",
                     "note": "kernel times summed over the four streams the passes run on, which overlap"},
    }
    print(json.dumps(line), flush=True)
    ctx.close()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1 "
                                   "(multi-GPU path sharding is a design note, not built)"}))
        sys.exit(2)
    if args.cpu_plan:
        print(json.dumps(cpu_plan(args.cpu_seconds / 3)), flush=True)
        return
    import torch
    import workloads as W
    from paper_2407_21084_amd import qrmc as Q

    if args.workload == LEARNED:
        run_learned(args, torch, W, Q)
        return
    if args.workload == ZREG:
        run_z(args, torch, W, Q)
        return
    if args.workload == BATCHED:
        if args.precision != "f64":
            sys.exit("the batched form runs in FP64")
        run_batched(args, torch, W, Q)
        return
    w = W.ALL[args.workload]
    if args.law != "logistic":
        w = w.with_(law=args.law, name=f"{w.name}-{args.law}")
    if args.damping:
        w = w.with_(damping_q=args.damping, name=f"{w.name}-q{args.damping:g}")
    if args.M:
        w = w.with_(M=args.M)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ctx = Q.Context(0)
    ctx.set_prec_kernel(args.prec_kernel)
    basis = Q.Basis(w.d, w.set_kind, w.level, law=w.law, basis=w.basis)
    prob = Q.problem_from(w)
    alpha = torch.zeros((w.N, basis.n_funcs), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    factored = args.precision != "f64" and args.prec_kernel != "walk" and w.driver != "zrat" \
        and basis.factored() is not None

    if args.copy_calibration_mib:
        src = torch.empty(args.copy_calibration_mib << 17, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    def solve():
        if args.precision == "f64":
            ctx.solve(prob, basis, w.M, w.seed, alpha, stream)
        else:
            ctx.solve_prec(prob, basis, w.M, w.seed, args.precision, alpha, stream)

    for k in range(args.warmup):
        solve()
        torch.cuda.synchronize()
        print(f"[bench] warmup solve {k + 1}/{args.warmup} done", file=sys.stderr, flush=True)

    ctx.reset_timing()
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        solve()
        if k + 1 < args.steps and args.steps > 1:
            print(f"[bench] timed solve {k + 1}/{args.steps} enqueued", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    print(f"[bench] timed region {elapsed:.2f} s", file=sys.stderr, flush=True)
    ctx.set_timing(False)

    evals_per_solve = w.M * basis.n_funcs * w.N * (w.N + 1) / 2
    value = evals_per_solve * args.steps / elapsed
    path_ms, path_n = ctx.kernel_time(Q.K_PATH)
    proj_ms, proj_n = ctx.kernel_time(Q.K_PROJECT)
    red_ms, red_n = ctx.kernel_time(Q.K_REDUCE)
    # algorithmic work of the dominant kernel (expansions at X_{j+1}, j+1 < N)
    grad = w.driver == "zrat"
    rhs = 1 + (w.d if grad else 0)
    n_reps = (basis.n_funcs + 1) // 2 if w.basis == "fourier" else basis.n_funcs
    path_evals = w.M * basis.n_funcs * w.N * (w.N - 1) / 2 * args.steps
    path_s = path_ms * 1e-3
    mfma = None
    if args.precision == "f64":
        # half a complex multiply of the walk (3 flops) and the contraction
        # (2 flops per right-hand side) per basis function
        flops_per_eval, peak, kernel, bound = 3.0 + 2.0 * rhs, FP64_VECTOR_PEAK_TFLOPS, "path_kernel", "alu"
    elif factored:
        # one complex multiply-add per representative and path on the matrix
        # cores (8 real flops, i.e. 4 per basis function); the padding of the
        # staircase blocks is not counted
        flops_per_eval, peak, kernel, bound = 4.0, MFMA_16BIT_PEAK_TFLOPS, "fac_path_kernel", "mfma"
        split, nrt, nkb, nblocks = basis.factored()
        mfma = {"layout": {"split": split, "row_tiles": nrt, "k_blocks": nkb, "blocks_per_step": nblocks,
                           "padding": nblocks * 128 / n_reps},
                "issued_tflops": w.M * nblocks * 8192 * 2 * w.N * (w.N - 1) / 2 * args.steps / 16 / path_s / 1e12
                if path_s > 0 else 0.0}
    else:
        # walk on the FP32 vector ALU; contraction on the matrix cores
        flops_per_eval, peak, kernel, bound = 3.0, FP32_VECTOR_PEAK_TFLOPS, "mfma_path_kernel", "alu"
        T = 1 if not grad else max((w.d + 4) // 4, 2 if max(w.d, w.nbm) <= 8 else 3)
        issued = path_evals * 2.0 * 4 * T / path_s / 1e12 if path_s > 0 else 0.0
        mfma = {"issued_tflops": issued, "useful_tflops": issued * rhs / (4 * T),
                "peak": MFMA_16BIT_PEAK_TFLOPS}
    achieved = path_evals * flops_per_eval / path_s / 1e12 if path_s > 0 else 0.0
    proj_evals = w.M * basis.n_funcs * w.N * args.steps
    proj_tflops = proj_evals * 5.0 / (proj_ms * 1e-3) / 1e12 if proj_ms > 0 else 0.0

    # accuracy of the last solve against the closed form at t_0 (stream-1 points)
    n_test = 1 << 16
    xt = torch.empty((w.d, n_test), dtype=torch.float64, device=dev)
    ctx.sample_points(w.d, w.seed, 1, 0, n_test, xt, stream=stream, law=w.law)
    wv = torch.tensor(w.sol_w, dtype=torch.float64, device=dev)
    u0 = w.sol_B + w.sol_A * math.exp(-w.sol_c * w.T) * torch.cos(wv @ xt + w.sol_p)

    def rel_l2_of(a):
        yt = torch.empty(n_test, dtype=torch.float64, device=dev)
        ctx.eval(basis, a[0].contiguous(), xt, yt, stream=stream)
        torch.cuda.synchronize()
        if w.damping_q:
            # the coefficients describe y / (1+|x|^2)^{q/2}
            yt = yt * (1.0 + (xt * xt).sum(dim=0)) ** (0.5 * w.damping_q)
        return float(torch.linalg.norm(yt - u0) / torch.linalg.norm(u0))

    rel_l2 = rel_l2_of(alpha)
    traffic, traffic_detail = counted_traffic(w.name, args.precision, w.M)
    form = "plain FP64" if args.precision == "f64" else \
        f"{args.precision} {'factored' if factored else 'walk'} form"
    line = {
        "metric": "basis-evals/s (plain FP64 full solve)" if args.precision == "f64"
                  else f"basis-evals/s & full-solve time at fixed L2 error: {form} vs plain FP64",
        "value": value,
        "unit": "basis-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": w.name, "form": form, "d": w.d, "N": w.N, "set": f"{w.set_kind}({w.level})",
                   "n_funcs": basis.n_funcs, "M": w.M, "evals_per_solve": evals_per_solve},
        "full_solve_s": elapsed / args.steps,
        "rel_l2_t0": rel_l2,
        "kernels_ms_per_solve": {"path": path_ms / args.steps, "project": proj_ms / args.steps,
                                 "reduce": red_ms / args.steps},
        "roofline": {"bound": bound, "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": traffic, "kernel": kernel,
                     "flops_per_eval": flops_per_eval,
                     "avg_launch_ms": path_ms / max(1, path_n),
                     "project_tflops": proj_tflops},
    }
    if traffic_detail:
        line["roofline"]["traffic_unit"] = "bytes per launch"
        line["roofline"]["traffic_detail"] = traffic_detail
    if mfma:
        line["mfma"] = mfma
    a64 = alpha
    if args.precision != "f64":
        # the plain FP64 solve of the same workload: its time and its error at
        # t_0 (the target of "equal L2 error"), and the reduced-precision
        # coefficients' error per time step
        a64 = torch.zeros_like(alpha)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.solve(prob, basis, w.M, w.seed, a64, stream)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t0
        print(f"[bench] plain FP64 solve {t64:.1f} s", file=sys.stderr, flush=True)
        rel64 = rel_l2_of(a64)
        rows = (torch.linalg.norm(alpha - a64, dim=1) / torch.linalg.norm(a64, dim=1).clamp_min(1e-300)).tolist()
        line["vs_plain_fp64"] = {
            "fp64_full_solve_s": t64, "fp64_basis_evals_per_s": evals_per_solve / t64,
            "speedup_at_equal_error": t64 / (elapsed / args.steps),
            "rel_l2_t0": {args.precision: rel_l2, "f64": rel64},
            "equal_error": rel_l2 <= 1.02 * rel64,
            "alpha_rel_err_per_step": rows}
    if w.law == "logistic" and not w.damping_q and w.basis == "fourier":
        # error split of the FP64 solve at t_0: projection floor + Monte-Carlo variance
        floor, u2 = projection_floor(w, basis.indices())
        s0 = torch.empty(w.M, dtype=torch.float64, device=dev)
        ctx.path_responses(prob, basis, 0, w.M, w.seed, a64, s0, stream=stream)
        torch.cuda.synchronize()
        ms2 = float((s0 * s0).mean())
        a2 = float((a64[0] * a64[0]).sum())
        var_rel = max(0.0, (basis.n_funcs * ms2 - a2) / w.M) / u2
        meas = line["vs_plain_fp64"]["rel_l2_t0"]["f64"] if "vs_plain_fp64" in line else rel_l2
        line["error_split_f64"] = {
            "rel_l2_t0_squared": meas * meas,
            "projection_floor": floor,
            "mc_variance": var_rel,
            "remainder": meas * meas - floor - var_rel,
            "note": "relative squared L2(nu) errors at t_0: ||u - P_Gamma u||^2/||u||^2 by 1-D quadrature of the "
                    "closed form, and sum_k Var(alpha_0k)/||u||^2 = (|Gamma| mean(S^2) - ||alpha_0||^2)/(M ||u||^2) "
                    "from the responses of step 0; the remainder holds the errors carried from later steps and "
                    "the time discretisation"}
    if w.basis == "cosine":
        line["paper_indicators"] = paper_indicators(ctx, basis, w, alpha, torch, dev, stream)
        if a64 is not alpha:
            line["paper_indicators_f64"] = paper_indicators(ctx, basis, w, a64, torch, dev, stream)
        base = w.name.split("-q")[0]
        if base in PAPER_CONTEXT:
            ctxp = PAPER_CONTEXT[base]
            mse = ctxp["mse"].get(round(w.damping_q, 1))
            line["paper_context"] = {"table": ctxp["table"], "gpu_s": ctxp["gpu_s"], "q": w.damping_q,
                                     "mse_max": mse[0] if mse else None, "mse_av": mse[1] if mse else None,
                                     "hardware": "1x GeForce GTX TITAN Black, single precision"}
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
