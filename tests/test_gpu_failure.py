"""Failure handling and recovery on the GPU: a full solve is its backward
steps (Algorithm 1) run one by one, a solve interrupted after time index k
resumes from the saved rows k+1..N-1 with the same result bit for bit, and a
workspace cap turns a would-be allocation into QR_ENOMEM before anything is
launched (the condition is forced from the host; no device allocation
actually fails)."""
import numpy as np
import pytest

import workloads as W
from gpu_common import dev, env, host, say  # noqa: F401 (env is a fixture)

pytestmark = pytest.mark.gpu


def test_solve_equals_its_steps(env):
    Q, ctx, torch = env
    w = W.D2_TENSOR4
    say(f"solve vs steps {w.name}")
    b = Q.Basis(w.d, w.set_kind, w.level)
    p = Q.problem_from(w)
    a = torch.zeros((w.N, b.n_funcs), dtype=torch.float64, device="cuda")
    ctx.solve(p, b, w.M, w.seed, a)
    s = torch.zeros_like(a)
    for i in range(w.N - 1, -1, -1):
        ctx.backward_step(p, b, i, w.M, w.seed, s)
    torch.cuda.synchronize()
    assert torch.equal(a, s)


RESUME = [("f64", "auto", "fourier"), ("bf16", "factored", "fourier"), ("f16", "walk", "fourier"),
          ("f64", "auto", "cosine"), ("bf16", "factored", "cosine")]


@pytest.mark.parametrize("prec,kernel,basis", RESUME, ids=["-".join(c) for c in RESUME])
def test_resume_from_saved_rows_is_bit_exact(env, prec, kernel, basis):
    Q, ctx, torch = env
    if basis == "cosine":
        w = W.paper_benchmark(3, 6, "total", 5, 3000)
    else:
        w = W.Workload(name="resume-d3", d=3, N=6, T=1.0, sigma=[[0.5 if r == c else 0.0 for c in range(3)]
                                                                 for r in range(3)],
                       b0=[0.0] * 3, b1=[-0.1] * 3, set_kind="hc_1p", level=12, M=3000, driver="allen_cahn",
                       f_a=0.0, sol_A=1.0, sol_c=1.0, sol_p=0.0, sol_w=[1.0, 1.0, 0.0], seed=5)
    say(f"resume {prec} {kernel} {w.name}")
    b = Q.Basis(w.d, w.set_kind, w.level, law=w.law, basis=w.basis)
    p = Q.problem_from(w)
    ctx.set_prec_kernel(kernel)
    try:
        full = torch.zeros((w.N, b.n_funcs), dtype=torch.float64, device="cuda")
        if prec == "f64":
            ctx.solve(p, b, w.M, w.seed, full)
        else:
            ctx.solve_prec(p, b, w.M, w.seed, prec, full)
        for k in (w.N - 1, 3, 0):
            part = full.clone()
            part[: k + 1] = float("nan")  # the rows a crash would have lost
            ctx.solve_from(p, b, k, w.M, w.seed, part, precision=prec)
            torch.cuda.synchronize()
            assert torch.equal(part, full), f"resume at {k}"
    finally:
        ctx.set_prec_kernel("auto")


def test_workspace_cap_returns_enomem(env):
    Q, _, torch = env
    w = W.D2_TENSOR4
    b = Q.Basis(w.d, w.set_kind, w.level)
    p = Q.problem_from(w)
    ref = torch.zeros((w.N, b.n_funcs), dtype=torch.float64, device="cuda")
    c0 = Q.Context(0)
    try:
        c0.solve(p, b, w.M, w.seed, ref)
        torch.cuda.synchronize()
        need = c0.mem_held()
        assert need > 0
    finally:
        c0.close()
    c = Q.Context(0)
    try:
        c.set_mem_limit(need // 4)
        a = torch.full_like(ref, 7.0)
        with pytest.raises(Q.QrError) as e:
            c.solve(p, b, w.M, w.seed, a)
        assert e.value.status == -2 and "limit" in str(e.value)
        torch.cuda.synchronize()
        assert c.mem_held() <= need // 4
        assert bool((a == 7.0).all())  # nothing was launched on the table
        c.set_mem_limit(need)
        c.solve(p, b, w.M, w.seed, a)
        torch.cuda.synchronize()
        assert torch.equal(a, ref) and c.mem_held() <= need
        with pytest.raises(Q.QrError):
            c.set_mem_limit(-1)
    finally:
        c.close()
