"""GPU parity with a damping exponent q > 0 (eq (yqi), Algorithm 1): the
coefficients describe y_i / (1+|x|^2)^{q/2}; along the paths the expansion is
multiplied back before T_L and the driver (gradient by the product rule), and
each response is divided by (1+|X_i|^2)^{q/2}.  The HIP path against the CPU
oracle with the tolerances of the undamped parity tests (relative 1e-10).
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_common import env, dev, host, say, assert_alpha, TOL  # noqa: F401 (env is a fixture)

pytestmark = pytest.mark.gpu



def _zrat(d, q, law="logistic"):
    return W.Workload(name=f"zrat-d{d}-q{q}", d=d, N=4, T=1.0,
                      sigma=[[0.5 if a == c else 0.0 for c in range(d)] for a in range(d)],
                      b0=[0.0] * d, b1=[0.0] * d, set_kind="hc_1p", level=12, M=3000, driver="zrat",
                      f_a=-0.05, sol_A=1.0, sol_c=1.0, sol_p=0.0,
                      sol_w=[1.0 if l < 2 else 0.0 for l in range(d)], seed=3, law=law, damping_q=q)


@pytest.mark.parametrize("q", [0.5, 2.5])
@pytest.mark.parametrize("wname,i,M", [("d2", 8, 777), ("d2", 0, 300), ("zrat3", 1, 500)])
def test_path_responses_damped(env, q, wname, i, M):
    Q, ctx, torch = env
    w = W.D2_TENSOR4.with_(damping_q=q) if wname == "d2" else _zrat(3, q)
    say(f"path_responses damped q={q} {w.name} i={i} M={M}")
    b = Q.Basis(w.d, w.set_kind, w.level)
    reps = O.reps_for(w)
    alpha = W.synthetic_alpha(b.n_funcs, w.N, seed=7, scale=0.2)
    s = torch.empty(M, dtype=torch.float64, device="cuda")
    ctx.path_responses(Q.problem_from(w), b, i, M, 5, dev(torch, alpha), s)
    torch.cuda.synchronize()
    sg = host(s)
    for m in sorted(set([0, M - 1] + list(np.random.default_rng(1).integers(0, M, 6)))):
        ref = O.path_response(w, reps, i, 5, int(m), alpha)
        assert abs(sg[m] - ref) <= TOL * max(1.0, abs(ref)), (m, sg[m], ref)


@pytest.mark.parametrize("q,law", [(2.5, "logistic"), (2.0, "cauchy"), (1.0, "student2")])
@pytest.mark.parametrize("i", [9, 3])
def test_backward_step_damped(env, q, law, i):
    Q, ctx, torch = env
    w = W.D2_TENSOR4.with_(damping_q=q, law=law)
    say(f"backward_step damped q={q} {law} i={i}")
    b = Q.Basis(w.d, w.set_kind, w.level, law=law)
    reps = O.reps_for(w)
    alpha = W.synthetic_alpha(b.n_funcs, w.N, seed=11, scale=0.2)
    a = dev(torch, alpha)
    ctx.backward_step(Q.problem_from(w), b, i, w.M, w.seed, a)
    torch.cuda.synchronize()
    ref, absum, _, _ = O.backward_step(w, reps, i, w.M, w.seed, alpha.copy())
    assert_alpha(host(a)[i], ref, absum, what=f"damped q={q} {law} row {i}")


@pytest.mark.parametrize("d,i", [(3, 0), (8, 1)])
def test_backward_step_damped_gradient_driver(env, d, i):
    """z-dependent driver: z uses the gradient of ybar (1+|x|^2)^{q/2}."""
    Q, ctx, torch = env
    w = _zrat(d, 1.5)
    say(f"backward_step damped zrat d={d} i={i}")
    b = Q.Basis(w.d, w.set_kind, w.level)
    reps = O.reps_for(w)
    alpha = W.synthetic_alpha(b.n_funcs, w.N, seed=d, scale=0.2, decay=0.7)
    a = dev(torch, alpha)
    ctx.backward_step(Q.problem_from(w), b, i, w.M, w.seed, a)
    torch.cuda.synchronize()
    ref, absum, _, _ = O.backward_step(w, reps, i, w.M, w.seed, alpha.copy())
    assert_alpha(host(a)[i], ref, absum, what=f"damped zrat d={d} row {i}")


def test_solve_damped_matches_oracle(env):
    """Full damped solve (q = 1): rows against the oracle, and the error of
    the prediction ybar (1+|x|^2)^{q/2} at t_0 equal to the oracle's."""
    Q, ctx, torch = env
    q = 1.0
    w = W.D2_TENSOR4.with_(damping_q=q)
    say("solve d2 tensor damped q=1")
    b = Q.Basis(w.d, w.set_kind, w.level)
    reps = O.reps_for(w)
    a = torch.zeros((w.N, b.n_funcs), dtype=torch.float64, device="cuda")
    ctx.solve(Q.problem_from(w), b, w.M, w.seed, a)
    torch.cuda.synchronize()
    got = host(a)
    ref = O.solve(w, reps)
    for i in (w.N - 1, w.N // 2, 0):
        _, absum, _, _ = O.backward_step(w, reps, i, w.M, w.seed, ref.copy())
        assert_alpha(got[i], ref[i], absum, what=f"damped solve row {i}")
    n = 1 << 14
    x = torch.empty((w.d, n), dtype=torch.float64, device="cuda")
    ctx.sample_points(w.d, w.seed, 1, 0, n, x)
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    ctx.eval(b, a[0].contiguous(), x, y)
    torch.cuda.synchronize()
    xh = host(x).T
    pred = host(y) * (1.0 + (xh ** 2).sum(axis=1)) ** (q / 2)
    u = np.exp(-1.0) * np.cos(xh[:, 0] + xh[:, 1])
    rel = np.linalg.norm(pred - u) / np.linalg.norm(u)
    _, _, rel_oracle = O.errors(w, reps, ref, seed=w.seed, n=n)
    assert abs(rel - rel_oracle) < 1e-8


def test_damping_argument_checks(env):
    Q, ctx, torch = env
    w = W.D2_TENSOR4
    b = Q.Basis(w.d, w.set_kind, w.level)
    a = torch.zeros((w.N, b.n_funcs), dtype=torch.float64, device="cuda")
    for bad in (-0.5, math.nan, 65.0):
        with pytest.raises(Q.QrError) as e:
            ctx.backward_step(Q.problem_from(w.with_(damping_q=bad)), b, w.N - 1, 100, 0, a)
        assert e.value.status == -1
    damped = Q.problem_from(w.with_(damping_q=1.0))
    with pytest.raises(Q.QrError) as e:
        ctx.solve_prec(damped, b, 100, 0, "bf16", a)
    assert e.value.status == -6
    with pytest.raises(Q.QrError) as e:
        ctx.solve_batched(damped, b, [(0.5, w.d, w.level, 100)], 0, a[None])
    assert e.value.status == -6
    with pytest.raises(Q.QrError) as e:
        ctx.solve_learned(damped, b, 100, 0, a, train_points=1 << 12, heldout_points=1 << 10,
                          epochs=1, batch=1024, gate=0.0)
    assert e.value.status == -6


@pytest.mark.parametrize("q", [0.0, 2.1, 5.1])
@pytest.mark.parametrize("basis", ["fourier", "cosine"])
def test_eval_y_damped_prediction(env, q, basis):
    """qr_eval_y: the prediction y = ybar (1+|x|^2)^{q/2} of a damped problem
    and its gradient by the product rule, against the oracle's eval_y point
    by point; with q = 0 it is qr_eval."""
    Q, ctx, torch = env
    w = (W.paper_benchmark(2, 4, "hc_max", 9, 100) if basis == "cosine" else _zrat(3, q)).with_(damping_q=q)
    say(f"eval_y q={q} {basis} {w.name}")
    b = Q.Basis(w.d, w.set_kind, w.level, law=w.law, basis=w.basis)
    reps = O.reps_for(w)
    alpha = W.synthetic_alpha(b.n_funcs, 1, seed=13, scale=0.3)[0]
    n = 300
    x = W.law_points(n, w.d, w.law, seed=8)
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    g = torch.empty((w.d, n), dtype=torch.float64, device="cuda")
    ctx.eval_y(Q.problem_from(w), b, dev(torch, alpha), dev(torch, x.T), y, g)
    torch.cuda.synchronize()
    yg, gg = host(y), host(g).T
    for p in range(n):
        ry, rg = O.eval_y(w, reps, alpha, x[p], grad=True)
        D = (1.0 + float(x[p] @ x[p])) ** (0.5 * q)
        scale = np.abs(alpha).sum() * 2 ** (w.d / 2) * D
        assert abs(yg[p] - ry) <= TOL * scale, (p, yg[p], ry)
        assert np.abs(gg[p] - rg).max() <= TOL * scale * 2 * math.pi * w.level * (1.0 + q), (p, gg[p], rg)
    if q == 0.0:
        # the same walk as qr_eval with the gradient (value-only walks sum in another order)
        y0, g0 = torch.empty_like(y), torch.empty_like(g)
        ctx.eval(b, dev(torch, alpha), dev(torch, x.T), y0, g0)
        torch.cuda.synchronize()
        assert torch.equal(y, y0) and torch.equal(g, g0)
