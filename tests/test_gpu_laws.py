"""GPU parity under the paper's own sampling laws (Sec. 5): Student's t with
mu = 2 and the Cauchy law.  The HIP path (through the C ABI, bases built with
qr_build_basis_law) against the CPU oracle on the same Philox streams, with
the tolerances of the logistic-law parity tests: relative 1e-10 per
coefficient against max(|alpha_k|, A_k) and for the row in the 2-norm.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_common import env, dev, host, say, assert_alpha, TOL  # noqa: F401 (env is a fixture)

pytestmark = pytest.mark.gpu

LAWS = ["student2", "cauchy"]


@pytest.mark.parametrize("law", LAWS)
@pytest.mark.parametrize("n", [1, 5000])
def test_sample_points_law(env, law, n):
    Q, ctx, torch = env
    say(f"sample_points {law} n={n}")
    d = 5
    x = torch.empty((d, n), dtype=torch.float64, device="cuda")
    ctx.sample_points(d, 11, 1, 3, n, x, m0=17, law=law)
    torch.cuda.synchronize()
    ref = O.sample_points(d, 11, 1, 3, n, m0=17, law=law)
    assert np.allclose(host(x).T, ref, rtol=1e-13, atol=1e-15)


def test_basis_reports_its_law(env):
    Q, ctx, torch = env
    for name, code in Q.LAWS.items():
        assert Q.Basis(2, "tensor", 2, law=name).law == code


@pytest.mark.parametrize("law", LAWS)
@pytest.mark.parametrize("d,kind,level,n", [(2, "tensor", 4, 4099), (6, "hc_max", 16, 700),
                                            (10, "hc_1p", 32, 300)])
def test_project_law(env, law, d, kind, level, n):
    Q, ctx, torch = env
    say(f"project {law} d={d} {kind} {level} n={n}")
    b = Q.Basis(d, kind, level, law=law)
    reps = O.enumerate_set(d, kind, level)
    x = W.law_points(n, d, law, seed=d + n)
    s = W.responses(n, seed=n)
    a = torch.empty(b.n_funcs, dtype=torch.float64, device="cuda")
    ctx.project(b, dev(torch, x.T), dev(torch, s), a)
    torch.cuda.synchronize()
    ref, absum = O.project(reps, x, s, with_abs=True, law=law)
    assert_alpha(host(a), ref, absum, what=f"project {law}")


@pytest.mark.parametrize("law", LAWS)
@pytest.mark.parametrize("d,kind,level,n,grad", [(2, "tensor", 4, 129, True), (6, "hc_max", 16, 300, False),
                                                 (3, "hc_1p", 12, 500, True)])
def test_eval_law(env, law, d, kind, level, n, grad):
    Q, ctx, torch = env
    say(f"eval {law} d={d} {kind} {level} n={n} grad={grad}")
    b = Q.Basis(d, kind, level, law=law)
    reps = O.enumerate_set(d, kind, level)
    alpha = W.synthetic_alpha(b.n_funcs, 1, seed=3)[0]
    x = W.law_points(n, d, law, seed=1)
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    g = torch.empty((d, n), dtype=torch.float64, device="cuda") if grad else None
    ctx.eval(b, dev(torch, alpha), dev(torch, x.T), y, g)
    torch.cuda.synchronize()
    if grad:
        ry, rg = O.evaluate(reps, alpha, x, grad=True, law=law)
        scale = np.abs(alpha).sum() * 2 * math.pi * level
        assert np.abs(host(g).T - rg).max() <= TOL * scale
    else:
        ry = O.evaluate(reps, alpha, x, law=law)
    assert np.abs(host(y) - ry).max() <= TOL * np.abs(alpha).sum()


@pytest.mark.parametrize("law", LAWS)
@pytest.mark.parametrize("i,M", [(9, 1), (8, 777), (0, 2000)])
def test_path_responses_law(env, law, i, M):
    Q, ctx, torch = env
    w = W.D2_TENSOR4.with_(law=law)
    say(f"path_responses {law} {w.name} i={i} M={M}")
    b = Q.Basis(w.d, w.set_kind, w.level, law=law)
    reps = O.reps_for(w)
    alpha = W.synthetic_alpha(b.n_funcs, w.N, seed=7, scale=0.2)
    s = torch.empty(M, dtype=torch.float64, device="cuda")
    x0 = torch.empty((w.d, M), dtype=torch.float64, device="cuda")
    ctx.path_responses(Q.problem_from(w), b, i, M, 5, dev(torch, alpha), s, x0)
    torch.cuda.synchronize()
    sg, xg = host(s), host(x0).T
    ms = sorted(set([0, M - 1] + list(np.random.default_rng(0).integers(0, M, 6))))
    for m in ms:
        ref = O.path_response(w, reps, i, 5, int(m), alpha)
        assert abs(sg[m] - ref) <= TOL * max(1.0, abs(ref)), (m, sg[m], ref)
        assert np.allclose(xg[m], [O.law_icdf(law, O.uniform(5, 0, int(m), i, l)) for l in range(w.d)],
                           rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("law", LAWS)
@pytest.mark.parametrize("i", [9, 4])
def test_backward_step_d2_tensor_law(env, law, i):
    Q, ctx, torch = env
    w = W.D2_TENSOR4.with_(law=law)
    say(f"backward_step {law} d2 tensor i={i}")
    b = Q.Basis(w.d, w.set_kind, w.level, law=law)
    reps = O.reps_for(w)
    alpha = W.synthetic_alpha(b.n_funcs, w.N, seed=11, scale=0.2)
    a = dev(torch, alpha)
    ctx.backward_step(Q.problem_from(w), b, i, w.M, w.seed, a)
    torch.cuda.synchronize()
    ref, absum, _, _ = O.backward_step(w, reps, i, w.M, w.seed, alpha.copy())
    assert_alpha(host(a)[i], ref, absum, what=f"{law} row {i}")


@pytest.mark.parametrize("law", LAWS)
@pytest.mark.parametrize("d,i", [(3, 0), (8, 1)])
def test_backward_step_gradient_driver_law(env, law, d, i):
    """z-dependent driver: the gradient goes through the law's density."""
    Q, ctx, torch = env
    w = W.Workload(name=f"zrat-d{d}-{law}", d=d, N=4, T=1.0,
                   sigma=[[0.5 if a == c else 0.0 for c in range(d)] for a in range(d)],
                   b0=[0.0] * d, b1=[0.0] * d, set_kind="hc_1p", level=12, M=3000, driver="zrat",
                   f_a=-0.05, sol_A=1.0, sol_c=1.0, sol_p=0.0,
                   sol_w=[1.0 if l < 2 else 0.0 for l in range(d)], seed=3, law=law)
    say(f"backward_step zrat {law} d={d} i={i}")
    b = Q.Basis(w.d, w.set_kind, w.level, law=law)
    reps = O.reps_for(w)
    alpha = W.synthetic_alpha(b.n_funcs, w.N, seed=d, scale=0.2, decay=0.7)
    a = dev(torch, alpha)
    ctx.backward_step(Q.problem_from(w), b, i, w.M, w.seed, a)
    torch.cuda.synchronize()
    ref, absum, _, _ = O.backward_step(w, reps, i, w.M, w.seed, alpha.copy())
    assert_alpha(host(a)[i], ref, absum, what=f"zrat {law} d={d} row {i}")


@pytest.mark.parametrize("law", LAWS)
def test_solve_d2_law_matches_oracle(env, law):
    """Full solve under the law, rows against the oracle, and the relative L2
    error at t_0 on stream-1 points of the law equal to the oracle's."""
    Q, ctx, torch = env
    w = W.D2_TENSOR4.with_(law=law)
    say(f"solve d2 tensor {law}")
    b = Q.Basis(w.d, w.set_kind, w.level, law=law)
    reps = O.reps_for(w)
    a = torch.zeros((w.N, b.n_funcs), dtype=torch.float64, device="cuda")
    ctx.solve(Q.problem_from(w), b, w.M, w.seed, a)
    torch.cuda.synchronize()
    got = host(a)
    ref = O.solve(w, reps)
    for i in (w.N - 1, w.N // 2, 0):
        _, absum, _, _ = O.backward_step(w, reps, i, w.M, w.seed, ref.copy())
        assert_alpha(got[i], ref[i], absum, what=f"solve {law} row {i}")
    n = 1 << 14
    x = torch.empty((w.d, n), dtype=torch.float64, device="cuda")
    ctx.sample_points(w.d, w.seed, 1, 0, n, x, law=law)
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    ctx.eval(b, a[0].contiguous(), x, y)
    torch.cuda.synchronize()
    xh = host(x).T
    u = np.exp(-1.0) * np.cos(xh[:, 0] + xh[:, 1])
    rel = np.linalg.norm(host(y) - u) / np.linalg.norm(u)
    _, _, rel_oracle = O.errors(w, reps, ref, seed=w.seed, n=n)
    assert abs(rel - rel_oracle) < 1e-8


# ---------------------------------------------------------------------------
# the other forms read the law from the basis too
# ---------------------------------------------------------------------------

UNIT = {"bf16": 2.0 ** -8, "f16": 2.0 ** -11}


@pytest.mark.parametrize("law", LAWS)
@pytest.mark.parametrize("prec", ["bf16", "f16"])
def test_prec_backward_step_law(env, law, prec):
    """Reduced-precision form under the law, z-dependent driver (value and
    gradient right-hand sides): rows within u (relative 2-norm) of the FP64
    oracle, the bound of the logistic-law precision tests."""
    Q, ctx, torch = env
    d = 3
    w = W.Workload(name=f"zrat-d{d}-{law}", d=d, N=4, T=1.0,
                   sigma=[[0.5 if a == c else 0.0 for c in range(d)] for a in range(d)],
                   b0=[0.0] * d, b1=[0.0] * d, set_kind="hc_1p", level=12, M=4000, driver="zrat",
                   f_a=-0.05, sol_A=1.0, sol_c=1.0, sol_p=0.0,
                   sol_w=[1.0 if l < 2 else 0.0 for l in range(d)], seed=5, law=law)
    say(f"prec backward step {law} {prec}")
    b = Q.Basis(w.d, w.set_kind, w.level, law=law)
    reps = O.reps_for(w)
    alpha = W.synthetic_alpha(b.n_funcs, w.N, seed=d, scale=0.2, decay=0.7)
    for i in (w.N - 2, 0):
        a = dev(torch, alpha)
        ctx.backward_step_prec(Q.problem_from(w), b, i, w.M, w.seed, prec, a)
        torch.cuda.synchronize()
        ref, _, _, _ = O.backward_step(w, reps, i, w.M, w.seed, alpha.copy())
        err = float(np.linalg.norm(host(a)[i] - ref) / np.linalg.norm(ref))
        say(f"  row {i}: rel err {err:.3e}")
        assert err <= UNIT[prec], (i, err)


@pytest.mark.parametrize("law", LAWS)
def test_batched_law_equals_unbatched(env, law):
    """Batched instances on the whole basis under the law give qr_solve's
    coefficients for their driver parameter, and the first matches the oracle."""
    Q, ctx, torch = env
    w = W.D2_TENSOR4.with_(law=law)
    b = Q.Basis(w.d, w.set_kind, w.level, law=law)
    fas = [0.2, 0.9]
    say(f"batched vs qr_solve, d2 tensor, {law}")
    a = torch.zeros((len(fas), w.N, b.n_funcs), dtype=torch.float64, device="cuda")
    ctx.solve_batched(Q.problem_from(w), b, [(f, w.d, w.level, w.M) for f in fas], w.seed, a)
    for r, f in enumerate(fas):
        ref = torch.zeros((w.N, b.n_funcs), dtype=torch.float64, device="cuda")
        ctx.solve(Q.problem_from(w.with_(f_a=f)), b, w.M, w.seed, ref)
        torch.cuda.synchronize()
        err = (a[r] - ref).abs().max().item()
        assert err <= TOL * ref.abs().max().item(), (f, err)
    w0 = w.with_(f_a=fas[0])
    reps = O.reps_for(w)
    oref = O.solve(w0, reps)
    got = host(a)[0]
    for i in (w.N - 1, 0):
        _, absum, _, _ = O.backward_step(w0, reps, i, w.M, w.seed, oref.copy())
        assert_alpha(got[i], oref[i], absum, what=f"batched {law} row {i}")


@pytest.mark.parametrize("law", LAWS)
def test_learned_law_closed_gate_is_the_plain_solve(env, law):
    """Learned form under the law with gate 0: the surrogates (trained on the
    law's points and features) are all rejected and the step-major pipeline
    reproduces qr_solve."""
    Q, ctx, torch = env
    w = W.D2_TENSOR4.with_(law=law)
    b = Q.Basis(w.d, w.set_kind, w.level, law=law)
    a = torch.zeros((w.N, b.n_funcs), dtype=torch.float64, device="cuda")
    rep = ctx.solve_learned(Q.problem_from(w), b, w.M, w.seed, a, train_points=1 << 12,
                            heldout_points=1 << 10, epochs=1, batch=1024, gate=0.0)
    ref = torch.zeros_like(a)
    ctx.solve(Q.problem_from(w), b, w.M, w.seed, ref)
    torch.cuda.synchronize()
    assert all(not r["used"] for r in rep)
    err = (a - ref).abs().max().item()
    assert err <= 1e-12 * ref.abs().max().item(), err
