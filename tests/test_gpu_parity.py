"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Both sides consume the same Philox streams; the tolerance for FP64 results is
relative 1e-10, applied per coefficient against max(|alpha_k|, A_k) where
A_k = (1/M) sum |S phi_k| bounds the cancellation in the Monte-Carlo sum,
and to the whole row in the 2-norm.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_common import env, dev, host, say, assert_alpha, TOL  # noqa: F401 (env is a fixture)

pytestmark = pytest.mark.gpu



# ---------------------------------------------------------------------------
# pieces
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 257, 5000])
def test_sample_points(env, n):
    Q, ctx, torch = env
    say(f"sample_points n={n}")
    d = 5
    x = torch.empty((d, n), dtype=torch.float64, device="cuda")
    ctx.sample_points(d, 11, 1, 3, n, x, m0=17)
    torch.cuda.synchronize()
    ref = O.sample_points(d, 11, 1, 3, n, m0=17)
    assert np.allclose(host(x).T, ref, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("d,kind,level,n", [(2, "tensor", 4, 1), (2, "tensor", 4, 4099),
                                            (3, "hc_1p", 12, 1000), (6, "hc_max", 16, 700),
                                            (1, "tensor", 0, 33), (10, "hc_1p", 32, 300)])
def test_project(env, d, kind, level, n):
    Q, ctx, torch = env
    say(f"project d={d} {kind} {level} n={n}")
    b = Q.Basis(d, kind, level)
    reps = O.enumerate_set(d, kind, level)
    x = W.logistic_points(n, d, seed=d + n)
    s = W.responses(n, seed=n)
    a = torch.empty(b.n_funcs, dtype=torch.float64, device="cuda")
    ctx.project(b, dev(torch, x.T), dev(torch, s), a)
    torch.cuda.synchronize()
    ref, absum = O.project(reps, x, s, with_abs=True)
    assert_alpha(host(a), ref, absum, what="project")


@pytest.mark.parametrize("d,kind,level,n,grad", [(2, "tensor", 4, 1000, False), (2, "tensor", 4, 129, True),
                                                 (6, "hc_max", 16, 300, False), (3, "hc_1p", 12, 500, True),
                                                 (10, "hc_1p", 32, 200, True)])
def test_eval(env, d, kind, level, n, grad):
    Q, ctx, torch = env
    say(f"eval d={d} {kind} {level} n={n} grad={grad}")
    b = Q.Basis(d, kind, level)
    reps = O.enumerate_set(d, kind, level)
    alpha = W.synthetic_alpha(b.n_funcs, 1, seed=3)[0]
    x = W.logistic_points(n, d, seed=1)
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    g = torch.empty((d, n), dtype=torch.float64, device="cuda") if grad else None
    ctx.eval(b, dev(torch, alpha), dev(torch, x.T), y, g)
    torch.cuda.synchronize()
    if grad:
        ry, rg = O.evaluate(reps, alpha, x, grad=True)
        scale = np.abs(alpha).sum() * 2 * math.pi * level
        assert np.abs(host(g).T - rg).max() <= TOL * scale
    else:
        ry = O.evaluate(reps, alpha, x)
    assert np.abs(host(y) - ry).max() <= TOL * np.abs(alpha).sum()


@pytest.mark.parametrize("d,kind,level,n", [(2, "tensor", 4, 1), (2, "tensor", 4, 300), (6, "hc_max", 16, 5000),
                                            (3, "hc_1p", 12, 257), (10, "hc_1p", 32, 700), (16, "hc_1p", 32, 600),
                                            (1, "tensor", 0, 33)])
def test_eval_split(env, d, kind, level, n):
    """The evaluation with the basis split across blocks (small point sets):
    the oracle's values, and qr_eval's up to rounding order, on sets of one
    and of many tasks, ragged batches and a single point."""
    Q, ctx, torch = env
    say(f"eval_split d={d} {kind} {level} n={n}")
    b = Q.Basis(d, kind, level)
    alpha = W.synthetic_alpha(b.n_funcs, 1, seed=5)[0]
    x = W.logistic_points(n, d, seed=2)
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    ctx.eval_split(b, dev(torch, alpha), dev(torch, x.T), y)
    y0 = torch.empty_like(y)
    ctx.eval(b, dev(torch, alpha), dev(torch, x.T), y0)
    torch.cuda.synchronize()
    bound = TOL * np.abs(alpha).sum()
    assert np.abs(host(y) - host(y0)).max() <= bound
    if b.n_funcs <= 200_000 and n <= 700:
        reps = O.enumerate_set(d, kind, level)
        ry = O.evaluate(reps, alpha, x)
        assert np.abs(host(y) - ry).max() <= bound


def test_eval_split_arguments(env):
    Q, ctx, torch = env
    b = Q.Basis(2, "tensor", 4)
    a = torch.zeros(b.n_funcs, dtype=torch.float64, device="cuda")
    n = (1 << 17) + 1
    x = torch.zeros((2, n), dtype=torch.float64, device="cuda")
    y = torch.zeros(n, dtype=torch.float64, device="cuda")
    with pytest.raises(Q.QrError) as e:
        ctx.eval_split(b, a, x, y)
    assert e.value.status == -1


# ---------------------------------------------------------------------------
# path responses and backward steps
# ---------------------------------------------------------------------------

def _small(w, **kw):
    return w.with_(**kw)


@pytest.mark.parametrize("wname,i,M", [("d2", 9, 1), ("d2", 8, 777), ("d2", 0, 2000),
                                       ("d6", 19, 300), ("d6", 17, 128)])
def test_path_responses(env, wname, i, M):
    Q, ctx, torch = env
    w = {"d2": W.D2_TENSOR4, "d6": W.D6_HCMAX16}[wname]
    say(f"path_responses {w.name} i={i} M={M}")
    b = Q.Basis(w.d, w.set_kind, w.level)
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
        assert np.allclose(xg[m], [O.logistic_icdf(O.uniform(5, 0, int(m), i, l)) for l in range(w.d)],
                           rtol=1e-14, atol=1e-14)


def _zrat(d, level=12, N=4, M=3000):
    return W.Workload(name=f"zrat-d{d}", d=d, N=N, T=1.0,
                      sigma=[[0.5 if a == b else 0.0 for b in range(d)] for a in range(d)],
                      b0=[0.0] * d, b1=[0.0] * d, set_kind="hc_1p", level=level, M=M, driver="zrat",
                      f_a=-0.05, sol_A=1.0, sol_c=1.0, sol_p=0.0,
                      sol_w=[1.0 if l < 2 else 0.0 for l in range(d)], seed=3)


@pytest.mark.parametrize("d,i", [(3, 0), (8, 1), (13, 2)])
def test_backward_step_gradient_driver(env, d, i):
    """z-dependent driver: the walk carries the x-gradient of ybar (FP64)."""
    Q, ctx, torch = env
    w = _zrat(d)
    say(f"backward_step zrat d={d} i={i}")
    b = Q.Basis(w.d, w.set_kind, w.level)
    reps = O.reps_for(w)
    alpha = W.synthetic_alpha(b.n_funcs, w.N, seed=d, scale=0.2, decay=0.7)
    a = dev(torch, alpha)
    ctx.backward_step(Q.problem_from(w), b, i, w.M, w.seed, a)
    torch.cuda.synchronize()
    ref, absum, _, _ = O.backward_step(w, reps, i, w.M, w.seed, alpha.copy())
    assert_alpha(host(a)[i], ref, absum, what=f"zrat d={d} row {i}")


@pytest.mark.parametrize("w,i", [(W.D10_HC1P32_ZRAT, 27), (W.D16_HC1P32, 38)], ids=["d10-zrat", "d16"])
def test_path_responses_full_basis_sampled(env, w, i):
    """The d=10 (gradient driver) and d=16 sets at their full size: responses
    of sampled paths of a step with two expansion levels ahead."""
    Q, ctx, torch = env
    M = 4096
    say(f"path_responses {w.name} i={i} M={M}")
    b = Q.Basis(w.d, w.set_kind, w.level)
    reps = O.reps_for(w)
    alpha = W.synthetic_alpha(b.n_funcs, w.N, seed=21, scale=0.05, decay=0.8)
    s = torch.empty(M, dtype=torch.float64, device="cuda")
    ctx.path_responses(Q.problem_from(w), b, i, M, 9, dev(torch, alpha), s)
    torch.cuda.synchronize()
    sg = host(s)
    for m in [0, 77, 2048, M - 1]:
        ref = O.path_response(w, reps, i, 9, m, alpha)
        assert abs(sg[m] - ref) <= TOL * max(1.0, abs(ref)), (m, sg[m], ref)


@pytest.mark.parametrize("i", [9, 8, 4])
def test_backward_step_d2_tensor(env, i):
    Q, ctx, torch = env
    w = W.D2_TENSOR4
    say(f"backward_step d2 tensor i={i}")
    b = Q.Basis(w.d, w.set_kind, w.level)
    reps = O.reps_for(w)
    alpha = W.synthetic_alpha(b.n_funcs, w.N, seed=11, scale=0.2)
    a = dev(torch, alpha)
    ctx.backward_step(Q.problem_from(w), b, i, w.M, w.seed, a)
    torch.cuda.synchronize()
    ref_tab = alpha.copy()
    ref, absum, _, _ = O.backward_step(w, reps, i, w.M, w.seed, ref_tab)
    got = host(a)
    assert_alpha(got[i], ref, absum, what=f"row {i}")
    # other rows untouched
    rows = [r for r in range(w.N) if r != i]
    assert np.array_equal(got[rows], alpha[rows])


def test_backward_step_d6_hcmax_reduced_M(env):
    """Full |Gamma| = 169,209 of the d=6 hyperbolic cross, M reduced so the
    oracle finishes: steps N-1 and N-2."""
    Q, ctx, torch = env
    w = W.D6_HCMAX16
    b = Q.Basis(w.d, w.set_kind, w.level)
    reps = O.reps_for(w)
    M = 600
    alpha = W.synthetic_alpha(b.n_funcs, w.N, seed=13, scale=0.1, decay=0.8)
    for i in (19, 18):
        say(f"backward_step d6 hc_max i={i} M={M}")
        a = dev(torch, alpha)
        ctx.backward_step(Q.problem_from(w), b, i, M, w.seed, a)
        torch.cuda.synchronize()
        ref, absum, _, _ = O.backward_step(w, reps, i, M, w.seed, alpha.copy())
        assert_alpha(host(a)[i], ref, absum, what=f"d6 hc_max row {i}")


def test_solve_d2_tensor_full(env):
    Q, ctx, torch = env
    w = W.D2_TENSOR4
    say("solve d2 tensor")
    b = Q.Basis(w.d, w.set_kind, w.level)
    reps = O.reps_for(w)
    a = torch.zeros((w.N, b.n_funcs), dtype=torch.float64, device="cuda")
    ctx.solve(Q.problem_from(w), b, w.M, w.seed, a)
    torch.cuda.synchronize()
    got = host(a)
    ref = O.solve(w, reps)
    for i in range(w.N - 1, -1, -1):
        _, absum, _, _ = O.backward_step(w, reps, i, w.M, w.seed, ref.copy())
        assert_alpha(got[i], ref[i], absum, what=f"solve row {i}")
    # deterministic: a second solve is bit-identical
    a2 = torch.zeros_like(a)
    ctx.solve(Q.problem_from(w), b, w.M, w.seed, a2)
    torch.cuda.synchronize()
    assert torch.equal(a, a2)


def test_solve_d2_tensor_error_against_closed_form(env):
    """Relative L2 error at t_0 against u(0,.) on stream-1 test points,
    evaluated with qr_eval, equals the oracle's figure."""
    Q, ctx, torch = env
    w = W.D2_TENSOR4
    b = Q.Basis(w.d, w.set_kind, w.level)
    reps = O.reps_for(w)
    a = torch.zeros((w.N, b.n_funcs), dtype=torch.float64, device="cuda")
    ctx.solve(Q.problem_from(w), b, w.M, w.seed, a)
    n = 1 << 14
    x = torch.empty((w.d, n), dtype=torch.float64, device="cuda")
    ctx.sample_points(w.d, w.seed, 1, 0, n, x)
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    ctx.eval(b, a[0].contiguous(), x, y)
    torch.cuda.synchronize()
    xh = host(x).T
    u = np.exp(-1.0) * np.cos(xh[:, 0] + xh[:, 1])
    rel = np.linalg.norm(host(y) - u) / np.linalg.norm(u)
    _, _, rel_oracle = O.errors(w, reps, O.solve(w, reps), seed=w.seed, n=n)
    assert abs(rel - rel_oracle) < 1e-9
    assert 0.3 < rel < 0.6


def test_ragged_and_degenerate_sizes(env):
    Q, ctx, torch = env
    say("degenerate sizes")
    # N = 1, d = 1, basis with only the constant (level 0)
    w = W.Workload(name="tiny", d=1, N=1, T=0.5, sigma=[[0.3]], b0=[0.1], b1=[0.2],
                   set_kind="tensor", level=0, M=5, driver="allen_cahn", f_a=0.0,
                   sol_A=0.5, sol_c=0.7, sol_p=0.1, sol_w=[1.3], clamp=0.8)
    b = Q.Basis(1, "tensor", 0)
    assert b.n_funcs == 1
    a = torch.zeros((1, 1), dtype=torch.float64, device="cuda")
    ctx.solve(Q.problem_from(w), b, w.M, 3, a)
    torch.cuda.synchronize()
    ref = O.solve(w, O.reps_for(w), M=5, seed=3)
    assert abs(host(a)[0, 0] - ref[0, 0]) <= TOL * abs(ref[0, 0])
    # invalid: i out of range, M = 0
    with pytest.raises(Q.QrError):
        ctx.backward_step(Q.problem_from(w), b, 1, 5, 3, a)
    with pytest.raises(Q.QrError):
        ctx.solve(Q.problem_from(w), b, 0, 3, a)
    # dimension mismatch between basis and problem
    with pytest.raises(Q.QrError):
        ctx.solve(Q.problem_from(W.D2_TENSOR4), b, 5, 3, a)


def test_prefix_property(env):
    """Path m uses counters (m, i, r) only: the first M' responses of a cloud
    of M > M' paths are those of the cloud of M' paths."""
    Q, ctx, torch = env
    w = W.D2_TENSOR4
    b = Q.Basis(w.d, w.set_kind, w.level)
    alpha = dev(torch, W.synthetic_alpha(b.n_funcs, w.N, seed=2, scale=0.2))
    s1 = torch.empty(1000, dtype=torch.float64, device="cuda")
    s2 = torch.empty(3333, dtype=torch.float64, device="cuda")
    ctx.path_responses(Q.problem_from(w), b, 3, 1000, 0, alpha, s1)
    ctx.path_responses(Q.problem_from(w), b, 3, 3333, 0, alpha, s2)
    torch.cuda.synchronize()
    assert torch.equal(s1, s2[:1000])


# ---------------------------------------------------------------------------
# the benchmarked configuration at full size (M = 2^20, |Gamma| = 169,209)
# ---------------------------------------------------------------------------

def test_d6_hcmax_full_size_sampled(env):
    """At full M: step N-1 coefficients for sampled k (the oracle projects its
    own responses onto a subset of the basis), and step N-2 responses for
    sampled paths."""
    Q, ctx, torch = env
    w = W.D6_HCMAX16
    b = Q.Basis(w.d, w.set_kind, w.level)
    reps = O.reps_for(w)
    say("d6 hc_max full size: step N-1")
    a = torch.zeros((w.N, b.n_funcs), dtype=torch.float64, device="cuda")
    ctx.backward_step(Q.problem_from(w), b, w.N - 1, w.M, w.seed, a)
    torch.cuda.synchronize()
    got = host(a)[w.N - 1]
    rng = np.random.default_rng(1)
    sub = np.concatenate([[0], np.sort(rng.choice(np.arange(1, reps.shape[0]), 24, replace=False))])
    sub_reps = np.ascontiguousarray(reps[sub])
    ref, absum, _, _ = O.backward_step(w, sub_reps, w.N - 1, w.M, w.seed,
                                       np.zeros((w.N, 2 * len(sub) - 1)))
    idx = [0] + [f for r in sub[1:] for f in (2 * r - 1, 2 * r)]
    assert_alpha(got[idx], ref, absum, what="d6 hc_max full N-1 sampled")
    say("d6 hc_max full size: responses of step N-2")
    alpha = W.synthetic_alpha(b.n_funcs, w.N, seed=17, scale=0.1, decay=0.8)
    s = torch.empty(w.M, dtype=torch.float64, device="cuda")
    ctx.path_responses(Q.problem_from(w), b, w.N - 2, w.M, w.seed, dev(torch, alpha), s)
    torch.cuda.synchronize()
    sg = host(s)
    for m in [0, w.M - 1] + list(rng.integers(0, w.M, 14)):
        ref = O.path_response(w, reps, w.N - 2, w.seed, int(m), alpha)
        assert abs(sg[m] - ref) <= TOL * max(1.0, abs(ref)), m


def test_d16_hc1p_full_size_sampled(env):
    """The d = 16 workload at full size (599,969 functions, M = 2^22): step
    N-1 coefficients for sampled k (the oracle projects its own responses of
    all 2^22 paths on the sampled representatives), and step N-2 responses
    (one 599,969-term expansion level ahead) for sampled paths."""
    Q, ctx, torch = env
    w = W.D16_HC1P32
    b = Q.Basis(w.d, w.set_kind, w.level)
    reps = O.reps_for(w)
    assert b.n_funcs == 599969 and w.M == 1 << 22
    say("d16 hc_1p full size: step N-1")
    a = torch.zeros((w.N, b.n_funcs), dtype=torch.float64, device="cuda")
    ctx.backward_step(Q.problem_from(w), b, w.N - 1, w.M, w.seed, a)
    torch.cuda.synchronize()
    got = host(a[w.N - 1])
    del a
    rng = np.random.default_rng(5)
    sub = np.concatenate([[0], np.sort(rng.choice(np.arange(1, reps.shape[0]), 16, replace=False))])
    ref, absum, _, _ = O.backward_step(w, np.ascontiguousarray(reps[sub]), w.N - 1, w.M, w.seed,
                                       np.zeros((w.N, 2 * len(sub) - 1)))
    idx = [0] + [f for r in sub[1:] for f in (2 * r - 1, 2 * r)]
    assert_alpha(got[idx], ref, absum, what="d16 hc_1p full N-1 sampled")
    say("d16 hc_1p full size: responses of step N-2")
    alpha = W.synthetic_alpha(b.n_funcs, w.N, seed=19, scale=0.05, decay=0.8)
    s = torch.empty(w.M, dtype=torch.float64, device="cuda")
    ctx.path_responses(Q.problem_from(w), b, w.N - 2, w.M, w.seed, dev(torch, alpha), s)
    torch.cuda.synchronize()
    sg = host(s)
    assert np.isfinite(sg).all()
    for m in [0, w.M - 1] + list(rng.integers(0, w.M, 6)):
        ref = O.path_response(w, reps, w.N - 2, w.seed, int(m), alpha)
        assert abs(sg[m] - ref) <= TOL * max(1.0, abs(ref)), m


# ---------------------------------------------------------------------------
# batched form: instances on one shared cloud
# ---------------------------------------------------------------------------

def _embed(reps, d):
    out = np.zeros((reps.shape[0], d), dtype=np.int32)
    out[:, :reps.shape[1]] = reps
    return out


def _func_index(full_reps, sub_reps):
    """Canonical function indices (of the full set) of the functions of sub_reps."""
    pos = {tuple(r): c for c, r in enumerate(full_reps)}
    idx = [0]
    for r in sub_reps[1:]:
        c = pos[tuple(r)]
        idx += [2 * c - 1, 2 * c]
    return np.array(idx)


def _check_batched_instance(got, w, full_reps, inst, seed, rows, what):
    """got: [N][nf] of one instance.  The oracle solves the group problem
    with the instance's f_a on its own index set (embedded) and cloud size."""
    f_a, d_r, level_r, M_r = inst
    wr = w.with_(f_a=f_a)
    reps = _embed(O.enumerate_set(d_r, w.set_kind, level_r), w.d)
    idx = _func_index(full_reps, reps)
    ref = O.solve(wr, reps, M=M_r, seed=seed)
    mask = np.ones(got.shape[1], dtype=bool)
    mask[idx] = False
    assert not got[:, mask].any(), f"{what}: coefficients outside the instance's set are not 0"
    for i in rows:
        _, absum, _, _ = O.backward_step(wr, reps, i, M_r, seed, ref.copy())
        assert_alpha(got[i, idx], ref[i], absum, what=f"{what} row {i}")


def test_batched_against_oracle(env):
    """Ten instances of uneven d, level and M (two passes, the second ragged)."""
    Q, ctx, torch = env
    w = W.Workload(name="batch-small", d=5, N=4, T=1.0, sigma=[[0.5 if a == b else 0.0 for b in range(5)]
                                                              for a in range(5)],
                   b0=[0.0] * 5, b1=[0.0] * 5, set_kind="hc_1p", level=12, M=3000, driver="sin",
                   f_a=0.5, sol_A=1.0, sol_c=1.0, sol_p=0.0, sol_w=[1.0, 1.0, 0.0, 0.0, 0.0], seed=7)
    inst = [(0.3, 5, 12, 3000), (0.7, 2, 12, 2000), (0.5, 3, 4, 2500), (0.2, 4, 6, 1000),
            (0.9, 5, 8, 1), (0.4, 2, 2, 700), (0.6, 5, 12, 129), (0.25, 1, 12, 3000),
            (0.8, 3, 12, 1500), (0.35, 4, 1, 900)]
    say("batched: 10 small instances")
    b = Q.Basis(w.d, w.set_kind, w.level)
    full_reps = O.enumerate_set(w.d, w.set_kind, w.level)
    a = torch.full((len(inst), w.N, b.n_funcs), 7.0, dtype=torch.float64, device="cuda")
    ctx.solve_batched(Q.problem_from(w), b, inst, w.seed, a)
    torch.cuda.synchronize()
    got = host(a)
    for r, it in enumerate(inst):
        _check_batched_instance(got[r], w, full_reps, it, w.seed, range(w.N), what=f"instance {r} {it}")
    # deterministic
    a2 = torch.zeros_like(a)
    ctx.solve_batched(Q.problem_from(w), b, inst, w.seed, a2)
    torch.cuda.synchronize()
    assert torch.equal(a, a2)


def test_batched_equals_unbatched_full_set(env):
    """Instances on the whole basis give qr_solve's coefficients for their f_a."""
    Q, ctx, torch = env
    w = W.D2_TENSOR4
    b = Q.Basis(w.d, w.set_kind, w.level)
    fas = [0.2, 0.5, 0.9]
    say("batched vs qr_solve, d2 tensor")
    a = torch.zeros((len(fas), w.N, b.n_funcs), dtype=torch.float64, device="cuda")
    ctx.solve_batched(Q.problem_from(w), b, [(f, w.d, w.level, w.M) for f in fas], w.seed, a)
    for r, f in enumerate(fas):
        ref = torch.zeros((w.N, b.n_funcs), dtype=torch.float64, device="cuda")
        ctx.solve(Q.problem_from(w.with_(f_a=f)), b, w.M, w.seed, ref)
        torch.cuda.synchronize()
        err = (a[r] - ref).abs().max().item()
        assert err <= TOL * ref.abs().max().item(), (f, err)


def test_batched_shared_pass_projection(env):
    """Passes whose members fill the pass's set and cloud take the pass
    projection (all members' responses against one walk of the set): eight
    full-set members equal qr_solve for their f_a, and a pass with members of
    smaller sets and clouds (which then take their own projections) beside
    one of eight equal members agrees with the oracle."""
    Q, ctx, torch = env
    w = W.Workload(name="batch-shared", d=3, N=4, T=1.0, sigma=[[0.5 if a == b else 0.0 for b in range(3)]
                                                                for a in range(3)],
                   b0=[0.0] * 3, b1=[0.0] * 3, set_kind="hc_1p", level=12, M=3001, driver="sin",
                   f_a=0.5, sol_A=1.0, sol_c=1.0, sol_p=0.0, sol_w=[1.0, 1.0, 0.0], seed=9)
    b = Q.Basis(w.d, w.set_kind, w.level)
    fas = [0.1 * (k + 1) for k in range(8)]
    say("batched: eight full-set members (pass projection)")
    a = torch.zeros((len(fas), w.N, b.n_funcs), dtype=torch.float64, device="cuda")
    ctx.solve_batched(Q.problem_from(w), b, [(f, w.d, w.level, w.M) for f in fas], w.seed, a)
    torch.cuda.synchronize()
    for r, f in enumerate(fas):
        ref = torch.zeros((w.N, b.n_funcs), dtype=torch.float64, device="cuda")
        ctx.solve(Q.problem_from(w.with_(f_a=f)), b, w.M, w.seed, ref)
        torch.cuda.synchronize()
        err = (a[r] - ref).abs().max().item()
        assert err <= TOL * ref.abs().max().item(), (f, err)
    full_reps = O.enumerate_set(w.d, w.set_kind, w.level)
    inst = [(f, w.d, w.level, w.M) for f in fas] + [(0.3, 2, 6, 1500), (0.6, 3, 4, 700)]
    say("batched: shared pass plus a pass of smaller members")
    a = torch.full((len(inst), w.N, b.n_funcs), 7.0, dtype=torch.float64, device="cuda")
    ctx.solve_batched(Q.problem_from(w), b, inst, w.seed, a)
    torch.cuda.synchronize()
    got = host(a)
    for r in (0, 7, 8, 9):
        _check_batched_instance(got[r], w, full_reps, inst[r], w.seed, range(w.N), what=f"instance {r} {inst[r]}")


def test_batched_graph_replays_equal_the_eager_solve(env):
    """qr_batch_graph: the batched solve captured into one graph.  Its
    creation solves once; every replay, with the program's own eager work
    (a plain solve and a smaller batched solve on the same context, which
    grow and reuse its workspace) and synchronisations in between, gives
    the eager result bit for bit."""
    Q, ctx, torch = env
    w = W.Workload(name="batch-graph", d=5, N=4, T=1.0, sigma=[[0.5 if a == b else 0.0 for b in range(5)]
                                                               for a in range(5)],
                   b0=[0.0] * 5, b1=[0.0] * 5, set_kind="hc_1p", level=12, M=3000, driver="sin",
                   f_a=0.5, sol_A=1.0, sol_c=1.0, sol_p=0.0, sol_w=[1.0, 1.0, 0.0, 0.0, 0.0], seed=7)
    inst = [(0.3, 5, 12, 3000), (0.7, 2, 12, 2000), (0.5, 3, 4, 2500), (0.2, 4, 6, 1000),
            (0.9, 5, 8, 1), (0.4, 2, 2, 700), (0.6, 5, 12, 129), (0.25, 1, 12, 3000),
            (0.8, 3, 12, 1500), (0.35, 4, 1, 900)] + [(0.1 * k, 5, 12, 3000) for k in range(1, 9)]
    say("batched graph: create and replay")
    b = Q.Basis(w.d, w.set_kind, w.level)
    prob = Q.problem_from(w)
    ref = torch.zeros((len(inst), w.N, b.n_funcs), dtype=torch.float64, device="cuda")
    ctx.solve_batched(prob, b, inst, w.seed, ref)
    torch.cuda.synchronize()
    st = torch.cuda.Stream()
    a = torch.full_like(ref, 7.0)
    torch.cuda.synchronize()
    g = ctx.batch_graph(prob, b, inst, w.seed, a, st)
    st.synchronize()
    assert torch.equal(a, ref)
    with pytest.raises(Q.QrError):
        ctx.batch_graph(prob, b, inst, w.seed, a, None)  # the null stream cannot be captured
    try:
        for k in range(3):
            a.fill_(float(k))
            other = torch.zeros((w.N, b.n_funcs), dtype=torch.float64, device="cuda")
            ctx.solve(Q.problem_from(w.with_(f_a=0.1 * k)), b, w.M + 17 * k, k, other)
            small = torch.zeros((2, w.N, b.n_funcs), dtype=torch.float64, device="cuda")
            ctx.solve_batched(prob, b, inst[:2], k, small)
            torch.cuda.synchronize()
            g.launch(st)
            st.synchronize()
            assert torch.equal(a, ref), f"replay {k}"
    finally:
        g.close()


def test_batched_invalid_arguments(env):
    Q, ctx, torch = env
    w = W.D2_TENSOR4
    b = Q.Basis(w.d, w.set_kind, w.level)
    a = torch.zeros((65, w.N, b.n_funcs), dtype=torch.float64, device="cuda")
    prob = Q.problem_from(w)
    for bad in ([], [(0.5, 2, 4, 100)] * 65, [(0.5, 3, 4, 100)], [(0.5, 2, 5, 100)],
                [(0.5, 2, 4, 0)], [(math.nan, 2, 4, 10)], [(0.5, 0, 4, 10)], [(0.5, 2, -1, 10)]):
        with pytest.raises(Q.QrError):
            ctx.solve_batched(prob, b, bad, 0, a)
    with pytest.raises(Q.QrError) as e:
        ctx.solve_batched(Q.problem_from(w.with_(driver="zrat")), b, [(0.5, 2, 4, 10)], 0, a)
    assert e.value.status == -6


def test_batched_group_full_size_sampled(env):
    """The first group of 64 of the 256-instance workload at its real sizes
    (d up to 12, levels 8/16/32, M up to 2^20): the last step's coefficients
    of three instances on sampled functions, and the step before for the
    instance with the smallest set."""
    Q, ctx, torch = env
    gw, inst, _ = W.batched_group(W.batched_instances())[0]
    b = Q.Basis(gw.d, gw.set_kind, gw.level)
    full_reps = O.enumerate_set(gw.d, gw.set_kind, gw.level)
    say(f"batched group 0: d={gw.d} level={gw.level} M={gw.M} R={len(inst)} n_funcs={b.n_funcs}")
    a = torch.zeros((len(inst), gw.N, b.n_funcs), dtype=torch.float64, device="cuda")
    ctx.solve_batched(Q.problem_from(gw), b, inst, gw.seed, a)
    torch.cuda.synchronize()
    sizes = [O.enumerate_set(d, gw.set_kind, L).shape[0] for _, d, L, _ in inst]
    order = np.argsort(sizes)
    rng = np.random.default_rng(5)
    for r in [int(order[-1]), int(order[len(order) // 2]), int(order[0])]:
        f_a, d_r, level_r, M_r = inst[r]
        say(f"  instance {r}: d={d_r} level={level_r} M={M_r} reps={sizes[r]}")
        wr = gw.with_(f_a=f_a)
        reps = _embed(O.enumerate_set(d_r, gw.set_kind, level_r), gw.d)
        pick = np.concatenate([[0], np.sort(rng.choice(np.arange(1, reps.shape[0]),
                                                       min(16, reps.shape[0] - 1), replace=False))])
        sub = np.ascontiguousarray(reps[pick])
        got = host(a[r])
        ref, absum, _, _ = O.backward_step(wr, sub, gw.N - 1, M_r, gw.seed,
                                           np.zeros((gw.N, 2 * len(pick) - 1)))
        assert_alpha(got[gw.N - 1, _func_index(full_reps, sub)], ref, absum,
                      what=f"instance {r} step N-1")
    r = int(order[0])
    f_a, d_r, level_r, M_r = inst[r]
    wr = gw.with_(f_a=f_a)
    reps = _embed(O.enumerate_set(d_r, gw.set_kind, level_r), gw.d)
    idx = _func_index(full_reps, reps)
    got = host(a[r])
    prev = np.zeros((gw.N, len(idx)))
    prev[gw.N - 1] = got[gw.N - 1, idx]
    say(f"  instance {r}: step N-2 in full")
    ref, absum, _, _ = O.backward_step(wr, reps, gw.N - 2, M_r, gw.seed, prev)
    assert_alpha(got[gw.N - 2, idx], ref, absum, what=f"instance {r} step N-2")


# ---------------------------------------------------------------------------
# the benchmark's workload at its full size (d = 6, 169,209 functions,
# M = 2^20): the launch configurations the benchmark times, checked on
# outputs the oracle computes one by one
# ---------------------------------------------------------------------------

def test_path_responses_bench_size_sampled(env):
    """Step i = 0 (all 20 Euler steps and 19 expansion levels) for 2^20 paths;
    sampled responses against the oracle's path by path."""
    Q, ctx, torch = env
    w = W.D6_HCMAX16
    M, i = w.M, 0
    say(f"path_responses {w.name} i={i} M={M}")
    b = Q.Basis(w.d, w.set_kind, w.level)
    reps = O.reps_for(w)
    alpha = W.synthetic_alpha(b.n_funcs, w.N, seed=17, scale=0.05, decay=0.8)
    s = torch.empty(M, dtype=torch.float64, device="cuda")
    ctx.path_responses(Q.problem_from(w), b, i, M, w.seed, dev(torch, alpha), s)
    torch.cuda.synchronize()
    sg = host(s)
    assert np.isfinite(sg).all()
    for m in [0, 255, 256, 131071, 524288, M - 1]:
        ref = O.path_response(w, reps, i, w.seed, m, alpha)
        assert abs(sg[m] - ref) <= TOL * max(1.0, abs(ref)), (m, sg[m], ref)


def test_project_bench_size_sampled(env):
    """Projection of 2^20 points on the full d = 6 basis (the benchmark's
    projection shape); sampled coefficients against the oracle, which projects
    the same points on just the sampled representatives."""
    Q, ctx, torch = env
    w = W.D6_HCMAX16
    n = w.M
    say(f"project {w.name} n={n}")
    b = Q.Basis(w.d, w.set_kind, w.level)
    reps = O.reps_for(w)
    x = W.logistic_points(n, w.d, seed=23)
    s = W.responses(n, seed=29)
    a = torch.empty(b.n_funcs, dtype=torch.float64, device="cuda")
    ctx.project(b, dev(torch, x.T), dev(torch, s), a)
    torch.cuda.synchronize()
    got = host(a)
    rng = np.random.default_rng(31)
    picks = np.unique(np.concatenate([[1, 2, reps.shape[0] - 1], rng.integers(1, reps.shape[0], 9)]))
    sub = np.concatenate([reps[:1], reps[picks]])           # the zero vector first
    ref, absum = O.project(sub, x, s, with_abs=True)
    idx = np.concatenate([[0], np.stack([2 * picks - 1, 2 * picks], axis=1).ravel()])
    assert_alpha(got[idx], ref, absum, what="bench-size projection")


# ---------------------------------------------------------------------------
# non-finite coefficients (QR_ENUMERIC)
# ---------------------------------------------------------------------------

def test_non_finite_coefficients_are_reported(env):
    """A manufactured solution of amplitude 1e120 makes the Allen-Cahn source
    h = ... - (u - u^3) overflow to infinity along the paths from the first
    iteration on: the full solves return QR_ENUMERIC naming time index N-1,
    an asynchronous backward step leaves the record for
    qr_ctx_numeric_status, and a finite problem afterwards reports nothing."""
    Q, ctx, torch = env
    w = W.D2_TENSOR4.with_(driver="allen_cahn", sol_A=1e120, clamp=math.inf, M=500)
    b = Q.Basis(w.d, w.set_kind, w.level)
    a = torch.zeros((w.N, b.n_funcs), dtype=torch.float64, device="cuda")
    say("numeric flag: overflowing driver")
    for solve in (lambda: ctx.solve(Q.problem_from(w), b, w.M, w.seed, a),
                  lambda: ctx.solve_prec(Q.problem_from(w), b, w.M, w.seed, "bf16", a),
                  lambda: ctx.solve_batched(Q.problem_from(w), b, [(0.0, w.d, w.level, w.M)], w.seed, a[None])):
        with pytest.raises(Q.QrError) as e:
            solve()
        assert e.value.status == -5 and f"time index {w.N - 1}" in str(e.value)
    assert ctx.numeric_status() == -1           # the solves cleared their record
    ctx.backward_step(Q.problem_from(w), b, w.N - 1, w.M, w.seed, a)
    with pytest.raises(Q.QrError) as e:
        ctx.numeric_status()
    assert e.value.status == -5
    assert ctx.numeric_status() == -1           # read and cleared
    ok = W.D2_TENSOR4.with_(M=500)
    ctx.solve(Q.problem_from(ok), b, ok.M, ok.seed, a)
    ctx.backward_step(Q.problem_from(ok), b, 0, ok.M, ok.seed, a)
    assert ctx.numeric_status() == -1
