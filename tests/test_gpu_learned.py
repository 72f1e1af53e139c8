"""Learned form: the surrogate network's kernels against the FP64 network
definition (oracle/mlp.py), and the learned solve.

Tolerances.  The kernels round the operands of every matrix product to
bfloat16 and sum in FP32; the reference that rounds the same operands
(forward_bf16 / loss_grad_bf16) then differs only by FP32 summation and the
rare operand that rounds the other way, so outputs and gradients are
compared with it to 2e-3 relative (2-norm per parameter block).  Against the
exact FP64 network the bfloat16 effect itself, O(2^-8), is allowed (3e-2).
"""

import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_common import env, say, rel_err  # noqa: F401 (env is a fixture)
from oracle import mlp

pytestmark = pytest.mark.gpu


def _f32(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


def _theta(seed):
    """Fan-in uniform weights and small nonzero biases, as float32 values."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in mlp.SIZES:
        fan = 16 if name == "W1" else 256
        p[name] = rng.uniform(-1, 1, shape) / np.sqrt(fan) if name[0] in "Ww" else rng.uniform(-0.1, 0.1, shape)
    return mlp.pack(p).astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("n", [1, 100, 4097])
def test_forward_against_oracle(env, n):
    Q, ctx, torch = env
    say(f"mlp forward n={n}")
    th = _theta(1)
    f = np.random.default_rng(n).uniform(-1, 1, (n, 16)).astype(np.float32).astype(np.float64)
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    ctx.mlp_forward(_f32(torch, th), _f32(torch, f), y)
    torch.cuda.synchronize()
    got = y.cpu().numpy().astype(np.float64)
    yb, _ = mlp.forward_bf16(th, f)
    ye, _ = mlp.forward(th, f)
    say(f"  vs bf16-operand reference {rel_err(got, yb):.2e}, vs exact {rel_err(got, ye):.2e}")
    assert rel_err(got, yb) <= 2e-3
    assert rel_err(got, ye) <= 3e-2


def test_loss_gradient_against_oracle(env):
    Q, ctx, torch = env
    n = 3000
    say("mlp loss gradient")
    rng = np.random.default_rng(7)
    th = _theta(2)
    f = rng.uniform(-1, 1, (n, 16)).astype(np.float32).astype(np.float64)
    t = rng.standard_normal(n).astype(np.float32).astype(np.float64)
    g = torch.empty(mlp.NPARAMS, dtype=torch.float32, device="cuda")
    loss = ctx.mlp_loss_grad(_f32(torch, th), _f32(torch, f), _f32(torch, t), g)
    got = g.cpu().numpy().astype(np.float64)
    lb, gb = mlp.loss_grad_bf16(th, f, t)
    le, ge = mlp.loss_grad(th, f, t)
    assert abs(loss - lb) <= 1e-4 * lb
    off = np.cumsum([0] + [int(np.prod(s)) for _, s in mlp.SIZES])
    for k, (name, _) in enumerate(mlp.SIZES):
        sl = slice(off[k], off[k + 1])
        rb, re = rel_err(got[sl], gb[sl]), rel_err(got[sl], ge[sl])
        say(f"  {name}: vs bf16-operand {rb:.2e}, vs exact {re:.2e}")
        assert rb <= 2e-3, name
        assert re <= 3e-2, name


def test_adam_step_against_oracle(env):
    Q, ctx, torch = env
    rng = np.random.default_rng(3)
    th = rng.standard_normal(mlp.NPARAMS).astype(np.float32).astype(np.float64)
    g = rng.standard_normal(mlp.NPARAMS).astype(np.float32).astype(np.float64)
    m = (0.1 * rng.standard_normal(mlp.NPARAMS)).astype(np.float32).astype(np.float64)
    v = (0.1 * rng.random(mlp.NPARAMS)).astype(np.float32).astype(np.float64)
    tt, tg, tm, tv = (_f32(torch, a) for a in (th, g, m, v))
    ctx.mlp_adam(tt, tg, tm, tv, 5, 1e-3)
    torch.cuda.synchronize()
    rt, rm, rv = mlp.adam(th, g, m, v, 5, 1e-3)
    # FP32 arithmetic: errors relative to the size of the terms combined
    # (the moment updates can cancel)
    assert np.all(np.abs(tm.cpu().numpy() - rm) <= 1e-6 * (0.9 * np.abs(m) + 0.1 * np.abs(g)))
    assert np.all(np.abs(tv.cpu().numpy() - rv) <= 1e-6 * (0.999 * v + 0.001 * g * g))
    assert np.all(np.abs(tt.cpu().numpy() - rt) <= 1e-6 * (np.abs(th) + 1e-3))


def test_features_and_init(env):
    Q, ctx, torch = env
    x = np.random.default_rng(8).logistic(size=(300, 5))
    feat = torch.empty((300, 16), dtype=torch.float32, device="cuda")
    ctx.mlp_features(5, torch.as_tensor(np.ascontiguousarray(x.T), device="cuda"), feat)
    th = torch.empty(mlp.NPARAMS, dtype=torch.float32, device="cuda")
    ctx.mlp_init(th, 11)
    torch.cuda.synchronize()
    assert np.allclose(feat.cpu().numpy(), mlp.features(x), atol=1e-7)
    p = mlp.unpack(th.cpu().numpy().astype(np.float64))
    assert np.abs(p["W1"]).max() <= 0.25 and np.abs(p["W2"]).max() <= 1 / 16
    assert not p["b1"].any() and not p["b2"].any() and p["b3"][0] == 0
    assert p["W2"].std() > 0.03      # uniform on [-1/16, 1/16]: std 0.036


def test_training_fits_a_smooth_function(env):
    """The kernels train: 600 full-batch Adam steps on a smooth target bring
    the loss down by two orders of magnitude."""
    Q, ctx, torch = env
    rng = np.random.default_rng(9)
    n = 8192
    f = rng.uniform(-1, 1, (n, 16))
    t = np.sin(np.pi * f[:, 0]) * np.cos(np.pi * f[:, 1]) + 0.5 * f[:, 2]
    th = torch.empty(mlp.NPARAMS, dtype=torch.float32, device="cuda")
    ctx.mlp_init(th, 1)
    g, m, v = (torch.zeros(mlp.NPARAMS, dtype=torch.float32, device="cuda") for _ in range(3))
    tf, tt = _f32(torch, f), _f32(torch, t)
    first = None
    for step in range(1, 601):
        loss = ctx.mlp_loss_grad(th, tf, tt, g)
        first = loss if first is None else first
        ctx.mlp_adam(th, g, m, v, step, 3e-3)
    say(f"  loss {first:.3e} -> {loss:.3e}")
    assert loss < 2e-2 * first


def _report(rep):
    return " ".join(f"{j}:{r['heldout_rel_l2']:.1e}{'*' if r['used'] else ''}" for j, r in enumerate(rep))


def test_learned_solve_with_closed_gate_is_the_plain_solve(env):
    """Gate 0: every surrogate is fitted and rejected, so every iteration runs
    the fused path kernel of qr_solve and the result is qr_solve's."""
    Q, ctx, torch = env
    w = W.D2_TENSOR4
    b = Q.Basis(w.d, w.set_kind, w.level)
    a = torch.zeros((w.N, b.n_funcs), dtype=torch.float64, device="cuda")
    rep = ctx.solve_learned(Q.problem_from(w), b, w.M, w.seed, a, train_points=1 << 12, heldout_points=1 << 10,
                            epochs=1, batch=1024, gate=0.0)
    ref = torch.zeros_like(a)
    ctx.solve(Q.problem_from(w), b, w.M, w.seed, ref)
    torch.cuda.synchronize()
    say("  " + _report(rep))
    assert all(r["trained"] and not r["used"] for r in rep[1:]) and not rep[0]["trained"]
    # no iteration has a surrogate ahead of it: qr_solve's own kernels, bit for bit
    assert torch.equal(a, ref)
    # and against the oracle
    got = a.cpu().numpy()
    oref = O.solve(w, O.reps_for(w))
    assert np.abs(got - oref).max() <= 1e-10 * np.abs(oref).max()


def test_learned_early_rejection(env):
    """A cloud of 100 paths for 81 functions: each ybar_j is Monte-Carlo
    noise, which no network fits.  With reject = 0.5 every screen (all four
    epochs on 1/32 of the pairs) ends above 0.5 and no full fit runs, none is
    used, and the result is qr_solve's bit for bit; without it the full fit
    runs every epoch."""
    Q, ctx, torch = env
    w = W.D2_TENSOR4.with_(M=100)
    b = Q.Basis(w.d, w.set_kind, w.level)
    ref = torch.zeros((w.N, b.n_funcs), dtype=torch.float64, device="cuda")
    ctx.solve(Q.problem_from(w), b, w.M, w.seed, ref)
    for reject in (0.5, 0.0):
        a = torch.zeros_like(ref)
        rep = ctx.solve_learned(Q.problem_from(w), b, w.M, w.seed, a, train_points=1 << 13,
                                heldout_points=1 << 10, epochs=4, batch=256, reject=reject)
        torch.cuda.synchronize()
        say(f"  reject={reject}: " + _report(rep) + " epochs " + " ".join(str(r["epochs_run"]) for r in rep))
        assert all(r["trained"] and not r["used"] and r["epochs_run"] == 4 for r in rep[1:])
        if reject:
            assert all(r["heldout_rel_l2"] > 0.5 for r in rep[1:])
        assert torch.equal(a, ref)


def test_learned_screen_passes_a_learnable_target(env):
    """A screen that ends within `reject` hands over to the full fit, which
    is the same fit as without a screen: on the level-1 set of the next test
    (expansions of degree 1) the screen's fit on 1/32 of the pairs ends at
    a held-out error of about 0.8 (the full fit reaches 0.04 to 0.09), so
    with reject = 0.95 every screen passes and the same time indices use
    their surrogate as without a screen.  (With reject = 0.5 these screens
    would turn the surrogates away: the screen trades recall for cost.)"""
    Q, ctx, torch = env
    w = W.D2_TENSOR4.with_(level=1)
    b = Q.Basis(w.d, w.set_kind, w.level)
    used = {}
    for reject in (0.0, 0.95):
        a = torch.zeros((w.N, b.n_funcs), dtype=torch.float64, device="cuda")
        rep = ctx.solve_learned(Q.problem_from(w), b, w.M, w.seed, a, train_points=1 << 16,
                                heldout_points=1 << 14, epochs=40, batch=1024, lr=2e-3, gate=5e-2, reject=reject)
        torch.cuda.synchronize()
        say(f"  reject={reject}: " + _report(rep))
        used[reject] = [j for j, r in enumerate(rep) if r["used"]]
    assert used[0.0], "no surrogate passed the gate"
    assert used[0.95] == used[0.0]


def test_learned_solve_uses_the_surrogate_where_it_passes(env):
    """d = 2 tensor set of level 1 (9 functions): the expansions are
    trigonometric polynomials of degree 1, which the network fits within this
    training budget.  With a gate of 5e-2 (the default gate, 1e-3, is beyond
    this budget) the surrogate replaces the expansion where it passes, and
    each row of alpha moves by no more than the surrogate's error allows: the
    driver is 0.5-Lipschitz in y, so S moves by at most 0.5 T gate ||y||
    (T = 1), taken with a factor 3 of margin."""
    Q, ctx, torch = env
    w = W.D2_TENSOR4.with_(level=1)
    b = Q.Basis(w.d, w.set_kind, w.level)
    a = torch.zeros((w.N, b.n_funcs), dtype=torch.float64, device="cuda")
    gate = 5e-2
    rep = ctx.solve_learned(Q.problem_from(w), b, w.M, w.seed, a, train_points=1 << 16, heldout_points=1 << 14,
                            epochs=40, batch=1024, lr=2e-3, gate=gate)
    ref = torch.zeros_like(a)
    ctx.solve(Q.problem_from(w), b, w.M, w.seed, ref)
    torch.cuda.synchronize()
    say("  " + _report(rep))
    used = [j for j, r in enumerate(rep) if r["used"]]
    assert used, "no surrogate passed the gate"
    got, r64 = a.cpu().numpy(), ref.cpu().numpy()
    for i in range(w.N):
        e = rel_err(got[i], r64[i])
        say(f"  row {i}: rel change {e:.2e}")
        assert e <= 3 * gate


def test_learned_solve_gate_open_matches_oracle(env):
    """Every fitted surrogate used (gate 1e9): each row i of the GPU's alpha
    against the oracle's learned step, which evaluates y_j = target_mean +
    target_sd * network_j (the fitted parameters, bfloat16 operands of the
    two matrix products, sums exact) in place of the expansion for every
    later time index, and the expansion of the GPU's rows elsewhere.  The
    kernels sum the products in FP32: the 256-term layer-2 sum carries a
    rounding error of at most 256 * 2^-24 = 1.5e-5 of the sum of its absolute
    terms, and about sqrt(256) * 2^-24 = 1e-6 of it for independent roundings;
    each response moves by that fraction of target_sd at most, and alpha is
    compared to 1e-6 relative to max(|alpha_k|, A_k) and in the row 2-norm."""
    from gpu_common import assert_alpha
    Q, ctx, torch = env
    w = W.D2_TENSOR4.with_(M=2000)
    b = Q.Basis(w.d, w.set_kind, w.level)
    reps = O.reps_for(w)
    a = torch.zeros((w.N, b.n_funcs), dtype=torch.float64, device="cuda")
    params = torch.empty((w.N, Q.MLP_NPARAMS), dtype=torch.float32, device="cuda")
    rep = ctx.solve_learned(Q.problem_from(w), b, w.M, w.seed, a, train_points=1 << 12, heldout_points=1 << 10,
                            epochs=2, batch=1024, gate=1e9, params=params)
    torch.cuda.synchronize()
    say("  " + _report(rep))
    assert all(r["used"] for r in rep[1:])
    th = params.cpu().numpy().astype(np.float64)
    assert not th[0].any()
    got = a.cpu().numpy()
    nets = [th[j] if rep[j]["used"] else None for j in range(w.N)]
    mu = [r["target_mean"] for r in rep]
    sd = [r["target_sd"] for r in rep]
    worst = 0.0
    for i in range(w.N - 1, -1, -1):
        ref, absum = O.backward_step_learned(w, reps, i, w.M, w.seed, got.copy(), nets, mu, sd)
        scale = np.maximum(np.abs(ref), absum)
        worst = max(worst, float(np.max(np.abs(got[i] - ref) / scale)))
        assert_alpha(got[i], ref, absum, tol=1e-6, what=f"learned row {i}")
    say(f"  worst |dalpha| / max(|alpha|, A): {worst:.2e}")
    # the surrogate changed the result: the rows differ from the plain solve
    plain = torch.zeros_like(a)
    ctx.solve(Q.problem_from(w), b, w.M, w.seed, plain)
    torch.cuda.synchronize()
    assert rel_err(got[0], plain.cpu().numpy()[0]) > 1e-6


def test_learned_solve_invalid_options(env):
    Q, ctx, torch = env
    w = W.D2_TENSOR4
    b = Q.Basis(w.d, w.set_kind, w.level)
    a = torch.zeros((w.N, b.n_funcs), dtype=torch.float64, device="cuda")
    prob = Q.problem_from(w)
    for kw in ({"batch": 32}, {"epochs": -1}, {"train_points": 100, "batch": 1024}, {"heldout_points": 0},
               {"lr": 0.0}, {"gate": -1.0}, {"reject": -1.0}):
        with pytest.raises(Q.QrError):
            ctx.solve_learned(prob, b, 100, 0, a, **kw)
    with pytest.raises(Q.QrError) as e:
        ctx.solve_learned(Q.problem_from(w.with_(driver="zrat")), b, 100, 0, a)
    assert e.value.status == -6
