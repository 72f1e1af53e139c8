"""Reduced-precision form (qr_*_prec), walk kernel: the expansion along the
paths is evaluated with 16-bit basis values and coefficients on the matrix
cores (FP32 accumulation); the projection and everything else stay FP64.

Tolerance (rounding model).  Each term c_k phi_k of the expansion is formed
from a 16-bit coefficient and a 16-bit basis value: a relative error of at
most 2u + u^2 (u = 2^-8 for bfloat16, 2^-11 for IEEE half), independent from
term to term, so the evaluation error has an rms of about (2/sqrt3) u ||c||_2
= 1.15 u ||ybar||.  It reaches S through the driver, scaled by |df/dy| dt
(and |df/dz| |sigma| dt for the gradient right-hand sides) per step, summed
over at most T = 1, with |df/dy| <= 1 and |df/dz| |z| <= 2 |f_a| for these
drivers; S and the rows of alpha then move by about u relative for the
parameter values here.  Rows are compared with the FP64 oracle in the
relative 2-norm against REL = u (3.9e-3 bf16, 4.9e-4 half), a few times the
measured errors; a wrong tile layout or a wrong gradient group moves S by
O(|f_a|) and fails it (the f_a = -2 cases make the gradient terms carry
weight).
"""

import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_common import env, dev, host, say, rel_err  # noqa: F401 (env is a fixture)

pytestmark = pytest.mark.gpu

UNIT = {"bf16": 2.0 ** -8, "f16": 2.0 ** -11}
REL = dict(UNIT)


def _zrat_small(d=3, f_a=-0.05):
    return W.Workload(name="zrat-small", d=d, N=4, T=1.0,
                      sigma=[[0.5 if a == b else 0.0 for b in range(d)] for a in range(d)],
                      b0=[0.0] * d, b1=[0.0] * d, set_kind="hc_1p", level=12, M=4000, driver="zrat",
                      f_a=f_a, sol_A=1.0, sol_c=1.0, sol_p=0.0,
                      sol_w=[1.0 if l < 2 else 0.0 for l in range(d)], seed=5)


@pytest.mark.parametrize("prec", ["bf16", "f16"])
@pytest.mark.parametrize("d,f_a", [(3, -0.05), (6, -0.05), (10, -0.05), (13, -0.05), (16, -0.05),
                                   (3, -2.0), (10, -2.0)])
def test_prec_backward_step_gradient_driver(env, prec, d, f_a):
    """z-dependent driver: value and d gradient components as right-hand
    sides (2, 2, 3, 4 and 5 groups of four for d = 3, 6, 10, 13, 16); with
    f_a = -2 the gradient terms move S by O(1)."""
    Q, ctx, torch = env
    w = _zrat_small(d, f_a)
    say(f"prec backward step zrat d={d} f_a={f_a} {prec}")
    b = Q.Basis(w.d, w.set_kind, w.level)
    reps = O.reps_for(w)
    alpha = W.synthetic_alpha(b.n_funcs, w.N, seed=d, scale=0.2, decay=0.7)
    for i in (w.N - 2, 0):
        a = dev(torch, alpha)
        ctx.backward_step_prec(Q.problem_from(w), b, i, w.M, w.seed, prec, a)
        torch.cuda.synchronize()
        ref, _, _, _ = O.backward_step(w, reps, i, w.M, w.seed, alpha.copy())
        err = rel_err(host(a)[i], ref)
        say(f"  row {i}: rel err {err:.3e} (tol {REL[prec]:.1e})")
        assert err <= REL[prec], (i, err)


@pytest.mark.parametrize("prec", ["bf16", "f16"])
def test_prec_solve_value_driver(env, prec):
    """Value-only driver (one right-hand side): full solve of the d=2 tensor
    workload against the oracle row by row, and the closed-form error."""
    Q, ctx, torch = env
    w = W.D2_TENSOR4
    say(f"prec solve d2 tensor {prec}")
    b = Q.Basis(w.d, w.set_kind, w.level)
    reps = O.reps_for(w)
    a = torch.zeros((w.N, b.n_funcs), dtype=torch.float64, device="cuda")
    ctx.set_prec_kernel("walk")
    try:
        ctx.solve_prec(Q.problem_from(w), b, w.M, w.seed, prec, a)
    finally:
        ctx.set_prec_kernel("auto")
    torch.cuda.synchronize()
    got = host(a)
    ref = O.solve(w, reps)
    errs = [rel_err(got[i], ref[i]) for i in range(w.N)]
    say("  per-row rel err " + " ".join(f"{e:.1e}" for e in errs))
    assert max(errs) <= REL[prec]
    # error against u(0,.) at the stream-1 test points: the precision form
    # does not move the method's error
    n = 1 << 14
    x = torch.empty((w.d, n), dtype=torch.float64, device="cuda")
    ctx.sample_points(w.d, w.seed, 1, 0, n, x)
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    ctx.eval(b, a[0].contiguous(), x, y)
    torch.cuda.synchronize()
    xh = host(x).T
    u = np.exp(-1.0) * np.cos(xh[:, 0] + xh[:, 1])
    rel = np.linalg.norm(host(y) - u) / np.linalg.norm(u)
    _, _, rel64 = O.errors(w, reps, ref, seed=w.seed, n=n)
    say(f"  closed-form rel L2: {rel:.4f} vs FP64 {rel64:.4f}")
    assert abs(rel - rel64) <= 0.02 * rel64


def test_prec_full_basis_gradient_sampled(env):
    """The d=10 hyperbolic cross prod(1+|k_l|) <= 32 (85,485 functions) with
    the z-dependent driver: step N-2 at M = 2^16 in bfloat16 against the oracle."""
    Q, ctx, torch = env
    w = W.D10_HC1P32_ZRAT.with_(M=1 << 16)
    say("prec d10 hc_1p basis, step N-2, M=2^16")
    b = Q.Basis(w.d, w.set_kind, w.level)
    reps = O.reps_for(w)
    alpha = W.synthetic_alpha(b.n_funcs, w.N, seed=31, scale=0.1, decay=0.8)
    i = w.N - 2
    for prec in ("bf16", "f16"):
        a = dev(torch, alpha)
        ctx.backward_step_prec(Q.problem_from(w), b, i, w.M, w.seed, prec, a)
        torch.cuda.synchronize()
        if prec == "bf16":
            ref, _, _, _ = O.backward_step(w, reps, i, w.M, w.seed, alpha.copy())
        err = rel_err(host(a)[i], ref)
        say(f"  {prec}: rel err {err:.3e}")
        assert err <= REL[prec]


def test_prec_invalid_and_f64_passthrough(env):
    Q, ctx, torch = env
    w = W.D2_TENSOR4
    b = Q.Basis(w.d, w.set_kind, w.level)
    a = torch.zeros((w.N, b.n_funcs), dtype=torch.float64, device="cuda")
    with pytest.raises(Q.QrError):
        ctx.solve_prec(Q.problem_from(w), b, 100, 0, 7, a)
    # QR_PREC_F64 is the plain path, bit for bit
    a2 = torch.zeros_like(a)
    ctx.solve_prec(Q.problem_from(w), b, 1000, 0, "f64", a)
    ctx.solve(Q.problem_from(w), b, 1000, 0, a2)
    torch.cuda.synchronize()
    assert torch.equal(a, a2)
