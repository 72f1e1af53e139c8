"""Reduced-precision form, factored kernel (qr_ctx_set_prec_kernel "factored"):
the expansion along the paths and the projection as products of the
staircase coefficient matrix with the paths' basis factors on the matrix
cores, against the FP64 oracle on the same Philox streams, in the relative
2-norm of each alpha row.

Tolerance (rounding model).  The expansion carries the error of the walk
kernel's (about u relative to S; test_gpu_precision.py).  The projection now
rounds W = S EA and EB to 16 bits as well: each term S phi_k(X_m) of the
Monte-Carlo sum gets an independent relative error of rms (2/sqrt3) u, so a
coefficient moves by about 1.15 u sqrt(sum_m (S phi_k)^2) / M, which is
1.15 u of the row's norm when alpha is dominated by the Monte-Carlo
variance (these rows are).  REL = 2u covers both (7.8e-3 bf16, 9.8e-4 half);
layout or indexing mistakes give O(1) errors.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_common import env, dev, host, say, rel_err  # noqa: F401 (env is a fixture)

pytestmark = pytest.mark.gpu

UNIT = {"bf16": 2.0 ** -8, "f16": 2.0 ** -11}
REL = {p: 2 * u for p, u in UNIT.items()}


def _w(d, set_kind, level, driver, M, N=4, f_a=0.5, clamp=float("inf"), b1=0.0):
    return W.Workload(name=f"fac-d{d}-{set_kind}{level}-{driver}", d=d, N=N, T=1.0,
                      sigma=[[0.5 if a == c else 0.0 for c in range(d)] for a in range(d)],
                      b0=[0.0] * d, b1=[b1] * d, set_kind=set_kind, level=level, M=M, driver=driver,
                      f_a=f_a, sol_A=1.0, sol_c=1.0, sol_p=0.0,
                      sol_w=[1.0 if l < 2 else 0.0 for l in range(d)], seed=11, clamp=clamp)


CASES = [
    (1, "tensor", 6, "sin", 777),
    (2, "tensor", 4, "sin", 1000),
    (3, "hc_1p", 12, "allen_cahn", 2049),
    (5, "hc_max", 9, "sin", 1500),
    (6, "hc_max", 16, "allen_cahn", 1024),
    (12, "hc_1p", 8, "sin", 600),
]


@pytest.mark.parametrize("prec", ["bf16", "f16"])
@pytest.mark.parametrize("case", CASES, ids=[f"d{c[0]}-{c[1]}{c[2]}-{c[3]}" for c in CASES])
def test_fac_backward_step(env, prec, case):
    d, kind, level, driver, M = case
    Q, ctx, torch = env
    w = _w(d, kind, level, driver, M, clamp=2.0 if driver == "allen_cahn" else float("inf"))
    b = Q.Basis(w.d, w.set_kind, w.level)
    lay = b.factored()
    assert lay is not None
    say(f"factored {prec} {w.name} M={M} split={lay[0]} tiles={lay[1]} kblocks={lay[2]} blocks={lay[3]}")
    reps = O.reps_for(w)
    alpha = W.synthetic_alpha(b.n_funcs, w.N, seed=d + 100, scale=0.2, decay=0.7)
    ctx.set_prec_kernel("factored")
    try:
        for i in (w.N - 2, 0):
            a = dev(torch, alpha)
            ctx.backward_step_prec(Q.problem_from(w), b, i, w.M, w.seed, prec, a)
            torch.cuda.synchronize()
            ref, _, _, _ = O.backward_step(w, reps, i, w.M, w.seed, alpha.copy())
            err = rel_err(host(a)[i], ref)
            say(f"  row {i}: rel err {err:.3e} (tol {REL[prec]:.1e})")
            assert err <= REL[prec], (i, err)
    finally:
        ctx.set_prec_kernel("auto")


@pytest.mark.parametrize("prec", ["bf16", "f16"])
def test_fac_solve_d2(env, prec):
    """Full solve of the d = 2 tensor workload with the factored kernel:
    every row against the oracle."""
    Q, ctx, torch = env
    w = W.D2_TENSOR4
    b = Q.Basis(w.d, w.set_kind, w.level)
    reps = O.reps_for(w)
    a = torch.zeros((w.N, b.n_funcs), dtype=torch.float64, device="cuda")
    ctx.set_prec_kernel("factored")
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


def test_fac_kernel_choice(env):
    """auto picks the factored kernel for value drivers (same result as forcing
    it); forcing it with a z-dependent driver is QR_ENOTSUP."""
    Q, ctx, torch = env
    w = _w(3, "hc_1p", 12, "sin", 500)
    b = Q.Basis(w.d, w.set_kind, w.level)
    alpha = W.synthetic_alpha(b.n_funcs, w.N, seed=7, scale=0.2, decay=0.7)
    outs = {}
    for k in ("auto", "factored", "walk"):
        ctx.set_prec_kernel(k)
        a = dev(torch, alpha)
        ctx.backward_step_prec(Q.problem_from(w), b, 1, w.M, w.seed, "bf16", a)
        torch.cuda.synchronize()
        outs[k] = host(a)[1]
    ctx.set_prec_kernel("auto")
    assert np.array_equal(outs["auto"], outs["factored"])
    assert not np.array_equal(outs["walk"], outs["factored"])
    wz = _w(3, "hc_1p", 12, "zrat", 500, f_a=-0.5)
    ctx.set_prec_kernel("factored")
    try:
        with pytest.raises(Q.QrError) as e:
            ctx.backward_step_prec(Q.problem_from(wz), b, 1, wz.M, wz.seed, "bf16", dev(torch, alpha))
        assert e.value.status == -6
    finally:
        ctx.set_prec_kernel("auto")
    with pytest.raises(Q.QrError):
        ctx.set_prec_kernel(9)
