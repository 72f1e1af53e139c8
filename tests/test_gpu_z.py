"""GPU parity of the gradient component: the regressions of Z_i of the
multistep scheme, eq (MDP:intro:0a), and of the one-step scheme, eq
(ODP:intro:a), through qr_backward_step_z / qr_solve_z against the oracle's
steps (same Philox streams, FP64, tolerance as for the Y rows), the solve
against its steps, the argument checks, and the estimates against
sigma^T grad u of the manufactured solution at a large cloud."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_common import env, dev, host, say, assert_alpha  # noqa: F401 (env is a fixture)

pytestmark = pytest.mark.gpu


def _diag_workload(name, d, N, set_kind, level, M, driver, f_a=0.0, seed=3):
    return W.Workload(name=name, d=d, N=N, T=1.0, sigma=[[0.5 if a == b else 0.0 for b in range(d)]
                                                         for a in range(d)],
                      b0=[0.0] * d, b1=[-0.1] * d, set_kind=set_kind, level=level, M=M, driver=driver,
                      f_a=f_a, sol_A=1.0, sol_c=1.0, sol_p=0.0,
                      sol_w=[1.0 if l < 2 else 0.0 for l in range(d)], seed=seed)


CASES = [
    # d = 2 tensor (two Brownian components), three time indices
    ("d2-tensor4", W.D2_TENSOR4, 9, None),
    ("d2-tensor4", W.D2_TENSOR4, 4, None),
    ("d2-tensor4", W.D2_TENSOR4, 0, None),
    # gradient driver: z of the expansion enters f, the Z rows are separate
    ("d3-zrat", _diag_workload("z-d3-zrat", 3, 5, "hc_1p", 12, 3000, "zrat", f_a=-0.05), 1, None),
    # nbm = 10: two chunks of responses (8 + 2)
    ("d10-hc1p", _diag_workload("z-d10", 10, 4, "hc_1p", 10, 2000, "allen_cahn"), 2, None),
    # ragged clouds: a single path and one past a wave
    ("d3-M1", _diag_workload("z-d3", 3, 4, "hc_max", 8, 1, "sin", f_a=0.5), 1, 1),
    ("d3-M257", _diag_workload("z-d3", 3, 4, "hc_max", 8, 257, "sin", f_a=0.5), 0, 257),
]


@pytest.mark.parametrize("scheme", ["multistep", "onestep"])
@pytest.mark.parametrize("name,w,i,M", CASES, ids=[f"{c[0]}-i{c[2]}" for c in CASES])
def test_backward_step_z_against_oracle(env, name, w, i, M, scheme):
    Q, ctx, torch = env
    M = w.M if M is None else M
    say(f"backward_step_z {scheme} {name} i={i} M={M}")
    b = Q.Basis(w.d, w.set_kind, w.level)
    reps = O.reps_for(w)
    alpha = W.synthetic_alpha(b.n_funcs, w.N, seed=w.d + i, scale=0.2, decay=0.7)
    a = dev(torch, alpha)
    az = torch.full((w.N, w.nbm, b.n_funcs), 7.0, dtype=torch.float64, device="cuda")
    ctx.backward_step_z(Q.problem_from(w), b, i, M, w.seed, a, az, scheme=scheme)
    torch.cuda.synchronize()
    ref_y, ab_y, _, _ = O.backward_step(w, reps, i, M, w.seed, alpha.copy())
    assert_alpha(host(a)[i], ref_y, ab_y, what=f"{name} Y row {i}")
    zref = O.backward_step_z if scheme == "multistep" else O.backward_step_z1
    ref_z, ab_z = zref(w, reps, i, M, w.seed, alpha)
    got = host(az)
    for k in range(w.nbm):
        assert_alpha(got[i, k], ref_z[k], ab_z[k], what=f"{name} Z row {i} component {k}")
    others = [r for r in range(w.N) if r != i]
    assert bool((got[others] == 7.0).all())


def test_backward_step_z_y_row_equals_backward_step(env):
    """The Y row of the Z step is the plain step's, bit for bit."""
    Q, ctx, torch = env
    w = W.D2_TENSOR4
    b = Q.Basis(w.d, w.set_kind, w.level)
    p = Q.problem_from(w)
    alpha = W.synthetic_alpha(b.n_funcs, w.N, seed=5, scale=0.2)
    a1, a2 = dev(torch, alpha), dev(torch, alpha)
    az = torch.zeros((w.N, w.nbm, b.n_funcs), dtype=torch.float64, device="cuda")
    for i in (w.N - 1, 3):
        ctx.backward_step(p, b, i, w.M, w.seed, a1)
        ctx.backward_step_z(p, b, i, w.M, w.seed, a2, az)
    torch.cuda.synchronize()
    assert torch.equal(a1, a2)


@pytest.mark.parametrize("scheme", ["multistep", "onestep"])
def test_solve_z_equals_solve_and_its_steps(env, scheme):
    Q, ctx, torch = env
    w = _diag_workload("z-d4", 4, 6, "hc_1p", 12, 5000, "allen_cahn")
    say(f"solve_z {w.name}")
    b = Q.Basis(w.d, w.set_kind, w.level)
    p = Q.problem_from(w)
    ref = torch.zeros((w.N, b.n_funcs), dtype=torch.float64, device="cuda")
    ctx.solve(p, b, w.M, w.seed, ref)
    a = torch.zeros_like(ref)
    az = torch.zeros((w.N, w.nbm, b.n_funcs), dtype=torch.float64, device="cuda")
    ctx.solve_z(p, b, w.M, w.seed, a, az, scheme=scheme)
    torch.cuda.synchronize()
    assert torch.equal(a, ref)
    s = torch.zeros_like(ref)
    sz = torch.zeros_like(az)
    for i in range(w.N - 1, -1, -1):
        ctx.backward_step_z(p, b, i, w.M, w.seed, s, sz, scheme=scheme)
    torch.cuda.synchronize()
    assert torch.equal(s, ref) and torch.equal(sz, az)
    # one slice against the oracle, from the solve's own rows
    reps = O.reps_for(w)
    ah = host(ref)
    zref = O.backward_step_z if scheme == "multistep" else O.backward_step_z1
    ref_z, ab_z = zref(w, reps, 2, w.M, w.seed, ah)
    for k in range(w.nbm):
        assert_alpha(host(az)[2, k], ref_z[k], ab_z[k], what=f"solve_z slice 2 component {k}")


def test_z_argument_checks(env):
    Q, ctx, torch = env
    w = W.D2_TENSOR4
    b = Q.Basis(w.d, w.set_kind, w.level)
    p = Q.problem_from(w)
    a = torch.zeros((w.N, b.n_funcs), dtype=torch.float64, device="cuda")
    az = torch.zeros((w.N, w.nbm, b.n_funcs), dtype=torch.float64, device="cuda")
    with pytest.raises(Q.QrError):
        ctx.backward_step_z(p, b, w.N, w.M, w.seed, a, az)
    with pytest.raises(Q.QrError):
        ctx.backward_step_z(p, b, 0, w.M, w.seed, a, None)
    with pytest.raises(Q.QrError) as e:
        ctx.backward_step_z(p, b, 0, w.M, w.seed, a, az, scheme=2)
    assert e.value.status == -1
    pq = Q.problem_from(w.with_(damping_q=2.0))
    with pytest.raises(Q.QrError) as e:
        ctx.backward_step_z(pq, b, 0, w.M, w.seed, a, az)
    assert e.value.status == -6
    wc = W.paper_benchmark(2, 4, "total", 5, 1000)
    bc = Q.Basis(wc.d, wc.set_kind, wc.level, law=wc.law, basis=wc.basis)
    ac = torch.zeros((wc.N, bc.n_funcs), dtype=torch.float64, device="cuda")
    azc = torch.zeros((wc.N, wc.nbm, bc.n_funcs), dtype=torch.float64, device="cuda")
    with pytest.raises(Q.QrError) as e:
        ctx.solve_z(Q.problem_from(wc), bc, wc.M, wc.seed, ac, azc)
    assert e.value.status == -6
    torch.cuda.synchronize()
    assert bool((az == 0).all())


def _z_exact(w, t, x):
    """sigma^T grad u of u = B + A exp(-c (T-t)) cos(w.x + p), points [n][d]."""
    e = np.exp(-w.sol_c * (w.T - t))
    ww = np.asarray(w.sol_w, dtype=np.float64)
    gu = -w.sol_A * e * np.sin(x @ ww + w.sol_p)[:, None] * ww[None, :]
    return gu @ np.asarray(w.sigma, dtype=np.float64)


def test_z_estimate_converges_to_the_projection_of_sigma_grad_u(env):
    """With the exact solution's gradient known, the Z coefficients of both
    schemes approach the coefficients of sigma^T grad u(t_i, .) (the
    basis is orthonormal under the sampling law, so these are E[Z phi_k]),
    up to the Monte-Carlo error, which shrinks with M, and a bias that does
    not: the regression targets sigma^T grad of E[g + the later terms | X_i],
    which differs from sigma^T grad u(t_i) by O(Delta) (the first term is left
    out), and from i < N-1 on the responses carry the error of the Y rows
    they read.  With Delta = 0.1 the bound at M = 2^21 is 2.5 Delta."""
    Q, ctx, torch = env
    w = W.D2_TENSOR4
    b = Q.Basis(w.d, w.set_kind, w.level)
    reps = O.reps_for(w)
    p = Q.problem_from(w)
    n = 1 << 18
    errs = {}
    wants = {}
    for i in (w.N - 1, 0):
        x = O.sample_points(w.d, 1234, 2, 0, n)
        zt = _z_exact(w, i * w.T / w.N, x)
        wants[i] = np.stack([O.project(reps, x, zt[:, k]) for k in range(w.nbm)])
    for scheme in ("multistep", "onestep"):
        for M in (1 << 14, 1 << 21):
            a = torch.zeros((w.N, b.n_funcs), dtype=torch.float64, device="cuda")
            az = torch.zeros((w.N, w.nbm, b.n_funcs), dtype=torch.float64, device="cuda")
            ctx.solve_z(p, b, M, w.seed, a, az, scheme=scheme)
            torch.cuda.synchronize()
            got = host(az)
            for i in (w.N - 1, 0):
                errs[(scheme, M, i)] = float(np.linalg.norm(got[i] - wants[i]) / np.linalg.norm(wants[i]))
    say(f"Z coefficient errors {errs}")
    for scheme in ("multistep", "onestep"):
        for i in (w.N - 1, 0):
            assert errs[(scheme, 1 << 21, i)] < errs[(scheme, 1 << 14, i)]
    for i in (w.N - 1, 0):
        assert errs[("multistep", 1 << 21, i)] < 2.5 * (w.T / w.N), errs
    # the one-step responses have far less variance: at the small cloud the
    # one-step estimate is the closer one
    for i in (w.N - 1, 0):
        assert errs[("onestep", 1 << 14, i)] < errs[("multistep", 1 << 14, i)], errs
    # but they read ybar_{i+1}, not the path: at i = N-1 that is g itself and
    # the bound above holds; at i = 0 the estimate keeps the error of the
    # expansion ybar_1, whose basis reproduces u(t_1) only to a relative 0.40
    # (its projection floor), so the bound there is that floor
    assert errs[("onestep", 1 << 21, w.N - 1)] < 2.5 * (w.T / w.N), errs
    assert errs[("onestep", 1 << 21, 0)] < 0.40, errs
