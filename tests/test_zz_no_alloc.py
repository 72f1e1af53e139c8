"""qr_eval_noalloc: the evaluation for callers that cannot allocate.

It runs qr_eval's kernels on a coefficient row staged in a fixed device array
instead of context workspace, so its outputs must equal qr_eval's bit for bit
(the stricter form of the FP64 parity bar).  Two calls in a row, the second
with a smaller basis and fewer points, check that what the first call leaves
in the shared array does not leak into the second.  The argument checks
(basis not resident, basis larger than the array) run without a launch.
"""
import numpy as np
import pytest

import workloads as W
from gpu_common import dev, env, say  # noqa: F401  (env is a fixture)

pytestmark = pytest.mark.gpu


def _eval_both(Q, ctx, torch, basis, alpha_row, x, grad):
    n = x.shape[1]
    y_ref = torch.empty(n, dtype=torch.float64, device="cuda")
    y_new = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    g_ref = torch.empty((basis.d, n), dtype=torch.float64, device="cuda") if grad else None
    g_new = torch.full((basis.d, n), float("nan"), dtype=torch.float64, device="cuda") if grad else None
    ctx.eval(basis, alpha_row, x, y_ref, g_ref)
    ctx.eval_noalloc(basis, alpha_row, x, y_new, g_new)
    torch.cuda.synchronize()
    assert torch.isfinite(y_new).all()
    assert torch.equal(y_new, y_ref)
    if grad:
        assert torch.equal(g_new, g_ref)


def test_noalloc_matches_eval_twice(env):
    Q, ctx, torch = env
    say("eval_noalloc: d=6 hc_max 16 (84,605 representatives), then d=2 tensor 4")
    big = Q.Basis(6, "hc_max", 16)
    small = Q.Basis(2, "tensor", 4)
    ctx.basis_upload(big)
    ctx.basis_upload(small)
    a_big = dev(torch, W.synthetic_alpha(big.n_funcs, 1, seed=41, scale=0.1, decay=0.8)[0])
    a_small = dev(torch, W.synthetic_alpha(small.n_funcs, 1, seed=43, scale=0.3, decay=0.7)[0])
    x_big = dev(torch, W.logistic_points(5000, 6, seed=45).T)
    x_small = dev(torch, W.logistic_points(301, 2, seed=47).T)
    _eval_both(Q, ctx, torch, big, a_big, x_big, grad=True)
    _eval_both(Q, ctx, torch, small, a_small, x_small, grad=False)
    # and back: the larger basis after the smaller one
    _eval_both(Q, ctx, torch, big, a_big, x_big[:, :777].contiguous(), grad=False)


def test_noalloc_argument_checks(env):
    Q, ctx, torch = env
    fresh = Q.Basis(3, "hc_max", 7)      # never used on the device
    a = torch.zeros(fresh.n_funcs, dtype=torch.float64, device="cuda")
    x = torch.zeros((3, 8), dtype=torch.float64, device="cuda")
    y = torch.empty(8, dtype=torch.float64, device="cuda")
    with pytest.raises(Q.QrError) as e:
        ctx.eval_noalloc(fresh, a, x, y)
    assert e.value.status == -1 and "qr_basis_upload" in str(e.value)
    huge = Q.Basis(6, "hc_max", 64)      # 854,929 representatives
    assert (huge.n_funcs + 1) // 2 > 524160
    with pytest.raises(Q.QrError) as e:
        ctx.eval_noalloc(huge, a, x, y)
    assert e.value.status == -4
    ctx.basis_upload(fresh)
    y0 = torch.empty(0, dtype=torch.float64, device="cuda")
    ctx.eval_noalloc(fresh, a, x[:, :0], y0)          # n = 0 is a no-op
    np.testing.assert_equal(y0.cpu().numpy().size, 0)
