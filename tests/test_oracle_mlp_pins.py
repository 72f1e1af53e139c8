"""Pins of the FP64 network definition (oracle/mlp.py), independent of it:
central finite differences of the loss, closed forms of silu, and the Adam
step on a case with a known answer."""
import numpy as np
import pytest

from oracle import mlp


def _theta(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(mlp.NPARAMS) * scale / np.sqrt(16)


def test_parameter_count():
    assert mlp.NPARAMS == 256 * 16 + 256 + 256 * 256 + 256 + 256 + 1 == 70401


def test_silu_closed_forms():
    z = np.array([-30.0, -2.0, 0.0, 1.5, 30.0])
    assert mlp.silu(np.array([0.0]))[0] == 0.0
    assert abs(mlp.silu_prime(np.array([0.0]))[0] - 0.5) < 1e-15
    assert np.allclose(mlp.silu(z)[-1], 30.0, rtol=1e-12) and abs(mlp.silu(z)[0]) < 1e-11
    # derivative by central differences
    h = 1e-6
    fd = (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h)
    assert np.allclose(mlp.silu_prime(z), fd, rtol=1e-7, atol=1e-9)


def test_features():
    x = np.array([[0.0, 100.0, -100.0]])
    f = mlp.features(x)
    assert f.shape == (1, 16)
    assert abs(f[0, 0]) < 1e-15 and abs(f[0, 1] - 1.0) < 1e-15 and abs(f[0, 2] + 1.0) < 1e-15
    assert not f[0, 3:].any()


def test_gradient_by_central_differences():
    rng = np.random.default_rng(0)
    theta = _theta(1)
    f = rng.uniform(-1, 1, size=(32, 16))
    t = rng.standard_normal(32)
    _, g = mlp.loss_grad(theta, f, t)
    offsets = np.cumsum([0] + [int(np.prod(s)) for _, s in mlp.SIZES])
    # a few entries of every parameter block
    idx = np.concatenate([rng.integers(offsets[b], offsets[b + 1], 4) for b in range(len(mlp.SIZES))])
    h = 1e-6
    for k in idx:
        e = np.zeros_like(theta)
        e[k] = h
        fd = (mlp.loss_grad(theta + e, f, t)[0] - mlp.loss_grad(theta - e, f, t)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_forward_reduces_to_a_linear_model():
    """With W2 = 0 and b2 = large, h2 = b2 (silu(z) -> z), so y = w3 . b2 + b3."""
    p = mlp.unpack(_theta(2))
    p["W2"][:] = 0.0
    p["b2"][:] = 40.0
    th = mlp.pack(p)
    y, _ = mlp.forward(th, np.random.default_rng(3).uniform(-1, 1, (5, 16)))
    assert np.allclose(y, 40.0 * p["w3"].sum() * (1 - 0) + p["b3"][0], rtol=1e-12)


def test_adam_first_step_is_sign_times_lr():
    """The bias-corrected first Adam step moves every parameter by lr sign(g)
    (up to eps)."""
    g = np.array([3.0, -0.5, 1e-3])
    th, m, v = mlp.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(th, -0.01 * np.sign(g), rtol=1e-4)


def test_bf16_rounding_values():
    """bfloat16 keeps 8 significant bits; ties go to the even neighbour."""
    one = 1.0
    assert mlp.bf16(one + 2.0 ** -8) == one                      # tie -> even (1.0)
    assert mlp.bf16(one + 3 * 2.0 ** -8) == one + 2.0 ** -6      # tie -> even (1 + 2^-6)
    assert mlp.bf16(one + 2.0 ** -8 + 2.0 ** -12) == one + 2.0 ** -7
    assert mlp.bf16(-3.0) == -3.0 and mlp.bf16(0.0) == 0.0
    x = np.random.default_rng(4).standard_normal(1000)
    r = mlp.bf16(x)
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x))


def test_bf16_network_tends_to_the_exact_one():
    """The bfloat16-operand network differs from the exact one by O(2^-8)."""
    rng = np.random.default_rng(5)
    th = _theta(6)
    f = rng.uniform(-1, 1, (64, 16))
    y, _ = mlp.forward(th, f)
    yb, _ = mlp.forward_bf16(th, f)
    assert np.linalg.norm(yb - y) <= 2e-2 * np.linalg.norm(y)
    assert np.linalg.norm(yb - y) > 0


# ---------------------------------------------------------------------------
# the oracle's learned step (oracle/qrmc_oracle.c: or_mlp_forward,
# or_backward_step_learned)
# ---------------------------------------------------------------------------

def test_c_network_equals_the_numpy_definition():
    """The C oracle's network (bfloat16 operands, exact sums) equals the numpy
    definition with the same rounding points, at states x of d <= 16
    coordinates (features 2 F(x_l) - 1, zero-padded), and is O(2^-8) from the
    exact network."""
    import oracle as O
    rng = np.random.default_rng(8)
    th = _theta(9)
    for d in (1, 3, 16):
        x = rng.standard_normal((40, d)) * 2.0
        got = O.mlp_forward(th, x)
        ref, _ = mlp.forward_bf16(th, mlp.features(x))
        exact, _ = mlp.forward(th, mlp.features(x))
        assert np.allclose(got, ref, rtol=1e-13, atol=1e-15)
        assert np.linalg.norm(got - exact) <= 2e-2 * np.linalg.norm(exact)


def test_learned_step_with_a_constant_network_is_a_constant_expansion():
    """A network with zero weights outputs b3, so y_j = mu_j + sd_j b3 at
    every point: the learned step must equal the plain step whose row j is
    the constant mu_j + sd_j b3 (alpha_0 alone).  Without networks it is the
    plain step itself."""
    import oracle as O
    import workloads as W
    w = W.D2_TENSOR4.with_(M=600, N=4)
    reps = O.reps_for(w)
    nf = O.nfuncs(reps)
    alpha = W.synthetic_alpha(nf, w.N, seed=3, scale=0.2, decay=0.7)
    const = mlp.unpack(np.zeros(mlp.NPARAMS))
    const["b3"][0] = 0.35
    net = mlp.pack(const)
    mu, sd = [0.0, 0.0, -0.2, 0.0], [1.0, 1.0, 1.5, 1.0]
    for i in (1, 0):
        plain, _ = O.backward_step_learned(w, reps, i, w.M, w.seed, alpha.copy(), [None] * w.N, mu, sd)
        ref, _, _, _ = O.backward_step(w, reps, i, w.M, w.seed, alpha.copy())
        assert np.array_equal(plain, ref)
        nets = [None, None, net, None]
        got, _ = O.backward_step_learned(w, reps, i, w.M, w.seed, alpha.copy(), nets, mu, sd)
        a2 = alpha.copy()
        a2[2] = 0.0
        a2[2, 0] = -0.2 + 1.5 * 0.35
        want, _, _, _ = O.backward_step(w, reps, i, w.M, w.seed, a2)
        assert np.allclose(got, want, rtol=1e-14, atol=1e-15)
        assert not np.allclose(got, ref, rtol=1e-6)
