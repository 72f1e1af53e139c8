"""Plain FP64 definition of the surrogate network of the learned form.

TEST INFRASTRUCTURE ONLY (like the rest of this package): imported by tests/,
never by the product package.  The network is not part of the paper's
method; this module is its textbook definition, written out so that the HIP
forward, backward and Adam kernels can be compared with it.

Network: features f in R^16 -> z1 = W1 f + b1 -> h1 = silu(z1) (256) ->
z2 = W2 h1 + b2 -> h2 = silu(z2) (256) -> y = w3 . h2 + b3, with
silu(z) = z / (1 + exp(-z)).  Loss: mean squared error over a batch.
Parameters are one flat vector, in this order: W1 [256][16] (row = output
unit), b1 [256], W2 [256][256], b2 [256], w3 [256], b3 [1].
Features of a state x in R^d: 2 F(x_l) - 1 for l < d (F the standard logistic
CDF), 0 for d <= l < 16.
"""
from __future__ import annotations

import numpy as np

IN, HID = 16, 256
SIZES = [("W1", (HID, IN)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)), ("w3", (HID,)),
         ("b3", (1,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def pack(parts) -> np.ndarray:
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).ravel() for name, _ in SIZES])


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * sigmoid(z)


def silu_prime(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def features(x) -> np.ndarray:
    """x: [n][d] states -> [n][16] features."""
    x = np.asarray(x, dtype=np.float64)
    f = np.zeros((x.shape[0], IN))
    f[:, :x.shape[1]] = 2.0 / (1.0 + np.exp(-x)) - 1.0
    return f


def forward(theta, f):
    p = unpack(theta)
    z1 = f @ p["W1"].T + p["b1"]
    h1 = silu(z1)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = silu(z2)
    y = h2 @ p["w3"] + p["b3"][0]
    return y, (z1, h1, z2, h2)


def loss_grad(theta, f, t):
    """(mean squared error, gradient) by backpropagation."""
    p = unpack(theta)
    y, (z1, h1, z2, h2) = forward(theta, f)
    n = f.shape[0]
    r = y - t
    loss = float(np.mean(r * r))
    dy = 2.0 * r / n
    g = {"w3": h2.T @ dy, "b3": np.array([dy.sum()])}
    dz2 = np.outer(dy, p["w3"]) * silu_prime(z2)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ p["W2"]) * silu_prime(z1)
    g["W1"] = dz1.T @ f
    g["b1"] = dz1.sum(axis=0)
    return loss, pack(g)


def adam(theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba), bias-corrected; returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------------------
# The network as computed with bfloat16 operands (products of bfloat16
# numbers summed exactly, i.e. in FP64 here): the reference for kernels that
# round the operands of every matrix product to bfloat16.
# ---------------------------------------------------------------------------
def bf16(a):
    """Round to the nearest bfloat16 (8 significant bits, ties to even),
    through float32 as the kernels do; finite inputs."""
    f = np.asarray(a, dtype=np.float64).astype(np.float32).view(np.uint32).astype(np.uint64)
    f = ((f + 0x7FFF + ((f >> 16) & 1)) >> 16) << 16
    return f.astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16(theta, f):
    p = unpack(theta)
    z1 = bf16(f) @ bf16(p["W1"]).T + p["b1"]
    h1 = silu(z1)
    z2 = bf16(h1) @ bf16(p["W2"]).T + p["b2"]
    h2 = silu(z2)
    y = h2 @ p["w3"] + p["b3"][0]
    return y, (z1, h1, z2, h2)


def loss_grad_bf16(theta, f, t):
    p = unpack(theta)
    y, (z1, h1, z2, h2) = forward_bf16(theta, f)
    n = f.shape[0]
    r = y - t
    loss = float(np.mean(r * r))
    dy = 2.0 * r / n
    g = {"w3": h2.T @ dy, "b3": np.array([dy.sum()])}
    dz2 = np.outer(dy, p["w3"]) * silu_prime(z2)
    g["W2"] = bf16(dz2).T @ bf16(h1)
    g["b2"] = dz2.sum(axis=0)
    dz1 = (bf16(dz2) @ bf16(p["W2"])) * silu_prime(z1)
    g["W1"] = bf16(dz1).T @ bf16(f)
    g["b1"] = dz1.sum(axis=0)
    return loss, pack(g)
