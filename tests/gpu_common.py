"""Shared pieces of the GPU parity tests: the context fixture, host/device
copies, progress output and the FP64 coefficient comparison.

Parity tolerance for FP64 results (relative 1e-10): the GPU and the oracle
sum in different orders and alpha_k can be much smaller than the terms it
sums, so each coefficient is compared against max(|alpha_k|, A_k) with
A_k = (1/M) sum |S phi_k| (the cancellation bound), and the row in the 2-norm.
"""
import sys

import numpy as np
import pytest

TOL = 1e-10


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2407_21084_amd import qrmc as Q
    ctx = Q.Context(0)
    yield Q, ctx, torch
    ctx.close()


def dev(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_err(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def assert_alpha(gpu, ref, absum, tol=TOL, what=""):
    scale = np.maximum(np.abs(ref), absum)
    bad = np.abs(gpu - ref) > tol * scale + 1e-300
    assert not bad.any(), f"{what}: {bad.sum()} coefficients off, worst {np.max(np.abs(gpu - ref) / (scale + 1e-300))}"
    assert np.linalg.norm(gpu - ref) <= tol * np.linalg.norm(ref) + 1e-300, what
