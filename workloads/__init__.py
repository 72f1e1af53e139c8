"""Workload descriptors and seeded synthetic inputs shared by tests and the benchmark.

This module holds *no* arithmetic of the method: only problem parameters (as
plain numbers) and seeded numpy generators for synthetic inputs (coefficient
tables, point clouds, responses).  Both the GPU library's tests and the CPU
oracle consume what it produces; neither side's arithmetic lives here.

The problem family is the one of the paper's Sec. 1 (decoupled FBSDE /
semi-linear PDE) solved with Algorithm 1 (GQRMDP):

* state dimension ``d`` with ``nbm`` Brownian dimensions, uniform grid
  ``t_j = j T / N`` (Sec. 2.1.1 uses N equidistant steps);
* drift ``b(t,x)_l = b0_l + b1_l x_l``, constant diffusion ``sigma`` (d x nbm);
* sampling law nu: product of identical one-dimensional laws, ``logistic``
  (standard logistic, the default), ``student2`` (Student's t with mu = 2 in
  the paper's scaling, density 0.5 (1+x^2)^{-3/2}) or ``cauchy``;
* index set over Z^d: ``tensor`` (max |k_l| <= level), ``hc_max``
  (prod max(1,|k_l|) <= level) or ``hc_1p`` (prod (1+|k_l|) <= level);
* driver ``f = f_nl(y, z) + h(t, x)`` where h makes the manufactured
  solution ``u(t,x) = A exp(-c (T-t)) cos(w.x + p)`` exact.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np

SET_KINDS = {"tensor": 0, "hc_max": 1, "hc_1p": 2, "total": 3}
DRIVERS = {"linear": 0, "sin": 1, "allen_cahn": 2, "zrat": 3, "paper": 4}
BASES = {"fourier": 0, "cosine": 1}
LAWS = {"logistic": 0, "student2": 1, "cauchy": 2}


@dataclass(frozen=True)
class Workload:
    name: str
    d: int
    N: int
    T: float
    sigma: List[List[float]]          # d x nbm
    b0: List[float]
    b1: List[float]
    set_kind: str
    level: int
    M: int
    driver: str
    f_a: float
    sol_A: float
    sol_c: float
    sol_p: float
    sol_w: List[float]
    clamp: float = math.inf
    seed: int = 0
    law: str = "logistic"
    damping_q: float = 0.0
    basis: str = "fourier"      # "cosine": the paper's cosine basis over N^d
    sol_B: float = 0.0          # constant offset of the manufactured solution
    b2: Optional[List[float]] = None       # bounded drift part b2_l sin(x_l) (None: 0)
    sigma_v: Optional[List[float]] = None  # sigma(t,x) row scale 1 + v_l cos(x_l + omega t)
    sigma_omega: float = 0.0
    notes: str = ""

    @property
    def nbm(self) -> int:
        return len(self.sigma[0])

    @property
    def times(self) -> List[float]:
        return [self.T * j / self.N for j in range(self.N + 1)]

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


def _diag(d: int, s: float) -> List[List[float]]:
    return [[s if a == b else 0.0 for b in range(d)] for a in range(d)]


def _first_two(d: int) -> List[float]:
    return [1.0 if l < 2 else 0.0 for l in range(d)]


# d=2, tensor |k_l|<=4 (81 functions), M=10^4, f = 0.5 sin y + h,
# u = exp(-(T-t)) cos(x1+x2), dX = 0.5 dW.
D2_TENSOR4 = Workload(
    name="d2-tensor4-sin", d=2, N=10, T=1.0, sigma=_diag(2, 0.5), b0=[0.0] * 2, b1=[0.0] * 2,
    set_kind="tensor", level=4, M=10_000, driver="sin", f_a=0.5,
    sol_A=1.0, sol_c=1.0, sol_p=0.0, sol_w=[1.0, 1.0])

# d=6, N=20, sigma=0.4 I, b=-0.1 x, hyperbolic cross prod max(1,|k_l|)<=16
# (169,209 functions), M=2^20, Allen-Cahn driver y - y^3 + h,
# u = exp(-(T-t)) cos(sum x)/2; T=1 and clamp L = 2 sup|u| = 1 are readings.
D6_HCMAX16 = Workload(
    name="d6-hcmax16-allen-cahn", d=6, N=20, T=1.0, sigma=_diag(6, 0.4), b0=[0.0] * 6,
    b1=[-0.1] * 6, set_kind="hc_max", level=16, M=1 << 20, driver="allen_cahn", f_a=0.0,
    sol_A=0.5, sol_c=1.0, sol_p=0.0, sol_w=[1.0] * 6, clamp=1.0)

# d=10, N=30, prod (1+|k_l|)<=32 (85,485 functions; the literal max(1,.) set
# has 1.8e8), M=2^22, f = -0.05|z|^2/(1+|z|^2) + y/(1+y^2) + h,
# u = exp(-(T-t)) cos(x1+x2); sigma = 0.5 I, b = 0, T = 1 are readings.
D10_HC1P32_ZRAT = Workload(
    name="d10-hc1p32-zrat", d=10, N=30, T=1.0, sigma=_diag(10, 0.5), b0=[0.0] * 10,
    b1=[0.0] * 10, set_kind="hc_1p", level=32, M=1 << 22, driver="zrat", f_a=-0.05,
    sol_A=1.0, sol_c=1.0, sol_p=0.0, sol_w=_first_two(10))

# d=16, N=40, prod (1+|k_l|)<=32 (599,969 functions), M=2^22, Allen-Cahn
# driver, u = exp(-(T-t)) cos(x1+x2), clamp L = 2.
D16_HC1P32 = Workload(
    name="d16-hc1p32-allen-cahn", d=16, N=40, T=1.0, sigma=_diag(16, 0.5), b0=[0.0] * 16,
    b1=[0.0] * 16, set_kind="hc_1p", level=32, M=1 << 22, driver="allen_cahn", f_a=0.0,
    sol_A=1.0, sol_c=1.0, sol_p=0.0, sol_w=_first_two(16), clamp=2.0)

# The benchmark of the paper's Sec. 5 (eq (pde2OnlyY)), d = 1: dX = dW,
# f = min(1, (y - u)^2), g = u(T, .) with u = 1 + kappa + sin(lambda x)
# e^{lambda^2 d (t-T)/2}, kappa = 0.6, lambda = 1/sqrt(d) = 1, T = 1, the
# Student (mu = 2) sampling law and the cosine basis of Gamma_F(K), K = 100
# (101 functions), Delta = 0.05 (N = 20), M = 2 10^4, q = 0: the first row of
# the paper's d = 1 accuracy table (u(0, 0) = 1.6).  sin(theta) is written as
# cos(theta - pi/2).
def paper_benchmark(d: int, N: int, set_kind: str, level: int, M: int, kappa: float = 0.6,
                    seed: int = 0) -> Workload:
    lam = 1.0 / math.sqrt(d)
    return Workload(
        name=f"paper-d{d}-{set_kind}{level}", d=d, N=N, T=1.0, sigma=_diag(d, 1.0), b0=[0.0] * d,
        b1=[0.0] * d, set_kind=set_kind, level=level, M=M, driver="paper", f_a=0.0,
        sol_A=1.0, sol_c=0.5 * lam * lam * d, sol_p=-0.5 * math.pi, sol_w=[lam] * d, seed=seed,
        law="student2", basis="cosine", sol_B=1.0 + kappa)


PAPER_D1 = paper_benchmark(1, 20, "tensor", 100, 20_000)

# Rows of the paper's Tables d1_mse and d2_mse (Sec. 5): Delta = 1/N, the set
# and its level, M; the cosine basis over N^d and the Student mu = 2 law.
PAPER_TABLES = (
    PAPER_D1,
    paper_benchmark(1, 50, "tensor", 150, 200_000),
    paper_benchmark(1, 100, "tensor", 200, 2_000_000),
    paper_benchmark(2, 20, "total", 20, 20_000),
    paper_benchmark(2, 20, "hc_max", 19, 20_000),
    paper_benchmark(2, 50, "total", 25, 200_000),
    paper_benchmark(2, 50, "hc_max", 24, 200_000),
    paper_benchmark(2, 100, "total", 31, 2_000_000),
    paper_benchmark(2, 100, "hc_max", 30, 2_000_000),
)

# The d=6 workload with state-dependent coefficients: drift -0.1 x + 0.2
# sin(x_l) and diffusion 0.4 (1 + 0.5 cos(x_l + 2t)) per coordinate; the
# manufactured source keeps u = exp(-(T-t)) cos(sum x)/2 the solution.
D6_HCMAX16_SDEP = D6_HCMAX16.with_(name="d6-hcmax16-allen-cahn-sdep", b2=[0.2] * 6, sigma_v=[0.5] * 6,
                                   sigma_omega=2.0)

ALL = {w.name: w for w in (D2_TENSOR4, D6_HCMAX16, D6_HCMAX16_SDEP, D10_HC1P32_ZRAT, D16_HC1P32) + PAPER_TABLES}


def batched_instances(n: int = 256, seed: int = 4):
    """Instance parameters of the batched form: d ~ U{2..12},
    M in {2^14..2^20}, level in {8,16,32}, driver c_j sin y + h_j with
    c_j ~ U[0.2, 1]; sigma = 0.5 I, b = 0, N = 10, u = exp(-(T-t)) cos(x1+x2)."""
    rng = np.random.default_rng(seed)
    out = []
    for j in range(n):
        d = int(rng.integers(2, 13))
        M = 1 << int(rng.integers(14, 21))
        level = int(rng.choice([8, 16, 32]))
        c = float(rng.uniform(0.2, 1.0))
        out.append(Workload(
            name=f"inst{j}", d=d, N=10, T=1.0, sigma=_diag(d, 0.5), b0=[0.0] * d,
            b1=[0.0] * d, set_kind="hc_1p", level=level, M=M, driver="sin", f_a=c,
            sol_A=1.0, sol_c=1.0, sol_p=0.0, sol_w=_first_two(d)))
    return out


def batched_group(instances, max_batch: int = 64):
    """Split instances that share sigma = s I, b, N, T, the sampling law and a
    solution depending on x1, x2 only into groups of at most max_batch.  Each
    group is (group workload in the largest d of the group, level = largest
    level, M = largest M; list of (f_a, d, level, M) per instance; indices)."""
    out = []
    for g0 in range(0, len(instances), max_batch):
        grp = list(range(g0, min(len(instances), g0 + max_batch)))
        ws = [instances[k] for k in grp]
        d = max(w.d for w in ws)
        w0 = ws[0]
        s = w0.sigma[0][0]
        gw = w0.with_(name=f"group{g0 // max_batch}", d=d, sigma=_diag(d, s), b0=[0.0] * d,
                      b1=[0.0] * d, level=max(w.level for w in ws), M=max(w.M for w in ws),
                      sol_w=_first_two(d))
        out.append((gw, [(w.f_a, w.d, w.level, w.M) for w in ws], grp))
    return out


# ---------------------------------------------------------------------------
# seeded synthetic inputs
# ---------------------------------------------------------------------------

def synthetic_alpha(nfuncs: int, rows: int, seed: int, scale: float = 0.3,
                    decay: float = 0.5) -> np.ndarray:
    """A [rows][nfuncs] table of expansion coefficients with a decaying
    envelope (entry f scaled by (1+f)^-decay) so that expansions stay O(1)."""
    rng = np.random.default_rng(seed)
    env = scale * (1.0 + np.arange(nfuncs, dtype=np.float64)) ** (-decay)
    return rng.standard_normal((rows, nfuncs)) * env[None, :]


def logistic_points(n: int, d: int, seed: int) -> np.ndarray:
    """n points of the product standard logistic law, row-major [n][d]
    (numpy's own generator; independent of the method's Philox streams)."""
    rng = np.random.default_rng(seed)
    return rng.logistic(0.0, 1.0, size=(n, d))


def law_points(n: int, d: int, law: str, seed: int) -> np.ndarray:
    """n points of the product law ``law``, row-major [n][d] (numpy's own
    generators: logistic, Student's t with 2 degrees of freedom divided by
    sqrt 2, standard Cauchy; independent of the method's Philox streams)."""
    rng = np.random.default_rng(seed)
    if law == "logistic":
        return rng.logistic(0.0, 1.0, size=(n, d))
    if law == "student2":
        return rng.standard_t(2.0, size=(n, d)) / math.sqrt(2.0)
    if law == "cauchy":
        return rng.standard_cauchy(size=(n, d))
    raise ValueError(f"unknown law {law!r}")


def responses(n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n)
