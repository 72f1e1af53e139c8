"""ctypes wrapper of the plain FP64 CPU oracle (qrmc_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
CPU-baseline leg of bench.py; never by the product package.  It shares no code
with the HIP library.  The shared library is built by ``build()`` (also run by
the repository's build step) with gcc, OpenMP and strict IEEE semantics.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qrmc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MAXD = 16
MAXN = 256

SET_KINDS = {"tensor": 0, "hc_max": 1, "hc_1p": 2, "total": 3}
DRIVERS = {"linear": 0, "sin": 1, "allen_cahn": 2, "zrat": 3, "paper": 4}
BASES = {"fourier": 0, "cosine": 1}
LAWS = {"logistic": 0, "student2": 1, "cauchy": 2}


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-shared", "-fPIC", "-o", _LIB, _SRC, "-lm"])
    return _LIB


class Problem(C.Structure):
    _fields_ = [
        ("d", C.c_int32), ("nbm", C.c_int32), ("N", C.c_int32), ("driver", C.c_int32),
        ("nu", C.c_int32), ("f_a", C.c_double), ("clamp", C.c_double),
        ("t", C.c_double * (MAXN + 1)),
        ("b0", C.c_double * MAXD), ("b1", C.c_double * MAXD),
        ("sigma", C.c_double * (MAXD * MAXD)),
        ("sol_A", C.c_double), ("sol_c", C.c_double), ("sol_p", C.c_double),
        ("sol_w", C.c_double * MAXD),
        ("damping_q", C.c_double),
        ("sol_B", C.c_double), ("basis", C.c_int32),
        ("b2", C.c_double * MAXD), ("sigma_v", C.c_double * MAXD), ("sigma_omega", C.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        P, D, I32, I64, U64, U32 = (C.c_void_p, C.c_double, C.c_int32, C.c_int64,
                                    C.c_uint64, C.c_uint32)
        sig = {
            "or_philox4x32_10": (None, [P, P, P]),
            "or_uniform": (D, [U64, U32, U64, U32, U32]),
            "or_norm_icdf": (D, [D]),
            "or_logistic_cdf": (D, [D]),
            "or_logistic_icdf": (D, [D]),
            "or_law_cdf": (D, [C.c_int, D]),
            "or_law_icdf": (D, [C.c_int, D]),
            "or_law_pdf": (D, [C.c_int, D]),
            "or_enumerate": (I64, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, P, I64]),
            "or_basis_values": (None, [C.c_int, C.c_int, C.c_int, I64, P, P, P]),
            "or_eval": (None, [C.c_int, C.c_int, C.c_int, I64, P, P, I64, P, P, P]),
            "or_msol_u": (D, [P, D, P]),
            "or_msol_h": (D, [P, D, P]),
            "or_path_response": (D, [P, I64, P, I32, U64, U64, P]),
            "or_damping": (D, [P, P]),
            "or_eval_y": (D, [P, I64, P, P, P, P]),
            "or_project": (None, [C.c_int, C.c_int, C.c_int, I64, P, I64, P, P, P, P]),
            "or_backward_step": (C.c_int, [P, I64, P, I32, I64, U64, P, P, P, P]),
            "or_solve": (C.c_int, [P, I64, P, I64, U64, P]),
            "or_backward_step_learned": (C.c_int, [P, I64, P, I32, I64, U64, P, P, P, P, P]),
            "or_backward_step_z": (C.c_int, [P, I64, P, I32, I64, U64, P, P, P]),
            "or_backward_step_z1": (C.c_int, [P, I64, P, I32, I64, U64, P, P, P]),
            "or_mlp_forward": (D, [P, C.c_int, C.c_int, P]),
            "or_sample_points": (None, [C.c_int, C.c_int, U64, U32, I32, I64, I64, P]),
            "or_errors": (None, [P, I64, P, P, U64, I64, P]),
            "or_num_threads": (C.c_int, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(_lib, name)
            f.restype = res
            f.argtypes = args
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------------------
# random streams and laws
# ---------------------------------------------------------------------------

def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def uniform(seed, stream, m, i, r) -> float:
    return lib().or_uniform(seed, stream, m, i, r)


def norm_icdf(u: float) -> float:
    return lib().or_norm_icdf(u)


def logistic_cdf(x: float) -> float:
    return lib().or_logistic_cdf(x)


def logistic_icdf(u: float) -> float:
    return lib().or_logistic_icdf(u)


def law_cdf(law: str, x: float) -> float:
    return lib().or_law_cdf(LAWS[law], x)


def law_icdf(law: str, u: float) -> float:
    return lib().or_law_icdf(LAWS[law], u)


def law_pdf(law: str, x: float) -> float:
    return lib().or_law_pdf(LAWS[law], x)


# ---------------------------------------------------------------------------
# index sets and basis
# ---------------------------------------------------------------------------

def enumerate_set(d: int, kind: str, level: int, nonneg: bool = False,
                  reps_only: bool = True) -> np.ndarray:
    L = lib()
    n = L.or_enumerate(d, SET_KINDS[kind], level, int(nonneg), int(reps_only), None, 0)
    if n < 0:
        raise ValueError("invalid index set")
    out = np.zeros((n, d), dtype=np.int32)
    L.or_enumerate(d, SET_KINDS[kind], level, int(nonneg), int(reps_only), _ptr(out), n)
    return out


def count_set(d: int, kind: str, level: int, nonneg: bool = False) -> int:
    return int(lib().or_enumerate(d, SET_KINDS[kind], level, int(nonneg), 0, None, 0))


def nfuncs(reps: np.ndarray, basis: str = "fourier") -> int:
    """Real basis functions of a set: 2 R - 1 for the Fourier basis over the
    R representatives, one per vector for the cosine basis over N^d."""
    return reps.shape[0] if basis == "cosine" else 2 * reps.shape[0] - 1


def basis_values(reps: np.ndarray, x, law: str = "logistic", basis: str = "fourier") -> np.ndarray:
    x = _f64(x)
    reps = np.ascontiguousarray(reps, dtype=np.int32)
    phi = np.zeros(nfuncs(reps, basis))
    lib().or_basis_values(reps.shape[1], LAWS[law], BASES[basis], reps.shape[0], _ptr(reps), _ptr(x), _ptr(phi))
    return phi


def evaluate(reps: np.ndarray, alpha_row, x, grad: bool = False, law: str = "logistic", basis: str = "fourier"):
    reps = np.ascontiguousarray(reps, dtype=np.int32)
    x = _f64(x)
    n, d = x.shape
    y = np.zeros(n)
    g = np.zeros((n, d)) if grad else None
    lib().or_eval(d, LAWS[law], BASES[basis], reps.shape[0], _ptr(reps), _ptr(_f64(alpha_row)), n, _ptr(x),
                  _ptr(y), _ptr(g) if grad else None)
    return (y, g) if grad else y


def project(reps: np.ndarray, x, s, with_abs: bool = False, law: str = "logistic", basis: str = "fourier"):
    reps = np.ascontiguousarray(reps, dtype=np.int32)
    x = _f64(x)
    s = _f64(s)
    n, d = x.shape
    a = np.zeros(nfuncs(reps, basis))
    ab = np.zeros(nfuncs(reps, basis))
    lib().or_project(d, LAWS[law], BASES[basis], reps.shape[0], _ptr(reps), n, _ptr(x), _ptr(s), _ptr(a),
                     _ptr(ab))
    return (a, ab) if with_abs else a


# ---------------------------------------------------------------------------
# problems and Algorithm 1
# ---------------------------------------------------------------------------

def problem(w) -> Problem:
    """Build the oracle's problem struct from a workloads.Workload."""
    p = Problem()
    p.d, p.nbm, p.N = w.d, w.nbm, w.N
    p.driver = DRIVERS[w.driver]
    p.nu = LAWS[w.law]
    p.f_a = w.f_a
    p.clamp = w.clamp
    for j, t in enumerate(w.times):
        p.t[j] = t
    for l in range(w.d):
        p.b0[l] = w.b0[l]
        p.b1[l] = w.b1[l]
        p.sol_w[l] = w.sol_w[l]
        for k in range(w.nbm):
            p.sigma[l * w.nbm + k] = w.sigma[l][k]
    p.sol_A, p.sol_c, p.sol_p = w.sol_A, w.sol_c, w.sol_p
    p.damping_q = w.damping_q
    p.sol_B = w.sol_B
    p.basis = BASES[w.basis]
    for l in range(w.d):
        p.b2[l] = 0.0 if w.b2 is None else w.b2[l]
        p.sigma_v[l] = 0.0 if w.sigma_v is None else w.sigma_v[l]
    p.sigma_omega = w.sigma_omega
    return p


def reps_for(w) -> np.ndarray:
    """The workload's index set: representatives over Z^d for the Fourier
    basis, every vector of the set over N^d for the cosine basis."""
    if w.basis == "cosine":
        return enumerate_set(w.d, w.set_kind, w.level, nonneg=True, reps_only=False)
    return enumerate_set(w.d, w.set_kind, w.level)


def msol_u(w, t, x) -> np.ndarray:
    p = problem(w)
    x = np.atleast_2d(_f64(x))
    return np.array([lib().or_msol_u(C.byref(p), t, _ptr(np.ascontiguousarray(r))) for r in x])


def msol_h(w, t, x) -> np.ndarray:
    p = problem(w)
    x = np.atleast_2d(_f64(x))
    return np.array([lib().or_msol_h(C.byref(p), t, _ptr(np.ascontiguousarray(r))) for r in x])


def backward_step(w, reps, i, M, seed, alpha, want_x=False, want_s=False):
    """Fill alpha[i] (in place, alpha is [N][nf]) and return
    (alpha_row, abs_row, x or None, s or None)."""
    p = problem(w)
    reps = np.ascontiguousarray(reps, dtype=np.int32)
    assert alpha.dtype == np.float64 and alpha.flags.c_contiguous
    nf = nfuncs(reps, w.basis)
    ab = np.zeros(nf)
    x = np.zeros((M, w.d)) if want_x else None
    s = np.zeros(M) if want_s else None
    rc = lib().or_backward_step(C.byref(p), reps.shape[0], _ptr(reps), i, M, seed, _ptr(alpha),
                                _ptr(ab), _ptr(x) if want_x else None,
                                _ptr(s) if want_s else None)
    if rc:
        raise ValueError("or_backward_step failed")
    return alpha[i].copy(), ab, x, s


def mlp_forward(theta, x, law: str = "logistic") -> np.ndarray:
    """The learned form's surrogate network (bfloat16 operands of its two
    matrix products, exact sums) at states x [n][d], features 2 F(x_l) - 1."""
    th = _f64(theta)
    x = np.atleast_2d(_f64(x))
    return np.array([lib().or_mlp_forward(_ptr(th), LAWS[law], x.shape[1], _ptr(np.ascontiguousarray(r)))
                     for r in x])


def backward_step_z(w, reps, i, M, seed, alpha):
    """Z of eq (MDP:intro:0a) at time index i from the rows i+1.. of alpha
    ([N][nf]): returns (alpha_z [nbm][nf], abs_z [nbm][nf])."""
    p = problem(w)
    reps = np.ascontiguousarray(reps, dtype=np.int32)
    nf = nfuncs(reps, w.basis)
    az = np.zeros((w.nbm, nf))
    ab = np.zeros((w.nbm, nf))
    rc = lib().or_backward_step_z(C.byref(p), reps.shape[0], _ptr(reps), i, M, seed, _ptr(_f64(alpha)), _ptr(az),
                                  _ptr(ab))
    if rc:
        raise ValueError("or_backward_step_z failed")
    return az, ab


def backward_step_z1(w, reps, i, M, seed, alpha):
    """Z of the one-step scheme, eq (ODP:intro:a), at time index i from the
    rows i+1.. of alpha ([N][nf]): returns (alpha_z [nbm][nf], abs_z [nbm][nf])."""
    p = problem(w)
    reps = np.ascontiguousarray(reps, dtype=np.int32)
    nf = nfuncs(reps, w.basis)
    az = np.zeros((w.nbm, nf))
    ab = np.zeros((w.nbm, nf))
    rc = lib().or_backward_step_z1(C.byref(p), reps.shape[0], _ptr(reps), i, M, seed, _ptr(_f64(alpha)), _ptr(az),
                                   _ptr(ab))
    if rc:
        raise ValueError("or_backward_step_z1 failed")
    return az, ab


def backward_step_learned(w, reps, i, M, seed, alpha, nets, mu, sd):
    """or_backward_step with surrogates: nets[j] (a parameter vector, or None
    for the expansion) with target scaling mu[j], sd[j] replaces ybar_j along
    the paths.  Fills alpha[i] in place; returns (alpha_row, abs_row)."""
    p = problem(w)
    reps = np.ascontiguousarray(reps, dtype=np.int32)
    assert alpha.dtype == np.float64 and alpha.flags.c_contiguous
    keep = [None if t is None else _f64(t) for t in nets]
    ptrs = (C.c_void_p * w.N)(*[None if t is None else t.ctypes.data for t in keep])
    mu_a, sd_a = _f64(mu), _f64(sd)
    ab = np.zeros(nfuncs(reps, w.basis))
    rc = lib().or_backward_step_learned(C.byref(p), reps.shape[0], _ptr(reps), i, M, seed, _ptr(alpha),
                                        _ptr(ab), ptrs, _ptr(mu_a), _ptr(sd_a))
    if rc:
        raise ValueError("or_backward_step_learned failed")
    return alpha[i].copy(), ab


def damping(w, x) -> float:
    """(1+|x|^2)^{q/2} of eq (yqi) for the workload's q."""
    p = problem(w)
    return lib().or_damping(C.byref(p), _ptr(np.ascontiguousarray(_f64(x))))


def eval_y(w, reps, alpha_row, x, grad: bool = False):
    """y(x) = ybar^{(q)}(x) (1+|x|^2)^{q/2} from one coefficient row, and its
    x-gradient (one point x of length d)."""
    p = problem(w)
    reps = np.ascontiguousarray(reps, dtype=np.int32)
    x = np.ascontiguousarray(_f64(x))
    g = np.zeros(w.d)
    y = lib().or_eval_y(C.byref(p), reps.shape[0], _ptr(reps), _ptr(_f64(alpha_row)), _ptr(x),
                        _ptr(g) if grad else None)
    return (y, g) if grad else y


def path_response(w, reps, i, seed, m, alpha) -> float:
    p = problem(w)
    reps = np.ascontiguousarray(reps, dtype=np.int32)
    return lib().or_path_response(C.byref(p), reps.shape[0], _ptr(reps), i, seed, m,
                                  _ptr(_f64(alpha)))


def solve(w, reps, M=None, seed=None) -> np.ndarray:
    p = problem(w)
    reps = np.ascontiguousarray(reps, dtype=np.int32)
    alpha = np.zeros((w.N, nfuncs(reps, w.basis)))
    rc = lib().or_solve(C.byref(p), reps.shape[0], _ptr(reps), w.M if M is None else M,
                        w.seed if seed is None else seed, _ptr(alpha))
    if rc:
        raise ValueError("or_solve failed")
    return alpha


def sample_points(d, seed, stream, i, n, m0=0, law: str = "logistic") -> np.ndarray:
    x = np.zeros((n, d))
    lib().or_sample_points(d, LAWS[law], seed, stream, i, m0, n, _ptr(x))
    return x


def errors(w, reps, alpha, seed=0, n=1 << 12):
    """(MSE_max, MSE_av, relative L2 error at t_0) of eq (mse)."""
    p = problem(w)
    reps = np.ascontiguousarray(reps, dtype=np.int32)
    out = np.zeros(3)
    lib().or_errors(C.byref(p), reps.shape[0], _ptr(reps), _ptr(_f64(alpha)), seed, n, _ptr(out))
    return tuple(out)


def num_threads() -> int:
    return int(lib().or_num_threads())
