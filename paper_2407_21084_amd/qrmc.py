"""Thin ctypes binding of libqrmc (include/qrmc.h).

Argument marshalling only: every step of the method runs in the HIP library.
Device buffers are torch tensors on a ROCm device (their data pointers are
passed through); streams are torch streams.  If the shared library has not
been built, importing this module raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("QRMC_LIB") or os.path.join(_HERE, "libqrmc.so")

MAX_D = 16
MAX_N = 128
MAX_BATCH = 64
MLP_IN, MLP_HIDDEN = 16, 256
MLP_NPARAMS = MLP_HIDDEN * MLP_IN + MLP_HIDDEN + MLP_HIDDEN * MLP_HIDDEN + MLP_HIDDEN + MLP_HIDDEN + 1
MLP_MAX_BATCH = 65536

SET_TENSOR, SET_HC_MAX, SET_HC_1P, SET_TOTAL = 0, 1, 2, 3
SET_KINDS = {"tensor": SET_TENSOR, "hc_max": SET_HC_MAX, "hc_1p": SET_HC_1P, "total": SET_TOTAL}
F_LINEAR, F_SIN, F_ALLEN_CAHN, F_ZRAT, F_PAPER = 0, 1, 2, 3, 4
BASIS_FOURIER, BASIS_COSINE = 0, 1
BASES = {"fourier": BASIS_FOURIER, "cosine": BASIS_COSINE}
LAW_LOGISTIC, LAW_STUDENT2, LAW_CAUCHY = 0, 1, 2
LAWS = {"logistic": LAW_LOGISTIC, "student2": LAW_STUDENT2, "cauchy": LAW_CAUCHY}
DRIVERS = {"linear": F_LINEAR, "sin": F_SIN, "allen_cahn": F_ALLEN_CAHN, "zrat": F_ZRAT, "paper": F_PAPER}

STATUS = {0: "QR_OK", -1: "QR_EINVAL", -2: "QR_ENOMEM", -3: "QR_EDEVICE", -4: "QR_ERANGE",
          -5: "QR_ENUMERIC", -6: "QR_ENOTSUP"}

PREC_F64, PREC_BF16, PREC_F16 = 0, 1, 2
PRECISIONS = {"f64": PREC_F64, "bf16": PREC_BF16, "f16": PREC_F16}
PREC_KERNELS = {"auto": 0, "walk": 1, "factored": 2}

# kernel classes of qr_ctx_kernel_time
K_PATH, K_PROJECT, K_REDUCE, K_GATHER = 0, 1, 2, 3

EXPORTS = ["qr_last_error", "qr_version", "qr_build_basis", "qr_build_basis_law", "qr_basis_law",
           "qr_basis_info", "qr_basis_indices", "qr_sample_points_law",
           "qr_basis_free", "qr_ctx_create", "qr_ctx_destroy", "qr_ctx_set_timing",
           "qr_ctx_kernel_time", "qr_ctx_reset_timing", "qr_backward_step", "qr_solve", "qr_eval",
           "qr_project", "qr_path_responses", "qr_sample_points", "qr_backward_step_prec",
           "qr_solve_prec", "qr_mlp_init", "qr_mlp_features", "qr_mlp_forward", "qr_mlp_loss_grad",
           "qr_mlp_adam", "qr_solve_learned", "qr_solve_batched",
           "qr_basis_upload", "qr_eval_noalloc", "qr_ctx_set_prec_kernel", "qr_basis_factored",
           "qr_ctx_numeric_status", "qr_build_basis_cos", "qr_basis_family_of", "qr_solve_from",
           "qr_ctx_set_mem_limit", "qr_ctx_mem_held", "qr_eval_y",
           "qr_batch_graph_create", "qr_batch_graph_launch", "qr_batch_graph_destroy",
           "qr_backward_step_z", "qr_solve_z", "qr_eval_split",
           "qr_host_uniform", "qr_host_norm_icdf", "qr_host_philox"]


Z_SCHEMES = {"multistep": 0, "onestep": 1}


class QrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Problem(C.Structure):
    _fields_ = [
        ("d", C.c_int32), ("nbm", C.c_int32), ("N", C.c_int32), ("driver", C.c_int32),
        ("f_a", C.c_double), ("clamp", C.c_double),
        ("t", C.c_double * (MAX_N + 1)),
        ("b0", C.c_double * MAX_D), ("b1", C.c_double * MAX_D),
        ("sigma", C.c_double * (MAX_D * MAX_D)),
        ("sol_A", C.c_double), ("sol_c", C.c_double), ("sol_p", C.c_double),
        ("sol_w", C.c_double * MAX_D),
        ("damping_q", C.c_double),
        ("sol_B", C.c_double),
        ("b2", C.c_double * MAX_D), ("sigma_v", C.c_double * MAX_D), ("sigma_omega", C.c_double),
    ]


class Instance(C.Structure):
    """One instance of a batched solve (qr_instance)."""
    _fields_ = [("f_a", C.c_double), ("d", C.c_int32), ("level", C.c_int32), ("M", C.c_int64)]


class LearnOpts(C.Structure):
    """Options of the learned form (qr_learn_opts)."""
    _fields_ = [("train_points", C.c_int64), ("heldout_points", C.c_int64), ("epochs", C.c_int32),
                ("batch", C.c_int32), ("lr", C.c_float), ("gate", C.c_double), ("reject", C.c_double)]


class LearnReport(C.Structure):
    """Per-time-index outcome of the learned form (qr_learn_report)."""
    _fields_ = [("heldout_rel_l2", C.c_double), ("train_loss", C.c_double), ("trained", C.c_int32),
                ("used", C.c_int32), ("target_mean", C.c_double), ("target_sd", C.c_double),
                ("epochs_run", C.c_int32)]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: run paper_2407_21084_amd/build.py (hipcc, gfx950)")

# torch ships its own HIP runtime.  Loading it first makes the library bind
# to that same runtime (one device context per process, shared streams and
# allocations); loaded the other way round, two runtimes would compete for
# the device.
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)
_P, _I32, _I64, _U64, _U32, _D = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_uint32, C.c_double
_SIGS = {
    "qr_last_error": (C.c_char_p, []),
    "qr_version": (C.c_char_p, []),
    "qr_build_basis": (C.c_int, [_I32, _I32, _I32, C.POINTER(_P)]),
    "qr_build_basis_law": (C.c_int, [_I32, _I32, _I32, _I32, C.POINTER(_P)]),
    "qr_basis_law": (C.c_int, [_P, C.POINTER(_I32)]),
    "qr_build_basis_cos": (C.c_int, [_I32, _I32, _I32, _I32, C.POINTER(_P)]),
    "qr_basis_family_of": (C.c_int, [_P, C.POINTER(_I32)]),
    "qr_solve_from": (C.c_int, [_P, C.POINTER(Problem), _P, _I32, _I64, _U64, _I32, _P, _P]),
    "qr_ctx_set_mem_limit": (C.c_int, [_P, _I64]),
    "qr_ctx_mem_held": (C.c_int, [_P, C.POINTER(_I64)]),
    "qr_eval_y": (C.c_int, [_P, C.POINTER(Problem), _P, _P, _I64, _P, _P, _P, _P]),
    "qr_batch_graph_create": (C.c_int, [_P, C.POINTER(Problem), _P, _I32, C.c_void_p, _U64, _P, _P, C.POINTER(_P)]),
    "qr_batch_graph_launch": (C.c_int, [_P, _P]),
    "qr_batch_graph_destroy": (None, [_P]),
    "qr_basis_info": (C.c_int, [_P, C.POINTER(_I64), C.POINTER(_I64), C.POINTER(_I32)]),
    "qr_basis_indices": (C.c_int, [_P, _P]),
    "qr_basis_free": (None, [_P]),
    "qr_ctx_create": (C.c_int, [_I32, C.POINTER(_P)]),
    "qr_ctx_destroy": (None, [_P]),
    "qr_ctx_set_timing": (C.c_int, [_P, _I32]),
    "qr_ctx_kernel_time": (C.c_int, [_P, _I32, C.POINTER(_D), C.POINTER(_I64)]),
    "qr_ctx_reset_timing": (C.c_int, [_P]),
    "qr_backward_step": (C.c_int, [_P, C.POINTER(Problem), _P, _I32, _I64, _U64, _P, _P]),
    "qr_solve": (C.c_int, [_P, C.POINTER(Problem), _P, _I64, _U64, _P, _P]),
    "qr_eval_split": (C.c_int, [_P, _P, _P, _I64, _P, _P, _P]),
    "qr_backward_step_z": (C.c_int, [_P, C.POINTER(Problem), _P, _I32, _I64, _U64, _I32, _P, _P, _P]),
    "qr_solve_z": (C.c_int, [_P, C.POINTER(Problem), _P, _I64, _U64, _I32, _P, _P, _P]),
    "qr_eval": (C.c_int, [_P, _P, _P, _I64, _P, _P, _P, _P]),
    "qr_basis_upload": (C.c_int, [_P, _P]),
    "qr_ctx_set_prec_kernel": (C.c_int, [_P, _I32]),
    "qr_ctx_numeric_status": (C.c_int, [_P, C.POINTER(_I32)]),
    "qr_basis_factored": (C.c_int, [_P, C.POINTER(_I32), C.POINTER(_I32), C.POINTER(_I32), C.POINTER(_I64)]),
    "qr_eval_noalloc": (C.c_int, [_P, _P, _P, _I64, _P, _P, _P, _P]),
    "qr_project": (C.c_int, [_P, _P, _I64, _P, _P, _P, _P]),
    "qr_path_responses": (C.c_int, [_P, C.POINTER(Problem), _P, _I32, _I64, _U64, _P, _P, _P, _P]),
    "qr_sample_points": (C.c_int, [_P, _I32, _U64, _U32, _I32, _I64, _I64, _P, _P]),
    "qr_sample_points_law": (C.c_int, [_P, _I32, _I32, _U64, _U32, _I32, _I64, _I64, _P, _P]),
    "qr_backward_step_prec": (C.c_int, [_P, C.POINTER(Problem), _P, _I32, _I64, _U64, _I32, _P, _P]),
    "qr_solve_prec": (C.c_int, [_P, C.POINTER(Problem), _P, _I64, _U64, _I32, _P, _P]),
    "qr_mlp_init": (C.c_int, [_P, _P, _U64, _P]),
    "qr_mlp_features": (C.c_int, [_P, _I32, _I64, _P, _P, _P]),
    "qr_mlp_forward": (C.c_int, [_P, _P, _I64, _P, _P, _P]),
    "qr_mlp_loss_grad": (C.c_int, [_P, _P, _I64, _P, _P, _P, C.POINTER(_D), _P]),
    "qr_mlp_adam": (C.c_int, [_P, _P, _P, _P, _P, _I64, C.c_float, _P]),
    "qr_solve_learned": (C.c_int, [_P, C.POINTER(Problem), _P, _I64, _U64, C.POINTER(LearnOpts), _P,
                                   C.POINTER(LearnReport), _P, _P]),
    "qr_solve_batched": (C.c_int, [_P, C.POINTER(Problem), _P, _I32, C.POINTER(Instance), _U64, _P, _P]),
    "qr_host_uniform": (_D, [_U64, _U32, _U64, _U32, _U32]),
    "qr_host_norm_icdf": (_D, [_D]),
    "qr_host_philox": (None, [_P, _P, _P]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def lib():
    return _lib


def _check(status: int) -> None:
    if status != 0:
        raise QrError(status, _lib.qr_last_error().decode())


def version() -> str:
    return _lib.qr_version().decode()


# ---------------------------------------------------------------------------
# host-side helpers (no device)
# ---------------------------------------------------------------------------

def host_uniform(seed, stream, m, i, r) -> float:
    return _lib.qr_host_uniform(seed, stream, m, i, r)


def host_norm_icdf(u: float) -> float:
    return _lib.qr_host_norm_icdf(u)


def host_philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _lib.qr_host_philox(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


class Basis:
    """Index set Gamma and its basis metadata for the sampling law `law`:
    the Fourier functions over Z^d (qr_build_basis_law), or the paper's cosine
    functions over N^d with basis="cosine" (qr_build_basis_cos)."""

    def __init__(self, d: int, kind, level: int, law="logistic", basis="fourier"):
        kind = SET_KINDS[kind] if isinstance(kind, str) else int(kind)
        law = LAWS[law] if isinstance(law, str) else int(law)
        basis = BASES[basis] if isinstance(basis, str) else int(basis)
        h = _P()
        build = _lib.qr_build_basis_cos if basis == BASIS_COSINE else _lib.qr_build_basis_law
        _check(build(d, kind, level, law, C.byref(h)))
        self._h = h
        self.d, self.kind, self.level = d, kind, level
        fam = _I32()
        _check(_lib.qr_basis_family_of(h, C.byref(fam)))
        self.family = fam.value
        got = _I32()
        _check(_lib.qr_basis_law(h, C.byref(got)))
        self.law = got.value
        nf, nr, mn = _I64(), _I64(), _I32()
        _check(_lib.qr_basis_info(h, C.byref(nf), C.byref(nr), C.byref(mn)))
        self.n_funcs, self.n_reps, self.max_nnz = nf.value, nr.value, mn.value

    @property
    def handle(self):
        return self._h

    def indices(self) -> np.ndarray:
        out = np.zeros((self.n_reps, self.d), dtype=np.int32)
        _check(_lib.qr_basis_indices(self._h, out.ctypes.data))
        return out

    def factored(self):
        """The factored layout of the reduced-precision form: (split, row tiles,
        K-blocks, coefficient blocks per time step), or None if no split qualifies."""
        sp, rt, kb, nb = _I32(), _I32(), _I32(), _I64()
        st = _lib.qr_basis_factored(self._h, C.byref(sp), C.byref(rt), C.byref(kb), C.byref(nb))
        if st == -6:
            return None
        _check(st)
        return sp.value, rt.value, kb.value, nb.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _lib.qr_basis_free(h)
            self._h = None


class BatchGraph:
    """A captured batched solve (qr_batch_graph); keeps its inputs alive."""

    def __init__(self, h, keep):
        self._h, self._keep = h, keep

    def launch(self, stream):
        _check(_lib.qr_batch_graph_launch(self._h, _stream_ptr(stream)))

    def close(self):
        if self._h:
            _lib.qr_batch_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


def make_problem(d, N, T=None, times=None, sigma=None, b0=None, b1=None, driver="sin", f_a=0.0,
                 sol_A=1.0, sol_c=1.0, sol_p=0.0, sol_w=None, clamp=math.inf, damping_q=0.0,
                 sol_B=0.0, b2=None, sigma_v=None, sigma_omega=0.0) -> Problem:
    sigma = np.eye(d) if sigma is None else np.asarray(sigma, dtype=np.float64)
    nbm = sigma.shape[1]
    if times is None:
        times = [T * j / N for j in range(N + 1)]
    p = Problem()
    p.d, p.nbm, p.N = d, nbm, N
    p.driver = DRIVERS[driver] if isinstance(driver, str) else int(driver)
    p.f_a, p.clamp = f_a, clamp
    for j, t in enumerate(times):
        p.t[j] = t
    b0 = [0.0] * d if b0 is None else b0
    b1 = [0.0] * d if b1 is None else b1
    sol_w = [1.0] * d if sol_w is None else sol_w
    for l in range(d):
        p.b0[l], p.b1[l], p.sol_w[l] = b0[l], b1[l], sol_w[l]
        for k in range(nbm):
            p.sigma[l * nbm + k] = sigma[l, k]
    p.sol_A, p.sol_c, p.sol_p = sol_A, sol_c, sol_p
    p.damping_q = damping_q
    p.sol_B = sol_B
    for l in range(d):
        p.b2[l] = 0.0 if b2 is None else b2[l]
        p.sigma_v[l] = 0.0 if sigma_v is None else sigma_v[l]
    p.sigma_omega = sigma_omega
    return p


def problem_from(w) -> Problem:
    """Marshal any object with the workload attributes (d, N, T, sigma, b0,
    b1, driver, f_a, sol_*, clamp, optionally damping_q, sol_B, b2, sigma_v and
    sigma_omega) into a qr_problem."""
    return make_problem(w.d, w.N, T=w.T, sigma=w.sigma, b0=w.b0, b1=w.b1, driver=w.driver,
                        f_a=w.f_a, sol_A=w.sol_A, sol_c=w.sol_c, sol_p=w.sol_p, sol_w=w.sol_w,
                        clamp=w.clamp, damping_q=getattr(w, "damping_q", 0.0), sol_B=getattr(w, "sol_B", 0.0),
                        b2=getattr(w, "b2", None), sigma_v=getattr(w, "sigma_v", None),
                        sigma_omega=getattr(w, "sigma_omega", 0.0))


# ---------------------------------------------------------------------------
# device side
# ---------------------------------------------------------------------------

def _stream_ptr(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _dptr(t) -> C.c_void_p:
    if t is None:
        return C.c_void_p(0)
    import torch
    assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous(), "float64 contiguous device tensor expected"
    return C.c_void_p(t.data_ptr())


def _fptr(t) -> C.c_void_p:
    if t is None:
        return C.c_void_p(0)
    import torch
    assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous(), "float32 contiguous device tensor expected"
    return C.c_void_p(t.data_ptr())


class Context:
    """qr_ctx on one device; owns the library workspace."""

    def __init__(self, device: int = 0):
        h = _P()
        _check(_lib.qr_ctx_create(device, C.byref(h)))
        self._h = h
        self.device = device

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            _lib.qr_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def numeric_status(self) -> int:
        """Time index of the latest non-finite row since the last check (-1 for
        none); raises QrError (QR_ENUMERIC) if there is one."""
        st = _I32()
        _check(_lib.qr_ctx_numeric_status(self._h, C.byref(st)))
        return st.value

    def set_prec_kernel(self, kind):
        k = PREC_KERNELS[kind] if isinstance(kind, str) else int(kind)
        _check(_lib.qr_ctx_set_prec_kernel(self._h, k))

    def set_timing(self, on: bool):
        _check(_lib.qr_ctx_set_timing(self._h, 1 if on else 0))

    def kernel_time(self, which: int):
        ms, n = _D(), _I64()
        _check(_lib.qr_ctx_kernel_time(self._h, which, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def reset_timing(self):
        _check(_lib.qr_ctx_reset_timing(self._h))

    # -- the method ----------------------------------------------------------
    def backward_step(self, prob: Problem, basis: Basis, i: int, M: int, seed: int, alpha, stream=None):
        _check(_lib.qr_backward_step(self._h, C.byref(prob), basis.handle, i, M, seed, _dptr(alpha),
                                     _stream_ptr(stream)))

    def solve(self, prob: Problem, basis: Basis, M: int, seed: int, alpha, stream=None):
        _check(_lib.qr_solve(self._h, C.byref(prob), basis.handle, M, seed, _dptr(alpha),
                             _stream_ptr(stream)))

    def eval_split(self, basis: Basis, alpha_row, x, y, stream=None):
        """qr_eval (values) with the basis split across blocks, for n <= 2^17 points."""
        n = y.shape[0]
        _check(_lib.qr_eval_split(self._h, basis.handle, _dptr(alpha_row), n, _dptr(x), _dptr(y),
                                  _stream_ptr(stream)))

    def backward_step_z(self, prob: Problem, basis: Basis, i: int, M: int, seed: int, alpha, alpha_z,
                        scheme="multistep", stream=None):
        """Row i of alpha and slice i of alpha_z ([N][nbm][n_funcs]): the Z regression of
        eq (MDP:intro:0a) (scheme "multistep") or eq (ODP:intro:a) ("onestep")."""
        _check(_lib.qr_backward_step_z(self._h, C.byref(prob), basis.handle, i, M, seed, Z_SCHEMES.get(scheme, scheme),
                                       _dptr(alpha), _dptr(alpha_z), _stream_ptr(stream)))

    def solve_z(self, prob: Problem, basis: Basis, M: int, seed: int, alpha, alpha_z, scheme="multistep",
                stream=None):
        _check(_lib.qr_solve_z(self._h, C.byref(prob), basis.handle, M, seed, Z_SCHEMES.get(scheme, scheme),
                               _dptr(alpha), _dptr(alpha_z), _stream_ptr(stream)))

    def backward_step_prec(self, prob: Problem, basis: Basis, i: int, M: int, seed: int, precision,
                           alpha, stream=None):
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        _check(_lib.qr_backward_step_prec(self._h, C.byref(prob), basis.handle, i, M, seed, prec,
                                          _dptr(alpha), _stream_ptr(stream)))

    def solve_prec(self, prob: Problem, basis: Basis, M: int, seed: int, precision, alpha, stream=None):
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        _check(_lib.qr_solve_prec(self._h, C.byref(prob), basis.handle, M, seed, prec, _dptr(alpha),
                                  _stream_ptr(stream)))

    def solve_from(self, prob: Problem, basis: Basis, i_start: int, M: int, seed: int, alpha, precision="f64",
                   stream=None):
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        _check(_lib.qr_solve_from(self._h, C.byref(prob), basis.handle, i_start, M, seed, prec, _dptr(alpha),
                                  _stream_ptr(stream)))

    def set_mem_limit(self, nbytes: int):
        _check(_lib.qr_ctx_set_mem_limit(self._h, int(nbytes)))

    def mem_held(self) -> int:
        v = _I64()
        _check(_lib.qr_ctx_mem_held(self._h, C.byref(v)))
        return v.value

    def eval(self, basis: Basis, alpha_row, x, y, grad=None, stream=None):
        n = y.shape[0]
        _check(_lib.qr_eval(self._h, basis.handle, _dptr(alpha_row), n, _dptr(x), _dptr(y),
                            _dptr(grad), _stream_ptr(stream)))

    def eval_y(self, prob: Problem, basis: Basis, alpha_row, x, y, grad=None, stream=None):
        n = y.shape[0]
        _check(_lib.qr_eval_y(self._h, C.byref(prob), basis.handle, _dptr(alpha_row), n, _dptr(x), _dptr(y),
                              _dptr(grad), _stream_ptr(stream)))

    def basis_upload(self, basis: Basis):
        _check(_lib.qr_basis_upload(self._h, basis.handle))

    def eval_noalloc(self, basis: Basis, alpha_row, x, y, grad=None, stream=None):
        n = y.shape[0]
        _check(_lib.qr_eval_noalloc(self._h, basis.handle, _dptr(alpha_row), n, _dptr(x), _dptr(y),
                                    _dptr(grad), _stream_ptr(stream)))

    def project(self, basis: Basis, x, s, alpha_row, stream=None):
        n = s.shape[0]
        _check(_lib.qr_project(self._h, basis.handle, n, _dptr(x), _dptr(s), _dptr(alpha_row),
                               _stream_ptr(stream)))

    def path_responses(self, prob: Problem, basis: Basis, i: int, M: int, seed: int, alpha, s,
                       x0=None, stream=None):
        _check(_lib.qr_path_responses(self._h, C.byref(prob), basis.handle, i, M, seed, _dptr(alpha),
                                      _dptr(s), _dptr(x0), _stream_ptr(stream)))

    def sample_points(self, d: int, seed: int, stream_id: int, i: int, n: int, x, m0: int = 0,
                      stream=None, law="logistic"):
        law = LAWS[law] if isinstance(law, str) else int(law)
        _check(_lib.qr_sample_points_law(self._h, law, d, seed, stream_id, i, m0, n, _dptr(x),
                                         _stream_ptr(stream)))

    def solve_batched(self, prob: Problem, basis: Basis, instances, seed: int, alpha, stream=None):
        """instances: sequence of (f_a, d, level, M); alpha: device [R][N][n_funcs]."""
        R = len(instances)
        arr = (Instance * max(R, 1))()
        for r, (f_a, d, level, M) in enumerate(instances):
            arr[r].f_a, arr[r].d, arr[r].level, arr[r].M = float(f_a), int(d), int(level), int(M)
        _check(_lib.qr_solve_batched(self._h, C.byref(prob), basis.handle, R, arr, seed, _dptr(alpha),
                                     _stream_ptr(stream)))

    def batch_graph(self, prob: Problem, basis: Basis, instances, seed: int, alpha, stream):
        """qr_batch_graph_create: solves once (alpha) and returns a BatchGraph
        whose launch() replays the whole batched solve."""
        R = len(instances)
        arr = (Instance * max(R, 1))()
        for r, (f_a, d, level, M) in enumerate(instances):
            arr[r].f_a, arr[r].d, arr[r].level, arr[r].M = float(f_a), int(d), int(level), int(M)
        h = _P()
        _check(_lib.qr_batch_graph_create(self._h, C.byref(prob), basis.handle, R, C.cast(arr, C.c_void_p), seed,
                                          _dptr(alpha), _stream_ptr(stream), C.byref(h)))
        return BatchGraph(h, (prob, basis, arr, alpha))

    # -- learned form ---------------------------------------------------------
    def mlp_init(self, params, seed: int, stream=None):
        _check(_lib.qr_mlp_init(self._h, _fptr(params), seed, _stream_ptr(stream)))

    def mlp_features(self, d: int, x, feat, stream=None):
        n = feat.shape[0]
        _check(_lib.qr_mlp_features(self._h, d, n, _dptr(x), _fptr(feat), _stream_ptr(stream)))

    def mlp_forward(self, params, feat, y, stream=None):
        _check(_lib.qr_mlp_forward(self._h, _fptr(params), y.shape[0], _fptr(feat), _fptr(y), _stream_ptr(stream)))

    def mlp_loss_grad(self, params, feat, target, grad, stream=None) -> float:
        loss = _D()
        _check(_lib.qr_mlp_loss_grad(self._h, _fptr(params), target.shape[0], _fptr(feat), _fptr(target),
                                     _fptr(grad), C.byref(loss), _stream_ptr(stream)))
        return loss.value

    def mlp_adam(self, params, grad, m, v, step: int, lr: float, stream=None):
        _check(_lib.qr_mlp_adam(self._h, _fptr(params), _fptr(grad), _fptr(m), _fptr(v), step, lr,
                                _stream_ptr(stream)))

    def solve_learned(self, prob: Problem, basis: Basis, M: int, seed: int, alpha, train_points=1 << 18,
                      heldout_points=1 << 16, epochs=8, batch=8192, lr=1e-3, gate=1e-3, params=None, stream=None,
                      reject=0.0):
        """Returns the per-time-index reports as a list of dicts; params (float32
        device [N][MLP_NPARAMS], optional) receives the fitted parameters."""
        o = LearnOpts(train_points, heldout_points, epochs, batch, lr, gate, reject)
        rep = (LearnReport * prob.N)()
        _check(_lib.qr_solve_learned(self._h, C.byref(prob), basis.handle, M, seed, C.byref(o), _dptr(alpha),
                                     rep, _fptr(params), _stream_ptr(stream)))
        return [{"heldout_rel_l2": r.heldout_rel_l2, "train_loss": r.train_loss, "trained": bool(r.trained),
                 "used": bool(r.used), "target_mean": r.target_mean, "target_sd": r.target_sd,
                 "epochs_run": r.epochs_run} for r in rep]
