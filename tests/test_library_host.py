"""Host-side checks of libqrmc that need no GPU: the library loads and
exports every symbol of include/qrmc.h, its host mirrors of the scalar device
routines agree with independent references, and the index-set enumeration
is bit-identical to the oracle's."""
import math
import os
import re

import numpy as np
import pytest
from scipy import special

import oracle as O
import workloads as W
from paper_2407_21084_amd import qrmc as Q

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")


def test_exports_every_declared_symbol():
    header = open(os.path.join(ROOT, "include", "qrmc.h")).read()
    declared = set(re.findall(r"\b(qr_[a-z_0-9]+)\s*\(", header))
    assert len(declared) >= 18
    for name in declared:
        assert hasattr(Q.lib(), name), name
    assert set(Q.EXPORTS) == declared
    assert "gfx950" in Q.version()


def test_host_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    for r in rows:
        v = [int(h, 16) for h in r]
        assert list(Q.host_philox(v[0:4], v[4:6])) == v[6:10]


def test_host_uniform_matches_oracle_stream():
    """Two independent implementations of the same stream layout agree bit for bit."""
    for seed in (0, 1, 0xDEADBEEF12345678):
        for stream in (0, 1, 4):
            for m in (0, 1, 12345, (1 << 33) + 7):
                for i in (0, 9):
                    for r in range(5):
                        assert Q.host_uniform(seed, stream, m, i, r) == O.uniform(seed, stream, m, i, r)


def test_host_norm_icdf_matches_scipy():
    us = np.concatenate([np.logspace(-300, -1, 300), np.linspace(0.01, 0.99, 99),
                         1 - np.logspace(-15, -2, 60), [2.0 ** -53, 0.5, 1 - 2.0 ** -53]])
    for u in us:
        a, b = Q.host_norm_icdf(float(u)), float(special.ndtri(u))
        assert abs(a - b) <= 2e-15 * max(1.0, abs(b)), (u, a, b)


@pytest.mark.parametrize("d,kind,level", [(1, "tensor", 6), (2, "tensor", 4), (3, "tensor", 2),
                                          (2, "hc_max", 4), (3, "hc_max", 7), (5, "hc_max", 9),
                                          (4, "hc_1p", 12), (6, "hc_1p", 20), (2, "tensor", 0),
                                          (3, "hc_max", 1), (1, "total", 5), (2, "total", 6),
                                          (4, "total", 4), (7, "total", 3), (3, "total", 0)])
def test_basis_enumeration_matches_oracle(d, kind, level):
    b = Q.Basis(d, kind, level)
    ref = O.enumerate_set(d, kind, level)
    assert b.n_reps == ref.shape[0]
    assert b.n_funcs == 2 * ref.shape[0] - 1 == O.count_set(d, kind, level)
    assert np.array_equal(b.indices(), ref)
    assert b.max_nnz == (int(np.max(np.count_nonzero(ref, axis=1))) if ref.shape[0] else 0)


@pytest.mark.parametrize("w", [W.D2_TENSOR4, W.D6_HCMAX16, W.D10_HC1P32_ZRAT, W.D16_HC1P32], ids=lambda w: w.name)
def test_configuration_bases_match_oracle(w):
    b = Q.Basis(w.d, w.set_kind, w.level)
    ref = O.enumerate_set(w.d, w.set_kind, w.level)
    assert np.array_equal(b.indices(), ref)
    assert b.max_nnz <= 8


@pytest.mark.parametrize("d,kind,level", [(1, "tensor", 100), (2, "tensor", 4), (3, "hc_max", 7),
                                          (5, "hc_max", 9), (4, "hc_1p", 12), (2, "total", 6),
                                          (5, "total", 4), (3, "tensor", 0), (6, "hc_max", 16)])
def test_cosine_basis_enumeration_matches_oracle(d, kind, level):
    """The cosine basis over N^d (Sec. 2.2, eq (phi:dim:d)) on the sets of
    Sec. 2.3.3: its vectors and coefficient order are the oracle's N^d
    enumeration (lexicographic), and the paper's own cardinality of
    Gamma_T(DEG) over N^d, binom(DEG + d, d), holds."""
    b = Q.Basis(d, kind, level, basis="cosine")
    ref = O.enumerate_set(d, kind, level, nonneg=True, reps_only=False)
    assert b.family == Q.BASIS_COSINE
    assert b.n_funcs == b.n_reps == ref.shape[0]
    assert np.array_equal(b.indices(), ref)
    if kind == "total":
        assert b.n_funcs == math.comb(level + d, d)
    # the Fourier basis of the same set is its carrier: every vector of N^d in
    # it has 2^{n-1} representatives over Z^d (n non-zero coordinates)
    f = Q.Basis(d, kind, level)
    assert f.family == Q.BASIS_FOURIER
    nnz = np.count_nonzero(ref, axis=1)
    assert f.n_reps == 1 + int(np.sum(2.0 ** (nnz[nnz > 0] - 1)))


def test_cosine_product_to_sum_identity():
    """The identity the kernels evaluate the cosine basis through: for k in
    N^d with n non-zero coordinates, prod_l c_{k_l}(u_l) (c_0 = 1,
    c_m = sqrt2 cos(m pi u)) equals 2^{1 - n/2} times the sum of
    cos(pi k'.u) over the vectors k' of Z^d with |k'| = k and first non-zero
    coordinate positive; checked against the oracle's cosine basis values."""
    rng = np.random.default_rng(3)
    d, level = 4, 3
    vecs = O.enumerate_set(d, "tensor", level, nonneg=True, reps_only=False)
    x = rng.standard_normal(d)
    u = np.array([0.5 * (1.0 + v / math.sqrt(1.0 + v * v)) for v in x])  # Student mu = 2 CDF
    phi = O.basis_values(vecs, x, law="student2", basis="cosine")
    for c, k in enumerate(vecs):
        nz = np.flatnonzero(k)
        if nz.size == 0:
            assert phi[c] == 1.0
            continue
        tot = 0.0
        for signs in range(1 << (nz.size - 1)):
            kp = k.astype(float).copy()
            for q in range(1, nz.size):
                if (signs >> (q - 1)) & 1:
                    kp[nz[q]] = -kp[nz[q]]
            tot += math.cos(math.pi * float(kp @ u))
        assert abs(2.0 ** (1 - nz.size / 2) * tot - phi[c]) <= 1e-12 * max(1.0, abs(phi[c])), (k, phi[c])


def test_invalid_arguments_are_rejected():
    with pytest.raises(Q.QrError) as e:
        Q.Basis(0, "tensor", 2)
    assert e.value.status == -1
    with pytest.raises(Q.QrError):
        Q.Basis(17, "tensor", 2)
    with pytest.raises(Q.QrError):
        Q.Basis(2, 7, 2)
    with pytest.raises(Q.QrError):
        Q.Basis(2, "tensor", -1)
    # hyperbolic crosses below level 1 are empty (the oracle agrees)
    for kind in ("hc_max", "hc_1p"):
        assert O.count_set(3, kind, 0) == 0
        with pytest.raises(Q.QrError):
            Q.Basis(3, kind, 0)
    assert Q.Basis(3, "tensor", 0).n_funcs == 1 == O.count_set(3, "tensor", 0)


def test_context_without_device_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(Q.QrError) as e:
        Q.Context(0)
    assert e.value.status == -3


def test_basis_law_is_recorded_and_unknown_laws_rejected():
    for name, code in Q.LAWS.items():
        b = Q.Basis(3, "hc_1p", 8, law=name)
        assert b.law == code
        # the law does not change the index set
        assert np.array_equal(b.indices(), O.enumerate_set(3, "hc_1p", 8))
    assert Q.Basis(2, "tensor", 2).law == Q.LAW_LOGISTIC
    for bad in (-1, 3, 99):
        with pytest.raises(Q.QrError) as e:
            Q.Basis(2, "tensor", 2, law=bad)
        assert e.value.status == -1


def test_header_is_plain_c():
    """include/qrmc.h is a C header: it compiles as C99 and as C++17 with
    warnings as errors (no torch or C++ types in the boundary)."""
    import shutil
    import subprocess
    hdr = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "qrmc.h")
    for cc, std, lang in (("gcc", "c99", "c"), ("g++", "c++17", "c++")):
        if shutil.which(cc) is None:
            pytest.skip(f"{cc} not available")
        r = subprocess.run([cc, f"-std={std}", "-Wall", "-Wextra", "-Werror", "-fsyntax-only", "-x", lang, hdr],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
