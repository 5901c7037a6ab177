"""FP64 CPU oracle for the one-sided Jacobi SVD.

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py, never by the library.  The numerical routines
live in oracle.c (plain C, FP64); this module loads liboracle.so with ctypes
and adds the SVD adjoint formula (adjoint.py, numpy FP64).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .adjoint import svd_backward_ref  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from .build import build
            build()
        lib = ctypes.CDLL(path)
        lib.oracle_svd.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, _dp,
                                   _dp, ctypes.c_int, _dp, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                   ctypes.c_int, _ip, _ip]
        lib.oracle_geqr2.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, _dp]
        lib.oracle_geqp3.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, _ip, _dp]
        lib.oracle_apply_q.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int,
                                       _dp, ctypes.c_int, _dp, ctypes.c_int]
        lib.oracle_rotation.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp, _dp]
        lib.oracle_gesvj.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int, _dp,
                                     ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int, _ip]
        lib.oracle_finalize.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, _dp,
                                        ctypes.c_int, _dp, ctypes.c_int]
        lib.oracle_sign_normalize.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, _dp, ctypes.c_int]
        lib.oracle_rr_pair.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _ip, _ip]
        lib.oracle_syevj.argtypes = [ctypes.c_int, _dp, ctypes.c_int, _dp, _dp, ctypes.c_int,
                                     ctypes.c_double, ctypes.c_int, ctypes.c_int, _ip]
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_max_threads.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def _d(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    return np.asfortranarray(np.asarray(a, dtype=np.float64))


def set_threads(t: int) -> None:
    _lib().oracle_set_threads(int(t))


def set_verbose(v: bool) -> None:
    """Progress lines on stderr during long oracle runs (phase ends, sweeps)."""
    _lib().oracle_set_verbose(int(bool(v)))


def max_threads() -> int:
    return int(_lib().oracle_max_threads())


def svd(A, precondition: bool = True, order: str = "cyclic", eps: float = 0.0,
        maxiter: int = 60, sign_normalize: bool = True):
    """SVD A = U diag(S) V^T (m >= n) by FP64 preconditioned one-sided Jacobi.

    Returns (U, S, V, info) with info = {status, sweeps, jpvt}.
    """
    A = _f64(A)
    m, n = A.shape
    U = np.zeros((m, n), order="F")
    S = np.zeros(n)
    V = np.zeros((n, n), order="F")
    sweeps = ctypes.c_int(0)
    jpvt = np.zeros(max(n, 1), dtype=np.int32)
    st = _lib().oracle_svd(m, n, _d(A), max(m, 1), _d(S), _d(U), max(m, 1), _d(V), max(n, 1),
                           int(precondition), 0 if order == "cyclic" else 1, float(eps),
                           int(maxiter), int(sign_normalize), ctypes.byref(sweeps),
                           jpvt.ctypes.data_as(_ip))
    if st < 0:
        raise ValueError(f"oracle_svd: bad argument ({st})")
    return U, S, V, {"status": st, "sweeps": sweeps.value, "jpvt": jpvt[:n].copy()}


def eigh(A, eps: float = 0.0, maxiter: int = 60, sign_normalize: bool = True):
    """Symmetric eigendecomposition A = X diag(w) X^T by FP64 cyclic two-sided
    Jacobi; w ascending.  Returns (w, X, info) with info = {status, sweeps}."""
    A = _f64(A)
    n = A.shape[0]
    if A.shape != (n, n):
        raise ValueError("A must be square")
    w = np.zeros(max(n, 1))
    X = np.zeros((n, n), order="F")
    sweeps = ctypes.c_int(0)
    st = _lib().oracle_syevj(n, _d(A), max(n, 1), _d(w), _d(X), max(n, 1), float(eps), int(maxiter),
                             int(sign_normalize), ctypes.byref(sweeps))
    if st < 0:
        raise ValueError(f"oracle_syevj: bad argument ({st})")
    return w[:n].copy(), X, {"status": st, "sweeps": sweeps.value}


def geqr2(A):
    """Householder QR: returns (factored A, tau)."""
    A = _f64(A).copy(order="F")
    m, n = A.shape
    tau = np.zeros(max(min(m, n), 1))
    _lib().oracle_geqr2(m, n, _d(A), max(m, 1), _d(tau))
    return A, tau[:min(m, n)]


def geqp3(A):
    """Businger-Golub QRCP: returns (factored A, jpvt, tau)."""
    A = _f64(A).copy(order="F")
    m, n = A.shape
    jpvt = np.zeros(max(n, 1), dtype=np.int32)
    tau = np.zeros(max(min(m, n), 1))
    _lib().oracle_geqp3(m, n, _d(A), max(m, 1), jpvt.ctypes.data_as(_ip), _d(tau))
    return A, jpvt[:n].copy(), tau[:min(m, n)]


def apply_q(Qf, tau, C, trans: bool = False):
    """Q C or Q^T C for Q held as reflectors (from geqr2 / geqp3)."""
    Qf = _f64(Qf)
    C = _f64(C).copy(order="F")
    m, k = Qf.shape[0], len(tau)
    tau = np.ascontiguousarray(tau, dtype=np.float64)
    _lib().oracle_apply_q(int(trans), m, k, _d(Qf), max(m, 1), _d(tau), C.shape[1], _d(C), max(m, 1))
    return C


def form_q(Qf, tau, ncols=None):
    m = Qf.shape[0]
    ncols = Qf.shape[1] if ncols is None else ncols
    return apply_q(Qf, tau, np.eye(m, ncols, order="F"))


def rotation(alpha: float, beta: float, gamma: float):
    c = ctypes.c_double()
    s = ctypes.c_double()
    _lib().oracle_rotation(alpha, beta, gamma, ctypes.byref(c), ctypes.byref(s))
    return c.value, s.value


def gesvj(X, V=None, eps: float = 0.0, maxiter: int = 60, order: str = "cyclic"):
    """Algorithm 1 sweeps on X (and V if given); returns (X, V, status, sweeps)."""
    X = _f64(X).copy(order="F")
    m, n = X.shape
    e = eps if eps > 0 else np.sqrt(m) * 2.0 ** -53
    sweeps = ctypes.c_int(0)
    vp = None
    nv = 0
    if V is not None:
        V = _f64(V).copy(order="F")
        nv = V.shape[0]
        vp = _d(V)
    st = _lib().oracle_gesvj(m, n, _d(X), max(m, 1), nv, vp, max(nv, 1), e, int(maxiter),
                             0 if order == "cyclic" else 1, ctypes.byref(sweeps))
    return X, V, st, sweeps.value


def finalize(X, V=None):
    X = _f64(X).copy(order="F")
    m, n = X.shape
    S = np.zeros(n)
    nv = 0
    vp = None
    if V is not None:
        V = _f64(V).copy(order="F")
        nv = V.shape[0]
        vp = _d(V)
    z = _lib().oracle_finalize(m, n, _d(X), max(m, 1), _d(S), nv, vp, max(nv, 1))
    return X, S, V, z


def sign_normalize(U, V):
    U = _f64(U).copy(order="F")
    V = _f64(V).copy(order="F")
    _lib().oracle_sign_normalize(U.shape[0], U.shape[1], _d(U), max(U.shape[0], 1), _d(V), max(V.shape[0], 1))
    return U, V


def rr_pair(n: int, r: int, k: int):
    p = ctypes.c_int()
    q = ctypes.c_int()
    _lib().oracle_rr_pair(n, r, k, ctypes.byref(p), ctypes.byref(q))
    return p.value, q.value
