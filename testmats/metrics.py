"""Accuracy measures used to judge an SVD (numpy FP64).

These evaluate a computed A = U diag(S) V^T; they are not part of the method.
The measures follow the paper's accuracy experiment (Section 7.3): relative
singular value difference, columnwise backward error and the Frobenius-norm
orthogonality of U and V.  kappa_s is the column-scaled condition number
kappa_2(A diag(||A(:, j)||)^-1) of Demmel and Veselic, which bounds the
relative perturbation of the singular values of one-sided Jacobi.
"""
from __future__ import annotations

import numpy as np


def kappa_s(A: np.ndarray) -> float:
    A = np.asarray(A, dtype=np.float64)
    cn = np.linalg.norm(A, axis=0)
    cn[cn == 0] = 1.0
    s = np.linalg.svd(A / cn, compute_uv=False)
    return float(s[0] / s[-1]) if s[-1] > 0 else float("inf")


def rel_sigma_err(S, Sref) -> float:
    S = np.asarray(S, dtype=np.float64)
    Sref = np.asarray(Sref, dtype=np.float64)
    return float(np.max(np.abs(S - Sref) / Sref)) if S.size else 0.0


def e_sigma(S, Sref, ks: float) -> float:
    """max_i |S_i - Sref_i| / Sref_i, divided by max(1, kappa_s)."""
    return rel_sigma_err(S, Sref) / max(1.0, ks)


def normwise_sigma_err(S, Sref) -> float:
    S = np.asarray(S, dtype=np.float64)
    Sref = np.asarray(Sref, dtype=np.float64)
    return float(np.max(np.abs(S - Sref)) / Sref[0]) if S.size else 0.0


def orth_err(Q) -> float:
    Q = np.asarray(Q, dtype=np.float64)
    return float(np.linalg.norm(Q.T @ Q - np.eye(Q.shape[1])))


def residual(A, U, S, V) -> float:
    A = np.asarray(A, dtype=np.float64)
    R = A - (U * S) @ V.T
    return float(np.linalg.norm(R) / np.linalg.norm(A))


def colwise_backward_err(A, U, S, V) -> float:
    A = np.asarray(A, dtype=np.float64)
    R = A - (U * S) @ V.T
    return float(np.max(np.linalg.norm(R, axis=0) / np.linalg.norm(A, axis=0)))


def gates(A, U, S, V, Sref, ks=None) -> dict:
    """The four pass/fail gates: e_sigma <= 1e-13, ||U^T U - I||_F and
    ||V^T V - I||_F <= 1e-13 n, ||A - U S V^T||_F / ||A||_F <= 1e-14 n."""
    n = A.shape[1]
    if ks is None:
        ks = kappa_s(A)
    r = {
        "e_sigma": e_sigma(S, Sref, ks),
        "rel_sigma": rel_sigma_err(S, Sref),
        "normwise_sigma": normwise_sigma_err(S, Sref),
        "orth_u": orth_err(U),
        "orth_v": orth_err(V),
        "residual": residual(A, U, S, V),
        "colwise_bwd": colwise_backward_err(A, U, S, V),
        "kappa_s": ks,
    }
    r["pass"] = bool(r["e_sigma"] <= 1e-13 and r["orth_u"] <= 1e-13 * n
                     and r["orth_v"] <= 1e-13 * n and r["residual"] <= 1e-14 * n)
    return r
