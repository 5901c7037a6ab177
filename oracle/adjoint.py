"""Reference SVD adjoint in numpy FP64 (test infrastructure only).

The paper does not differentiate the SVD; this is the standard matrix-calculus
result for A = U diag(s) V^T with U m x n (orthonormal columns), V n x n
orthogonal and distinct singular values.  With J = U^T gU, K = V^T gV and
F_ij = 1 / (s_j^2 - s_i^2) (i != j), F_ii = 0:

    gA = U [ (F o (J - J^T)) S + diag(gs) + S (F o (K - K^T)) ] V^T
         + (I_m - U U^T) gU S^{-1} V^T

(the companion term U S^{-1} gV^T (I_n - V V^T) vanishes because V is
square).  Near-degenerate pairs are guarded by replacing 1/d with
d / (d^2 + eta^2), d = s_j^2 - s_i^2, eta = eps_deg * s_1^2.
"""
from __future__ import annotations

import numpy as np


def f_matrix(s: np.ndarray, eps_deg: float = 1e-12) -> np.ndarray:
    s = np.asarray(s, dtype=np.float64)
    s2 = s * s
    d = s2[None, :] - s2[:, None]          # d_ij = s_j^2 - s_i^2
    eta = eps_deg * (s2.max() if s.size else 0.0)
    with np.errstate(divide="ignore", invalid="ignore"):
        f = d / (d * d + eta * eta)
    np.fill_diagonal(f, 0.0)
    f[~np.isfinite(f)] = 0.0
    return f


def svd_backward_ref(U, s, V, gU=None, gs=None, gV=None, eps_deg: float = 1e-12):
    """gA for one matrix; any cotangent may be None (= zero)."""
    U = np.asarray(U, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    m, n = U.shape
    F = f_matrix(s, eps_deg)
    inner = np.zeros((n, n))
    if gU is not None:
        J = U.T @ gU
        inner += (F * (J - J.T)) * s[None, :]
    if gs is not None:
        inner += np.diag(np.asarray(gs, dtype=np.float64))
    if gV is not None:
        K = V.T @ gV
        inner += s[:, None] * (F * (K - K.T))
    gA = U @ inner @ V.T
    if gU is not None and m > n:
        proj = gU - U @ (U.T @ gU)
        gA += (proj / s[None, :]) @ V.T
    return gA
