"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests and the bench.

This module draws random matrices only; it holds none of the SVD method's
arithmetic.  Matrices follow the construction of the paper's test families
(Section 7.1 and Tables 1-2): A = U diag(sigma) V^T with Haar-distributed
orthogonal factors, optionally followed by a column scaling D (A = B D).

All matrices are returned as float64 numpy arrays in Fortran (column-major)
order, the layout the library consumes.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "haar", "sigma_geometric", "sigma_log_uniform", "compose", "xlatm1",
    "config_c1", "config_c2", "config_c3a", "config_c3b", "config_c4",
    "config_c5", "graded", "CONFIG_SHAPES",
]

CONFIG_SHAPES = {
    "C1": (128, 128),
    "C2": (1024, 1024),
    "C3a": (8192, 2048),
    "C3b": (4096, 4096),
    "C5": (128, 64),
}


def haar(rng: np.random.Generator, k: int, n: int) -> np.ndarray:
    """k-by-n matrix with orthonormal columns, Haar distributed.

    Gaussian G = QR, then Q diag(sign(diag R)) with sign(0) = +1; without the
    sign fix the Q factor of a Gaussian matrix is not Haar distributed.
    """
    g = rng.standard_normal((k, n))
    q, r = np.linalg.qr(g)
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return q * d


def sigma_geometric(n: int, e: float) -> np.ndarray:
    """sigma_i = 10^(-e (i-1)/(n-1)): Table 2 MODE 3 with kappa = 10^e."""
    if n == 1:
        return np.ones(1)
    i = np.arange(n, dtype=np.float64)
    return 10.0 ** (-e * i / (n - 1))


def sigma_log_uniform(rng: np.random.Generator, n: int, e: float) -> np.ndarray:
    """Logarithms uniform on (-e, 0), sorted descending: Table 2 MODE 5 style."""
    r = rng.uniform(0.0, 1.0, n)
    return np.sort(10.0 ** (-e * r))[::-1].copy()


def xlatm1(mode: int, n: int, kappa: float, rng: np.random.Generator | None = None) -> np.ndarray:
    """Diagonal generator with the five modes of Table 2 (largest entry 1)."""
    i = np.arange(n, dtype=np.float64)
    if mode == 1:
        d = np.full(n, 1.0 / kappa)
        d[0] = 1.0
    elif mode == 2:
        d = np.ones(n)
        d[-1] = 1.0 / kappa
    elif mode == 3:
        d = kappa ** (-i / max(n - 1, 1))
    elif mode == 4:
        # 1 - (i-1)/(n-1) (1 - 1/kappa), rearranged so that the last entry is
        # 1/kappa rather than a cancellation to 0 when 1/kappa < u
        d = 1.0 / kappa + (n - 1 - i) / max(n - 1, 1) * (1.0 - 1.0 / kappa)
    elif mode == 5:
        assert rng is not None
        d = np.exp(rng.uniform(np.log(1.0 / kappa), 0.0, n))
    else:
        raise ValueError(mode)
    return d


def compose(u: np.ndarray, s: np.ndarray, v: np.ndarray) -> np.ndarray:
    """A = U diag(s) V^T in float64, column-major."""
    return np.asfortranarray((u * s) @ v.T)


def graded(seed: int, m: int, n: int, mode_sigma: int, kappa_b: float,
           mode_d: int, kappa_d: float) -> np.ndarray:
    """A = B D with B = W1 Sigma W2 and D diagonal (Section 7.1 family).

    The unit-column-norm factor W3 of the paper is not reproduced (its
    construction is not given); B keeps the column norms of W1 Sigma W2.
    """
    rng = np.random.default_rng(seed)
    w1 = haar(rng, m, n)
    w2 = haar(rng, n, n)
    s = xlatm1(mode_sigma, n, kappa_b, rng)
    d = xlatm1(mode_d, n, kappa_d, rng)
    b = (w1 * s) @ w2.T
    return np.asfortranarray(b * d)


def config_c1(n: int = 128, seed: int = 1):
    """128x128, Haar U, V, sigma geometric from 1 to 1e-8."""
    rng = np.random.default_rng(seed)
    u = haar(rng, n, n)
    v = haar(rng, n, n)
    s = sigma_geometric(n, 8.0)
    return compose(u, s, v), s


def config_c2(n: int = 1024, seed: int = 2):
    """A = B D: B = U diag(sigma) V^T, sigma log-uniform in [1e-6, 1],
    D = diag(10^w), w ~ U(-6, 0), unsorted."""
    rng = np.random.default_rng(seed)
    u = haar(rng, n, n)
    v = haar(rng, n, n)
    s = sigma_log_uniform(rng, n, 6.0)
    w = rng.uniform(-6.0, 0.0, n)
    b = (u * s) @ v.T
    return np.asfortranarray(b * (10.0 ** w)), None


def config_c3a(m: int = 8192, n: int = 2048, seed: int = 3):
    """Tall m x n, Haar U (m x n), V (n x n), sigma geometric from 1 to 1e-10."""
    rng = np.random.default_rng(seed)
    u = haar(rng, m, n)
    v = haar(rng, n, n)
    s = sigma_geometric(n, 10.0)
    return compose(u, s, v), s


def config_c3b(n: int = 4096, seed: int = 4):
    """Square n x n, Haar U, V, sigma log-uniform in [1e-12, 1]."""
    rng = np.random.default_rng(seed)
    u = haar(rng, n, n)
    v = haar(rng, n, n)
    s = sigma_log_uniform(rng, n, 12.0)
    return compose(u, s, v), s


def config_c4(batch: int = 2000, seed: int = 5, mmin: int = 16, mmax: int = 256,
              first: int = 0, count: int | None = None):
    """Ragged batch: m_j ~ U{mmin..mmax}, n_j ~ U{mmin..m_j}; Haar U, V,
    sigma log-uniform in [1e-8, 1].

    Child 0 of SeedSequence(seed) draws the shapes, child j+1 draws matrix j,
    so any sub-range [first, first+count) is reproducible on its own.
    Returns (shapes, list of matrices, list of sigma).
    """
    ss = np.random.SeedSequence(seed)
    children = ss.spawn(batch + 1)
    rng0 = np.random.default_rng(children[0])
    ms = rng0.integers(mmin, mmax + 1, size=batch)
    ns = np.array([rng0.integers(mmin, m + 1) for m in ms])
    shapes = list(zip(ms.tolist(), ns.tolist()))
    if count is None:
        count = batch - first
    mats, sigs = [], []
    for j in range(first, first + count):
        rng = np.random.default_rng(children[j + 1])
        m, n = shapes[j]
        u = haar(rng, m, n)
        v = haar(rng, n, n)
        s = sigma_log_uniform(rng, n, 8.0)
        mats.append(compose(u, s, v))
        sigs.append(s)
    return shapes, mats, sigs


def config_c5(batch: int = 256, m: int = 128, n: int = 64, seed: int = 6,
              cot_seed: int = 7, dir_seed: int = 8, ndir: int = 8):
    """Gradient workload: batch of m x n matrices, sigma ~ U(0.1, 10) sorted
    descending and redrawn until the minimum relative gap is >= 1e-3;
    cotangents gU, gS, gV ~ N(0, 1); unit-Frobenius FD directions.

    Returns dict with A (batch, m, n) row-major stack of column-major
    matrices given as a (batch, n, m) transposed view is avoided: A[b] is a
    Fortran-ordered m x n array.
    """
    rng = np.random.default_rng(seed)
    mats, sigs = [], []
    for _ in range(batch):
        u = haar(rng, m, n)
        v = haar(rng, n, n)
        while True:
            s = np.sort(rng.uniform(0.1, 10.0, n))[::-1].copy()
            gap = np.min((s[:-1] - s[1:]) / s[:-1]) if n > 1 else 1.0
            if gap >= 1e-3:
                break
        mats.append(compose(u, s, v))
        sigs.append(s)
    crng = np.random.default_rng(cot_seed)
    gu = crng.standard_normal((batch, m, n))
    gs = crng.standard_normal((batch, n))
    gv = crng.standard_normal((batch, n, n))
    drng = np.random.default_rng(dir_seed)
    dirs = drng.standard_normal((batch, ndir, m, n))
    dirs /= np.linalg.norm(dirs, axis=(2, 3), keepdims=True)
    return {"A": mats, "sigma": sigs, "gU": gu, "gS": gs, "gV": gv, "E": dirs}
