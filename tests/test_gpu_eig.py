"""GPU parity: eig_mixed (Algorithm 6) through the C ABI against the FP64
oracle eigendecomposition (cyclic two-sided Jacobi).

Gates on every case: e_lambda = max_i |w_i - w_i^ref| / |w_i^ref| divided by
max(1, kappa_s(A)) <= 1e-13, ||X^T X - I||_F <= 1e-13 n, and
||A X - X diag(w)||_F / ||A||_F <= 1e-14 n.  The inputs are A = Q diag(lam) Q^T
with Haar Q and indefinite lam, including +-pairs of equal magnitude (the case
that needs the blocks of U^T A U) and repeated eigenvalues.
"""
import numpy as np
import pytest

import oracle
import testmats
from testmats import metrics

pytestmark = pytest.mark.gpu


def sym_known(n, seed, e=6.0, pairs=(), repeats=(), sign=None):
    rng = np.random.default_rng(seed)
    mag = 10.0 ** -rng.uniform(0, e, n)
    if sign is None:
        lam = mag * np.where(rng.random(n) < 0.5, -1.0, 1.0)
    else:
        lam = sign * mag
    for i in pairs:
        lam[i + 1] = -lam[i]
    for i in repeats:
        lam[i + 1] = lam[i]
    Q = testmats.haar(rng, n, n)
    A = (Q * lam) @ Q.T
    return (A + A.T) / 2, lam


def run_eig(lib, A, **kw):
    import torch
    At = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    W, X, info = lib.eigh(At, **kw)
    torch.cuda.synchronize()
    return W.cpu().numpy(), X.cpu().numpy(), info


def eig_gates(A, W, X, Wref):
    n = A.shape[0]
    ks = metrics.kappa_s(A) if n > 1 else 1.0
    rel = np.max(np.abs(W - Wref) / np.abs(Wref))
    e = rel / max(1.0, ks)
    orth = np.linalg.norm(X.T @ X - np.eye(n))
    res = np.linalg.norm(A @ X - X * W) / np.linalg.norm(A)
    return {"e_lambda": e, "rel": rel, "kappa_s": ks, "orth": orth, "residual": res,
            "pass": bool(e <= 1e-13 and orth <= 1e-13 * n and res <= 1e-14 * n)}


@pytest.mark.parametrize("n", [1, 2, 5, 64, 65, 130, 200])
def test_eig_parity_sizes(lib, n):
    print(f"case eig n={n}", flush=True)
    pairs = [0, 3] if n >= 5 else []
    repeats = [7] if n >= 9 else []
    A, lam = sym_known(n, seed=100 + n, pairs=pairs, repeats=repeats)
    Wref, Xref, _ = oracle.eigh(A)
    W, X, info = run_eig(lib, A)
    g = eig_gates(A, W, X, Wref)
    assert info["status"] == 0 and g["pass"], (g, info)
    if n >= 5:
        assert info["n_clusters"] >= 2, info
    # vectors of well separated eigenvalues agree with the oracle's (same sign rule)
    gap = np.ones(n)
    if n > 1:
        d = np.abs(np.diff(Wref)) / np.maximum(np.abs(Wref[:-1]), np.abs(Wref[1:]))
        gap[:-1] = np.minimum(gap[:-1], d)
        gap[1:] = np.minimum(gap[1:], d)
    sep = gap > 1e-3
    if sep.any():
        assert np.max(np.abs(X[:, sep] - Xref[:, sep])) < 1e-8


def test_eig_exact_plus_minus_pair_2x2(lib):
    """[[0, 1], [1, 0]]: eigenvalues -1 and 1, one block of two equal singular
    values."""
    A = np.array([[0.0, 1.0], [1.0, 0.0]])
    W, X, info = run_eig(lib, A)
    assert info["status"] == 0 and info["n_clusters"] == 1 and info["max_cluster"] == 2, info
    assert np.max(np.abs(W - np.array([-1.0, 1.0]))) <= 4e-16
    Wref, Xref, _ = oracle.eigh(A)
    assert np.max(np.abs(X - Xref)) <= 1e-15


def test_eig_multiplicity_block(lib):
    """0.5 three times and -0.5 twice: one block of five equal singular values."""
    n = 80
    A, lam = sym_known(n, seed=7)
    rng = np.random.default_rng(8)
    lam[10:13] = 0.5
    lam[13:15] = -0.5
    Q = testmats.haar(rng, n, n)
    A = (Q * lam) @ Q.T
    A = (A + A.T) / 2
    Wref, _, _ = oracle.eigh(A)
    W, X, info = run_eig(lib, A)
    g = eig_gates(A, W, X, Wref)
    assert info["status"] == 0 and g["pass"], (g, info)
    assert info["max_cluster"] == 5, info
    assert np.max(np.abs(W - np.sort(lam))) <= 1e-14


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_eig_definite(lib, sign):
    """Definite matrices: every block is a single column."""
    A, lam = sym_known(150, seed=9, sign=sign)
    Wref, _, _ = oracle.eigh(A)
    W, X, info = run_eig(lib, A)
    g = eig_gates(A, W, X, Wref)
    assert info["status"] == 0 and g["pass"] and info["n_clusters"] == 0, (g, info)
    assert np.all(np.sign(W) == sign)


def test_eig_cluster_too_large_reports_status(lib):
    """A block of 70 equal singular values (the identity) exceeds the 64-column
    limit: the status says so, nothing is launched for it."""
    W, X, info = run_eig(lib, np.eye(70))
    assert info["status"] == 4 and info["max_cluster"] == 70, info


def test_eig_graded_definite_accuracy(lib):
    """A = D H D with D graded over 8 orders: the eigenvalues meet the
    kappa_s-adjusted gate; the unadjusted relative error is reported."""
    rng = np.random.default_rng(12)
    n = 96
    G = rng.standard_normal((n, n))
    H = G @ G.T / n + np.eye(n)
    d = 10.0 ** -rng.uniform(0, 8, n)
    A = (H * d).T * d
    A = (A + A.T) / 2
    Wref, _, _ = oracle.eigh(A)
    W, X, info = run_eig(lib, A)
    g = eig_gates(A, W, X, Wref)
    print(f"graded: rel {g['rel']:.2e} kappa_s {g['kappa_s']:.2e}", flush=True)
    assert info["status"] == 0 and g["pass"], (g, info)


def test_eig_relative_accuracy_beyond_library_eigh(lib):
    """Section 8's point: on a graded definite matrix (eigenvalues over 16
    orders) the Jacobi-refined eigenvalues keep their leading digits where a
    normwise library solver (torch.linalg.eigh) loses the small ones.  The
    relative error is bounded by the rows' grading, which the column-pivoted
    preconditioner does not remove (measured 1.2e-10; the library 0.22)."""
    import torch
    rng = np.random.default_rng(13)
    n = 128
    G = rng.standard_normal((n, n))
    H = G @ G.T / n + np.eye(n)
    d = 10.0 ** -rng.uniform(0, 8, n)
    A = (H * d).T * d
    A = (A + A.T) / 2
    Wref, _, _ = oracle.eigh(A)
    W, X, info = run_eig(lib, A)
    rel = float(np.max(np.abs(W - Wref) / np.abs(Wref)))
    Wt = torch.linalg.eigvalsh(torch.from_numpy(A).cuda()).cpu().numpy()
    rel_lib = float(np.max(np.abs(Wt - Wref) / np.abs(Wref)))
    print(f"graded, eigenvalues over 16 orders: eig_mixed rel {rel:.2e}, "
          f"torch.linalg.eigvalsh rel {rel_lib:.2e}", flush=True)
    assert info["status"] == 0 and rel <= 1e-9, (rel, info)
    assert rel_lib > 1e6 * rel
