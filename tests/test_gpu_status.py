"""GPU checks of the numerical status paths, the branch tests of Section 3.5
and Proposition 1's fail-safe property, through the C ABI.

- status: NaN / Inf input -> SVD_ERR_NONFINITE; an exactly zero singular
  value -> SVD_WARN_RANK_DEFICIENT with a zero U column and a finite,
  orthogonal V (the triangular solve for V meets a zero pivot and takes the
  other route of Section 3.4); a capped FP64 stage -> SVD_WARN_NOCONV; a
  bounded cross-workgroup wait forced to give up -> a non-OK status, never
  NaN with SVD_OK.
- branch tests: each of Section 3.5's three triggers (small cond_R, many
  small trailing columns, nearly orthogonal X_t) alone takes the SKIP branch;
  info.orth agrees with max|X_t^T X_t - I| formed in numpy from the pivoted
  QR and the LQ of A (on inputs whose pivot order is fixed).
- Proposition 1: with the FP32 stage forced and cut short (0, 1 or 2
  sweeps), the FP64 refinement still meets every gate.
"""
import numpy as np
import pytest

import oracle
import testmats
from testmats import metrics

pytestmark = pytest.mark.gpu


def run(lib, A, mode, **kw):
    import torch
    At = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    U, S, V, info = lib.svd(At, mode, **kw)
    torch.cuda.synchronize()
    return U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy(), info


def known(m, n, seed, e=8.0):
    rng = np.random.default_rng(seed)
    return testmats.compose(testmats.haar(rng, m, n), testmats.sigma_log_uniform(rng, n, e),
                            testmats.haar(rng, n, n))


@pytest.mark.parametrize("mode", ["plain", "mixed"])
@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
def test_nonfinite_input(lib, mode, bad):
    print(f"case nonfinite {bad} mode={mode}", flush=True)
    A = known(150, 120, seed=1)
    A[37, 91] = bad
    U, S, V, info = run(lib, A, mode)
    assert info["status"] == lib.SVD_ERR_NONFINITE, info


def zero_sigma_matrix(n, seed):
    """A = H diag(d) with orthonormal H and d_n = 0: the last column of A is
    exactly zero and so is the last column of X = L (its only entry l_nn is
    zero), so sigma_n = 0 exactly."""
    rng = np.random.default_rng(seed)
    H = testmats.haar(rng, n, n)
    d = testmats.sigma_geometric(n, 4.0)
    d[-1] = 0.0
    return np.asfortranarray(H * d), d


@pytest.mark.parametrize("mode", ["plain", "mixed"])
@pytest.mark.parametrize("v_method", [0, 1])
def test_rank_deficient_zero_column(lib, mode, v_method):
    print(f"case zero column mode={mode} v_method={v_method}", flush=True)
    n = 200
    A, d = zero_sigma_matrix(n, seed=5)
    U, S, V, info = run(lib, A, mode, v_method=v_method, branch=1 if mode == "mixed" else 0)
    assert info["status"] == lib.SVD_WARN_RANK_DEFICIENT, info
    assert np.all(np.isfinite(U)) and np.all(np.isfinite(S)) and np.all(np.isfinite(V))
    assert S[-1] == 0.0 and np.all(U[:, -1] == 0.0)
    assert metrics.orth_err(V) <= 1e-13 * n
    assert metrics.orth_err(U[:, :-1]) <= 1e-13 * n
    assert metrics.residual(A, U, S, V) <= 1e-14 * n
    ds = np.sort(d)[::-1]
    assert np.max(np.abs(S[:-1] - ds[:-1]) / ds[:-1]) < 1e-12
    if v_method == 1:
        # the solve met the zero pivot of L: V came from the other route
        assert info["v_method_taken"] == 2, info


@pytest.mark.parametrize("mode", ["plain", "mixed"])
def test_duplicated_column(lib, mode):
    """A duplicated column: sigma_n is at the rounding level, not exactly zero;
    every output stays finite and the orthogonality and residual gates hold."""
    print(f"case duplicated column mode={mode}", flush=True)
    n = 180
    A = known(n, n, seed=9, e=4.0)
    A[:, n - 1] = A[:, 3]
    U, S, V, info = run(lib, A, mode)
    assert info["status"] in (lib.SVD_OK, lib.SVD_WARN_RANK_DEFICIENT), info
    assert np.all(np.isfinite(U)) and np.all(np.isfinite(V)) and np.all(np.isfinite(S))
    assert S[-1] <= 1e-13 * S[0]
    assert metrics.orth_err(V) <= 1e-13 * n
    assert metrics.residual(A, U, S, V) <= 1e-14 * n


@pytest.mark.parametrize("mode", ["plain", "mixed"])
def test_sweep_cap_reports_noconv(lib, mode):
    print(f"case maxsweep_work=1 mode={mode}", flush=True)
    A = known(256, 256, seed=11, e=10.0)
    U, S, V, info = run(lib, A, mode, maxsweep_work=1, branch=1 if mode == "mixed" else 0)
    assert info["status"] == lib.SVD_WARN_NOCONV and info["sweeps_work"] == 1, info


@pytest.mark.parametrize("mode", ["plain", "mixed"])
def test_forced_wait_timeout_is_reported(lib, mode):
    """wait_polls = -1 makes every bounded wait give up at its first check
    (each kernel still runs to its end).  n = 600 spans three row groups of
    the one-launch Householder panel, so its waits are real; the FP32 pivot
    pass falls back to per-step launches.  The call must report a non-OK
    status; it never returns NaN with SVD_OK.  The same matrix with the
    default bound meets the gates."""
    print(f"case wait_polls=-1 mode={mode}", flush=True)
    n = 600
    A = known(n, n, seed=13, e=8.0)
    U, S, V, info = run(lib, A, mode, wait_polls=-1)
    ok_result = np.all(np.isfinite(S))
    assert info["status"] == lib.SVD_ERR_WAIT_TIMEOUT or (info["status"] == 0 and ok_result), info
    assert not (info["status"] == 0 and not ok_result)
    Uo, So, Vo, _ = oracle.svd(A)
    U, S, V, info = run(lib, A, mode)
    g = metrics.gates(A, U, S, V, So)
    assert info["status"] == 0 and g["pass"], (g, info)


def test_pivot_pass_timeout_falls_back(lib):
    """n = 128 has a single row group per Householder panel (no waits there);
    with wait_polls = -1 only the one-launch FP32 pivot pass gives up, and its
    step-by-step fallback yields a correct SVD with SVD_OK."""
    print("case pivot fallback n=128", flush=True)
    A = known(128, 128, seed=17)
    Uo, So, Vo, _ = oracle.svd(A)
    U, S, V, info = run(lib, A, "mixed", wait_polls=-1, branch=1)
    g = metrics.gates(A, U, S, V, So)
    assert info["status"] == 0 and g["pass"], (g, info)


# ----------------------------------------------------------------- branch tests
def x_of(A):
    """X = L of the preconditioner with FP64 Businger-Golub pivots: A P = Q1 R
    (oracle QRCP), R = L Q2 (numpy QR of R^T).  Column signs of L do not
    change max|X_t^T X_t - I|."""
    Af, jpvt, tau = oracle.geqp3(A)
    n = A.shape[1]
    R = np.triu(Af[:n, :n])
    return np.linalg.qr(R.T, mode="r").T, jpvt


def orth_ref(X):
    Xt = (X / np.linalg.norm(X, axis=0)).astype(np.float32).astype(np.float64)
    return float(np.max(np.abs(Xt.T @ Xt - np.eye(X.shape[1]))))


def test_skip_on_small_cond_r(lib):
    print("case skip cond_R", flush=True)
    n = 256
    rng = np.random.default_rng(21)
    A = np.asfortranarray(np.eye(n) + 0.05 * rng.standard_normal((n, n)) / np.sqrt(n))
    U, S, V, info = run(lib, A, "mixed")
    assert info["branch_taken"] == lib.BRANCH_SKIP, info
    assert info["cond_r"] <= 1.5 * n ** 0.25 and info["orth"] == -1.0, info
    So = oracle.svd(A)[1]
    assert metrics.gates(A, U, S, V, So)["pass"]


def test_skip_on_many_small_trailing_columns(lib):
    print("case skip small columns", flush=True)
    n = 256
    A = known(n, n, seed=22, e=2.0)
    k = n // 4 + 3
    A[:, -k:] *= 1e-20
    U, S, V, info = run(lib, A, "mixed")
    assert info["branch_taken"] == lib.BRANCH_SKIP, info
    assert info["n_small"] >= int(np.ceil(0.25 * n)) and info["orth"] == -1.0, info
    assert info["cond_r"] > 1.5 * n ** 0.25
    So = oracle.svd(A)[1]
    assert metrics.gates(A, U, S, V, So)["pass"]


def test_skip_on_nearly_orthogonal_x(lib):
    """A = H D, H orthonormal, D graded over six decades: cond_R = 1e6 and no
    small columns, but X = L is diagonal up to rounding, so X_t is orthogonal
    to FP32 accuracy and the orth test alone skips the FP32 stage."""
    print("case skip orth", flush=True)
    n = 256
    rng = np.random.default_rng(23)
    H = testmats.haar(rng, n, n)
    d = 10.0 ** (-6.0 * rng.uniform(0, 1, n))
    d[0], d[1] = 1.0, 1e-6
    A = np.asfortranarray(H * d)
    U, S, V, info = run(lib, A, "mixed")
    assert info["cond_r"] > 1.5 * n ** 0.25 and info["n_small"] == 0, info
    X, _ = x_of(A)
    ref = orth_ref(X)
    assert ref <= 1e-5
    assert 0.0 <= info["orth"] <= 1e-5 and info["branch_taken"] == lib.BRANCH_SKIP, (info, ref)
    So = oracle.svd(A)[1]
    assert metrics.gates(A, U, S, V, So)["pass"]


def pivot_determined(n, seed):
    """Upper triangular A with a_kk = +-0.9^k and a_ic = 0.9^c g_ic, g_ic ~
    0.3 N(0,1)/sqrt(n) (i < c): the trailing norm of column c at any step k < c
    is at most 1.05 0.9^c < 0.95 |a_kk|, so Businger-Golub keeps the identity
    order in any precision, and the QR of A P = A is A itself."""
    rng = np.random.default_rng(seed)
    d = 0.9 ** np.arange(n)
    A = np.triu(rng.standard_normal((n, n)) * 0.3 / np.sqrt(n)) * d[None, :]
    A[np.arange(n), np.arange(n)] = d * np.where(rng.standard_normal(n) < 0, -1.0, 1.0)
    return np.asfortranarray(A)


@pytest.mark.parametrize("seed", [31, 32])
def test_orth_measure_matches_numpy(lib, seed):
    """info.orth (FP32 SYRK of X_t on the matrix cores) against max|X_t^T X_t
    - I| from the FP32-rounded X_t in FP64, on the same X: the input fixes the
    pivot order (identity, checked on the oracle's QRCP), so X = L of the LQ of
    R = A is the GPU's X up to column signs."""
    print(f"case orth measure seed={seed}", flush=True)
    n = 192
    A = pivot_determined(n, seed)
    U, S, V, info = run(lib, A, "mixed", branch=1)
    X, jpvt = x_of(A)
    assert np.array_equal(jpvt, np.arange(n))
    ref = orth_ref(X)
    assert ref > 1e-3, ref
    assert abs(info["orth"] - ref) <= 1e-5 + 1e-3 * ref, (info["orth"], ref)
    So = oracle.svd(A)[1]
    assert metrics.gates(A, U, S, V, So)["pass"]


# ----------------------------------------------------------------- Proposition 1
@pytest.mark.parametrize("maxsweep_low", [0, 1, 2])
@pytest.mark.parametrize("shape", [(300, 300), (260, 130)])
def test_fp32_stage_cut_short_still_accurate(lib, maxsweep_low, shape):
    """Section 4: the refinement's accuracy does not depend on how far the
    FP32 stage got.  With the stage forced and capped at 0, 1 or 2 sweeps the
    FP64 sweeps take longer but every gate holds."""
    m, n = shape
    print(f"case T3 maxsweep_low={maxsweep_low} shape={shape}", flush=True)
    A = known(m, n, seed=41 + maxsweep_low, e=10.0)
    Uo, So, Vo, _ = oracle.svd(A)
    U, S, V, info = run(lib, A, "mixed", branch=1, maxsweep_low=maxsweep_low)
    g = metrics.gates(A, U, S, V, So)
    assert info["status"] == 0 and info["branch_taken"] == lib.BRANCH_LOW, info
    assert info["sweeps_low"] <= maxsweep_low
    assert g["pass"], (g, info)
