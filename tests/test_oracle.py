"""Pins for the FP64 CPU oracle (no GPU).

Each test ties an oracle routine to something other than the oracle itself:
closed forms, exact arithmetic (mpmath at 60 digits), an independent
implementation (LAPACK via numpy/scipy), or invariants that any correct SVD
satisfies.  Each check is chosen so that a plausible slip (a dropped term, a
wrong sign, a transposed operand or permutation) fails at least one of them.
"""
import json
import os

import mpmath
import numpy as np
import pytest
import scipy.linalg
from scipy.linalg import lapack

import oracle
import testmats
from testmats import metrics

HERE = os.path.dirname(os.path.abspath(__file__))
U53 = 2.0 ** -53


def dgejsv_sigma(A):
    """LAPACK DGEJSV singular values (JOBA='F': full relative accuracy, no
    rank truncation; JOBR='N', JOBP='N'), rescaled by WORK(1)/WORK(2)."""
    res = lapack.dgejsv(A, joba=2, jobr=0, jobp=0)
    assert res[5] == 0
    return res[0] * (res[3][0] / res[3][1])


def exact_sigma(A, dps=60):
    """Singular values of the stored FP64 matrix A in 60-digit arithmetic."""
    with mpmath.workdps(dps):
        M = mpmath.matrix(A.tolist())
        s = mpmath.svd_r(M, compute_uv=False)
        return np.array(sorted([float(x) for x in s], reverse=True))


# --------------------------------------------------------------------------
# 2x2 rotation (Section 2.1)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("cancel", [False, True])
def test_rotation_orthogonalises_pair(seed, cancel):
    rng = np.random.default_rng(seed)
    m = 50
    x = rng.standard_normal((m, 2)) * np.array([1.0, 10.0 ** rng.uniform(-8, 0)])
    if cancel:
        x[:, 1] += 0.3 * x[:, 0]          # x_q mostly parallel to x_p
    else:
        x[:, 1] += 0.3 * x[:, 0] * np.abs(x[0, 1])
    a, b, g = x[:, 0] @ x[:, 0], x[:, 1] @ x[:, 1], x[:, 0] @ x[:, 1]
    c, s = oracle.rotation(a, b, g)
    # closest-to-identity root: |theta| <= pi/4, i.e. |t| <= 1, c >= 1/sqrt(2)
    assert c >= 1 / np.sqrt(2) - 1e-15 and abs(s / c) <= 1.0 + 1e-15
    assert abs(c * c + s * s - 1) < 4 * U53
    J = np.array([[c, s], [-s, c]])
    y = x @ J
    a2, b2, g2 = y[:, 0] @ y[:, 0], y[:, 1] @ y[:, 1], y[:, 0] @ y[:, 1]
    # new columns orthogonal to the rounding level of the rotation and dot
    # product, measured against the norms before the rotation (the rotation
    # may cancel most of x_q)
    assert abs(g2) <= 4 * m * U53 * np.sqrt(a * b)
    # the rotated column norms are the exact singular values of [x_p, x_q],
    # to a relative error of the rounding in the rotation:
    # ||x_q||_old / ||x_q||_new u (large when the rotation cancels)
    ex = exact_sigma(x)
    amp = max(1.0, np.sqrt(b / min(a2, b2)))
    assert np.allclose(np.sqrt(np.sort([a2, b2])[::-1]), ex, rtol=8 * m * U53 * amp, atol=0)
    # exact update formulas alpha' = alpha - t gamma, beta' = beta + t gamma
    t = s / c
    assert abs(a2 - (a - t * g)) <= 8 * m * U53 * max(a, abs(t * g))
    assert abs(b2 - (b + t * g)) <= 8 * m * U53 * max(b, abs(t * g))


def test_rotation_equal_norms_is_45_degrees():
    # alpha = beta gives zeta = 0, sign(0) = +1, t = 1: a 45-degree rotation
    c, s = oracle.rotation(2.0, 2.0, 0.5)
    assert np.isclose(c, 1 / np.sqrt(2), rtol=1e-15) and np.isclose(s, 1 / np.sqrt(2), rtol=1e-15)
    c, s = oracle.rotation(2.0, 2.0, -0.5)
    assert np.isclose(s, 1 / np.sqrt(2), rtol=1e-15)


# --------------------------------------------------------------------------
# Householder QR, QRCP, apply-Q (Sections 2.2 and 3.1)
# --------------------------------------------------------------------------
def unpack_r(F):
    n = F.shape[1]
    return np.triu(F[:n, :])


@pytest.mark.parametrize("shape", [(40, 40), (70, 30), (33, 1), (5, 5)])
def test_geqr2_matches_lapack_and_is_backward_stable(shape):
    rng = np.random.default_rng(11)
    A = rng.standard_normal(shape) * 10.0 ** rng.uniform(-3, 3, shape[1])
    F, tau = oracle.geqr2(A)
    R = unpack_r(F)
    Q = oracle.form_q(F, tau)
    m, n = shape
    # same sign convention as LAPACK's dgeqrf (beta = -sign(alpha) ||x||)
    Rl = np.linalg.qr(A, mode="r")
    assert np.allclose(R, Rl, rtol=1e-12, atol=1e-13 * np.abs(Rl).max())
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) < 10 * m * U53
    # columnwise backward stability (eq. RRQR-error): ||(A - QR)(:, i)|| <= c n u ||A(:, i)||
    col = np.linalg.norm(A - Q @ R, axis=0) / np.linalg.norm(A, axis=0)
    assert col.max() < 10 * m * U53


def test_apply_q_transpose_is_inverse():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((30, 20))
    F, tau = oracle.geqr2(A)
    C = rng.standard_normal((30, 7))
    C1 = oracle.apply_q(F, tau, C, trans=False)
    C2 = oracle.apply_q(F, tau, C1, trans=True)
    assert np.allclose(C2, C, atol=1e-13)
    Q = oracle.form_q(F, tau, 30)
    assert np.allclose(Q @ C, C1, atol=1e-13)
    assert np.allclose(Q.T @ C, oracle.apply_q(F, tau, C, trans=True), atol=1e-13)


def test_geqp3_pivot_property_and_lapack_pivots():
    # strongly graded columns: the pivot order is well separated (no near ties)
    rng = np.random.default_rng(5)
    n = 24
    A = rng.standard_normal((n, n)) * 10.0 ** (-rng.permutation(n) * 0.5)
    F, jpvt, tau = oracle.geqp3(A)
    R = unpack_r(F)
    # Businger-Golub property: |r_kk| >= ||R(k:j, j)|| for every j > k
    for k in range(n):
        for j in range(k + 1, n):
            assert abs(R[k, k]) >= np.linalg.norm(R[k:j + 1, j]) * (1 - 1e-12)
    # |r_kk| non-increasing
    d = np.abs(np.diag(R))
    assert np.all(d[:-1] >= d[1:] * (1 - 1e-12))
    Q = oracle.form_q(F, tau)
    assert np.allclose(Q @ R, A[:, jpvt], atol=1e-14 * np.abs(A).max())
    # independent implementation: LAPACK dgeqp3 picks the same columns here
    _, _, p = scipy.linalg.qr(A, pivoting=True)
    assert np.array_equal(jpvt, p)


def test_geqp3_ties_go_to_lowest_original_index():
    A = np.eye(6)
    _, jpvt, _ = oracle.geqp3(A)
    assert list(jpvt) == list(range(6))


# --------------------------------------------------------------------------
# Algorithm 1 sweeps
# --------------------------------------------------------------------------
def test_round_robin_schedule_is_a_perfect_tournament():
    for n in (2, 3, 8, 9, 16):
        nn = n + (n & 1)
        seen = set()
        for r in range(nn - 1):
            used = set()
            for k in range(nn // 2):
                p, q = oracle.rr_pair(n, r, k)
                if p < 0:
                    continue
                assert 0 <= p < q < n
                assert p not in used and q not in used
                used |= {p, q}
                seen.add((p, q))
        assert len(seen) == n * (n - 1) // 2


@pytest.mark.parametrize("order", ["cyclic", "rr"])
def test_gesvj_converges_and_accumulates_v(order):
    rng = np.random.default_rng(9)
    X0 = rng.standard_normal((40, 25))
    X, V, st, sw = oracle.gesvj(X0, np.eye(25), order=order)
    assert st == 0 and 3 <= sw <= 20
    G = X.T @ X
    d = np.sqrt(np.diag(G))
    off = np.abs(G / np.outer(d, d) - np.eye(25)).max()
    assert off <= np.sqrt(40) * U53 * 4
    assert np.allclose(X0 @ V, X, atol=1e-13 * np.abs(X0).max())
    assert np.linalg.norm(V.T @ V - np.eye(25)) < 1e-13


def test_gesvj_maxiter_reports_noconv():
    rng = np.random.default_rng(1)
    _, _, st, sw = oracle.gesvj(rng.standard_normal((20, 20)), maxiter=1)
    assert st == 1 and sw == 1


def test_finalize_sorts_stably_and_normalises():
    X = np.asfortranarray(np.diag([1.0, 3.0, 3.0, 2.0]))
    V = np.eye(4, order="F")
    U, S, V2, z = oracle.finalize(X, V)
    assert list(S) == [3.0, 3.0, 2.0, 1.0] and z == 0
    # equal values keep their original order: columns 1 then 2
    assert np.array_equal(V2[:, 0], np.eye(4)[:, 1]) and np.array_equal(V2[:, 1], np.eye(4)[:, 2])
    assert np.allclose(np.abs(U), np.abs(V2))


def test_sign_rule():
    U = np.eye(3)
    V = np.array([[0.1, 0.0, 0.0], [-0.9, 1.0, 0.0], [0.0, 0.0, -1.0]])
    U2, V2 = oracle.sign_normalize(U, V)
    assert V2[1, 0] > 0 and U2[0, 0] == -1.0 and V2[2, 2] == 1.0 and U2[2, 2] == -1.0


# --------------------------------------------------------------------------
# Whole SVD
# --------------------------------------------------------------------------
@pytest.mark.parametrize("shape,seed", [((8, 8), 0), ((12, 7), 1), ((16, 16), 2), ((24, 24), 3)])
def test_svd_matches_exact_sigma_of_stored_matrix(shape, seed):
    m, n = shape
    rng = np.random.default_rng(seed)
    u = testmats.haar(rng, m, n)
    v = testmats.haar(rng, n, n)
    s = testmats.sigma_geometric(n, 8.0)
    A = testmats.compose(u, s, v)
    ex = exact_sigma(A)
    for pre in (True, False):
        U, S, V, info = oracle.svd(A, precondition=pre)
        assert info["status"] == 0
        g = metrics.gates(A, U, S, V, ex)
        assert g["pass"], g


@pytest.mark.parametrize("seed", range(3))
def test_svd_high_relative_accuracy_on_graded_matrix(seed):
    # A = B D with kappa(D) = 1e20: tiny singular values must keep their
    # relative accuracy (about u kappa(B)), which a normwise method loses.
    n = 12
    A = testmats.graded(seed, n, n, mode_sigma=3, kappa_b=10.0, mode_d=3, kappa_d=1e20)
    # unsorted column scales, as in the C2 construction
    A = np.asfortranarray(A[:, np.random.default_rng(seed).permutation(n)])
    ex = exact_sigma(A)
    U, S, V, info = oracle.svd(A)
    assert info["status"] == 0
    assert metrics.rel_sigma_err(S, ex) < 1e-13
    # the normwise LAPACK SVD loses the small ones
    sn = np.linalg.svd(A, compute_uv=False)
    assert metrics.rel_sigma_err(sn, ex) > 1e-6
    # columnwise backward error stays small even though columns span 1e20
    assert metrics.colwise_backward_err(A, U, S, V) < 1e-13


def test_svd_known_sigma_c1():
    A, s = testmats.config_c1()
    U, S, V, info = oracle.svd(A)
    assert info["status"] == 0
    g = metrics.gates(A, U, S, V, s)
    assert g["pass"], g


def test_svd_agrees_with_lapack_dgejsv():
    # LAPACK's DGEJSV is the paper's FP64 baseline (Algorithm 2).
    A = testmats.config_c2(n=160)[0]
    s_lap = dgejsv_sigma(A)
    U, S, V, _ = oracle.svd(A)
    ks = metrics.kappa_s(A)
    assert metrics.e_sigma(S, s_lap, ks) < 1e-13
    assert metrics.rel_sigma_err(S, s_lap) < 1e-10


def test_svd_power_of_two_scaling_is_exact():
    A, _ = testmats.config_c1(n=40)
    _, S1, _, _ = oracle.svd(A)
    _, S2, _, _ = oracle.svd(A * 2.0 ** 7)
    assert np.array_equal(S2, S1 * 2.0 ** 7)


def test_svd_column_permutation_invariance():
    # QRCP undoes a column permutation, so the result is bitwise the same
    A, _ = testmats.config_c1(n=40)
    perm = np.random.default_rng(0).permutation(40)
    U1, S1, V1, _ = oracle.svd(A)
    U2, S2, V2, _ = oracle.svd(A[:, perm])
    assert np.array_equal(S1, S2)
    assert np.allclose(V2, V1[perm, :], atol=1e-15)


def test_svd_cyclic_and_round_robin_agree():
    A = testmats.config_c3b(n=96)[0]
    _, S1, _, _ = oracle.svd(A, order="cyclic")
    U, S2, V, _ = oracle.svd(A, order="rr")
    assert metrics.e_sigma(S2, S1, metrics.kappa_s(A)) < 1e-13
    assert metrics.gates(A, U, S2, V, S1)["pass"]


def test_svd_tall_matrix():
    rng = np.random.default_rng(4)
    u = testmats.haar(rng, 90, 30)
    v = testmats.haar(rng, 30, 30)
    s = testmats.sigma_geometric(30, 10.0)
    A = testmats.compose(u, s, v)
    U, S, V, info = oracle.svd(A)
    assert U.shape == (90, 30) and info["status"] == 0
    assert metrics.gates(A, U, S, V, exact_sigma(A))["pass"]


def test_svd_rank_deficient_and_edge_sizes():
    A = np.zeros((5, 3), order="F")
    A[:, 0] = 1.0
    U, S, V, info = oracle.svd(A)
    assert info["status"] == 3
    assert np.isclose(S[0], np.sqrt(5)) and S[1] == 0 and S[2] == 0
    assert np.all(U[:, 1:] == 0)
    U, S, V, info = oracle.svd(np.array([[-3.0]]))
    assert S[0] == 3.0 and V[0, 0] == 1.0 and U[0, 0] == -1.0
    U, S, V, info = oracle.svd(np.zeros((4, 0)))
    assert S.size == 0


def test_svd_paper_accuracy_yardsticks_small_analogue():
    """Section 7.3: 16 matrix types of Table 1 with (kappa(D), kappa(B)) =
    (1e20, 1e2).  The paper reports, for its mixed algorithm at n = 1024, a
    maximum relative difference to DGEJSV of 4.79e-14 and a columnwise backward
    error of 3.21e-14; the FP64 oracle must stay within those figures on the
    same family (here at n = 64)."""
    with open(os.path.join(HERE, "golden", "paper_values.json")) as f:
        paper = json.load(f)
    y = paper["accuracy_experiment"]
    n = 64
    worst_rel, worst_bwd = 0.0, 0.0
    for i, (md, ms) in enumerate(paper["table1_modes"]):
        A = testmats.graded(100 + i, n, n, ms, y["kappa_B"], md, y["kappa_D"])
        U, S, V, info = oracle.svd(A)
        assert info["status"] == 0
        s_lap = dgejsv_sigma(A)
        worst_rel = max(worst_rel, metrics.rel_sigma_err(S, s_lap))
        worst_bwd = max(worst_bwd, metrics.colwise_backward_err(A, U, S, V))
    assert worst_rel <= y["max_rel_sigma_diff_vs_dgejsv"]
    assert worst_bwd <= y["max_colwise_backward_error"]


def test_tolerance_parameters_match_paper():
    with open(os.path.join(HERE, "golden", "paper_values.json")) as f:
        paper = json.load(f)
    p = paper["parameters"]
    assert p["tol_alg"] == 1e-2 and p["tol_orth"] == 1e-5 and p["tol_cond_coef"] == 1.5


# --------------------------------------------------------------------------
# SVD adjoint reference
# --------------------------------------------------------------------------
def _loss(A, gU, gs, gV):
    U, S, V, _ = oracle.svd(A)
    return np.sum(gU * U) + np.sum(gs * S) + np.sum(gV * V)


def test_adjoint_sigma_only_is_u_diag_v():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((9, 5))
    U, S, V, _ = oracle.svd(A)
    gs = rng.standard_normal(5)
    gA = oracle.svd_backward_ref(U, S, V, None, gs, None)
    assert np.allclose(gA, (U * gs) @ V.T, atol=1e-14)


def _mp_loss(A, gU, gs, gV, t, E):
    """L(A + t E) in high precision with the same sign rule as the oracle."""
    M = mpmath.matrix(A.tolist()) + t * mpmath.matrix(E.tolist())
    U, S, V = mpmath.svd_r(M)
    m, n = A.shape
    Vt = V  # mpmath returns V^T as V
    L = mpmath.mpf(0)
    order = sorted(range(n), key=lambda i: -S[i])
    for col, i in enumerate(order):
        vcol = [Vt[i, j] for j in range(n)]
        k = max(range(n), key=lambda j: abs(vcol[j]))
        sg = -1 if vcol[k] < 0 else 1
        L += gs[col] * S[i]
        for j in range(n):
            L += gV[j, col] * sg * vcol[j]
        for r in range(m):
            L += gU[r, col] * sg * U[r, i]
    return L


def test_adjoint_matches_high_precision_derivative():
    rng = np.random.default_rng(2)
    m, n = 6, 4
    A = testmats.compose(testmats.haar(rng, m, n), np.array([3.0, 2.0, 1.2, 0.5]), testmats.haar(rng, n, n))
    gU, gs, gV = rng.standard_normal((m, n)), rng.standard_normal(n), rng.standard_normal((n, n))
    E = rng.standard_normal((m, n))
    U, S, V, _ = oracle.svd(A)
    gA = oracle.svd_backward_ref(U, S, V, gU, gs, gV)
    with mpmath.workdps(40):
        d = mpmath.diff(lambda t: _mp_loss(A, gU, gs, gV, t, E), 0)
    assert abs(float(d) - np.sum(gA * E)) <= 1e-10 * max(1.0, abs(float(d)))


def test_adjoint_square_diagonal_by_hand():
    """A = diag(d), d distinct, positive and descending: U = V = I and S = d
    (the sign rule keeps the identity).  First-order perturbation of the SVD
    at a diagonal matrix (differentiate A = U S V^T with U^T dU and V^T dV
    antisymmetric): dS_i = E_ii, (U^T dU)_ij = (s_j E_ij + s_i E_ji) /
    (s_j^2 - s_i^2), (V^T dV)_ij = (s_i E_ij + s_j E_ji) / (s_j^2 - s_i^2).
    Collecting the coefficient of E_ij in <gU, dU> + <gs, dS> + <gV, dV>:
    gA_ii = gs_i and, for i != j,
    gA_ij = (s_j (gU_ij - gU_ji) + s_i (gV_ij - gV_ji)) / (s_j^2 - s_i^2)."""
    rng = np.random.default_rng(4)
    n = 5
    d = np.array([3.0, 2.0, 1.25, 0.75, 0.5])
    A = np.diag(d)
    U, S, V, _ = oracle.svd(A)
    assert np.array_equal(U, np.eye(n)) and np.array_equal(V, np.eye(n)) and np.array_equal(S, d)
    gU, gs, gV = rng.standard_normal((n, n)), rng.standard_normal(n), rng.standard_normal((n, n))
    gA = oracle.svd_backward_ref(U, S, V, gU, gs, gV)
    hand = np.diag(gs).astype(np.float64)
    for i in range(n):
        for j in range(n):
            if i != j:
                hand[i, j] = (d[j] * (gU[i, j] - gU[j, i]) + d[i] * (gV[i, j] - gV[j, i])) / (d[j] ** 2 - d[i] ** 2)
    assert np.allclose(gA, hand, rtol=1e-12, atol=1e-14), np.max(np.abs(gA - hand))


def test_adjoint_degenerate_pair_with_gauge_invariant_cotangents():
    """sigma_1 = sigma_2 exactly: U and V are defined only up to a rotation
    of that pair, and a loss through U M and V N with M, N symmetric does not
    see the rotation (U^T gU - gU^T U = M - M^T = 0).  Its gradient is
    U diag(gs) V^T; the guard on 1 / (s_j^2 - s_i^2) must give that instead
    of 0 * inf."""
    rng = np.random.default_rng(6)
    n = 6
    s = np.array([2.0, 2.0, 1.5, 1.0, 0.6, 0.3])
    A = testmats.compose(testmats.haar(rng, n, n), s, testmats.haar(rng, n, n))
    U, S, V, _ = oracle.svd(A)
    M = rng.standard_normal((n, n)); M = M + M.T
    N = rng.standard_normal((n, n)); N = N + N.T
    gs = rng.standard_normal(n)
    gA = oracle.svd_backward_ref(U, S, V, U @ M, gs, V @ N)
    assert np.all(np.isfinite(gA))
    assert np.allclose(gA, (U * gs) @ V.T, atol=1e-12)


def test_adjoint_central_differences_on_c5_shape():
    data = testmats.config_c5(batch=2, ndir=4)
    for b in range(2):
        A = data["A"][b]
        U, S, V, _ = oracle.svd(A)
        gA = oracle.svd_backward_ref(U, S, V, data["gU"][b], data["gS"][b], data["gV"][b])
        h = 1e-6
        for E in data["E"][b]:
            lp = _loss(A + h * E, data["gU"][b], data["gS"][b], data["gV"][b])
            lm = _loss(A - h * E, data["gU"][b], data["gS"][b], data["gV"][b])
            fd = (lp - lm) / (2 * h)
            an = np.sum(gA * E)
            assert abs(fd - an) <= 1e-5 * max(1.0, abs(an)), (fd, an)


# ---------------------------------------------------------------------------
# Symmetric eigendecomposition (cyclic two-sided Jacobi, the oracle of the
# eigensolver of Section 8)
# ---------------------------------------------------------------------------

def exact_eig(A, dps=60):
    """Eigenvalues of the stored symmetric FP64 matrix A in 60-digit arithmetic,
    ascending."""
    with mpmath.workdps(dps):
        E = mpmath.eigsy(mpmath.matrix(A.tolist()), eigvals_only=True)
        return np.array(sorted(float(x) for x in E))


@pytest.mark.parametrize("a,b,c", [(2.0, 1.0, -1.0), (1.0, 1e-9, 1.0), (0.0, 3.0, 0.0),
                                   (-5.0, 2.0, 7.0), (1e-8, 1e-12, 2e-8)])
def test_eig_2x2_closed_form(a, b, c):
    """[[a, b], [b, c]]: eigenvalues (a + c)/2 -+ sqrt(((a - c)/2)^2 + b^2),
    evaluated at 50 digits; X diagonalises A."""
    A = np.array([[a, b], [b, c]])
    w, X, info = oracle.eigh(A)
    assert info["status"] == 0
    with mpmath.workdps(50):
        m = (mpmath.mpf(a) + c) / 2
        r = mpmath.sqrt(((mpmath.mpf(a) - c) / 2) ** 2 + mpmath.mpf(b) ** 2)
        ref = np.array([float(m - r), float(m + r)])
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(w - ref)) <= 4 * U53 * scale
    D = X.T @ A @ X
    assert abs(D[0, 1]) <= 4 * U53 * scale
    assert np.linalg.norm(X.T @ X - np.eye(2)) <= 4 * U53


def test_eig_diagonal_is_exact_permutation():
    """A diagonal matrix needs no rotation: w is its sorted diagonal exactly and
    X the matching permutation."""
    rng = np.random.default_rng(3)
    d = rng.standard_normal(17)
    w, X, info = oracle.eigh(np.diag(d))
    assert info["sweeps"] == 1 and np.array_equal(w, np.sort(d))
    assert np.array_equal(X, np.eye(17)[:, np.argsort(d, kind="stable")])


@pytest.mark.parametrize("seed", [0, 1])
def test_eig_known_spectrum_with_plus_minus_pairs(seed):
    """A = Q diag(lam) Q^T with Haar Q, lam indefinite with +-pairs of equal
    magnitude and a double eigenvalue: eigenvalues to normwise backward
    accuracy, residual, orthogonality."""
    rng = np.random.default_rng(seed)
    n = 40
    mag = 10.0 ** -rng.uniform(0, 6, n)
    lam = mag * np.where(rng.random(n) < 0.5, -1.0, 1.0)
    lam[1] = -lam[0]
    lam[5] = -lam[4]
    lam[9] = lam[8]
    Q = testmats.haar(rng, n, n)
    A = (Q * lam) @ Q.T
    A = (A + A.T) / 2
    w, X, info = oracle.eigh(A)
    assert info["status"] == 0
    nA = np.linalg.norm(A, 2)
    assert np.max(np.abs(w - np.sort(lam))) <= 50 * n * U53 * nA
    assert np.linalg.norm(A @ X - X * w) <= 50 * n * U53 * np.linalg.norm(A)
    assert np.linalg.norm(X.T @ X - np.eye(n)) <= 50 * n * U53


def test_eig_matches_lapack_and_invariants():
    """Against LAPACK (numpy eigh) normwise; trace and Frobenius norm kept."""
    rng = np.random.default_rng(11)
    n = 33
    B = rng.standard_normal((n, n))
    A = (B + B.T) / 2
    w, X, info = oracle.eigh(A)
    nA = np.linalg.norm(A, 2)
    assert np.max(np.abs(w - np.linalg.eigvalsh(A))) <= 20 * n * U53 * nA
    assert abs(w.sum() - np.trace(A)) <= 10 * n * U53 * nA
    assert abs((w ** 2).sum() - np.linalg.norm(A) ** 2) <= 20 * n * U53 * np.linalg.norm(A) ** 2


@pytest.mark.parametrize("seed", [4, 5])
def test_eig_relative_accuracy_on_graded_definite(seed):
    """A = D H D, H well-conditioned positive definite, D graded over 10 orders:
    Jacobi with the relative test keeps every eigenvalue to high relative
    accuracy (60-digit reference of the stored matrix), where normwise methods
    lose the small ones."""
    rng = np.random.default_rng(seed)
    n = 12
    G = rng.standard_normal((n, n))
    H = G @ G.T / n + np.eye(n)
    d = 10.0 ** -rng.uniform(0, 10, n)
    A = (H * d).T * d
    A = (A + A.T) / 2
    w, X, info = oracle.eigh(A)
    ref = exact_eig(A)
    assert np.max(np.abs(w - ref) / np.abs(ref)) <= 1e-13
