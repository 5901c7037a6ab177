"""GPU parity: svd_plain / svd_mixed through the C ABI against the FP64 oracle.

Gates (on every case): e_sigma <= 1e-13 against the oracle's sigma on the same
stored matrix, ||U^T U - I||_F and ||V^T V - I||_F <= 1e-13 n,
||A - U S V^T||_F / ||A||_F <= 1e-14 n.  Sizes span several 64-column tiles
with ragged tails; the Jacobi ordering differs from the oracle's, so the
comparison is tolerance-based, never bitwise.
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


def known(m, n, seed, e=8.0, kind="geo"):
    rng = np.random.default_rng(seed)
    u = testmats.haar(rng, m, n)
    v = testmats.haar(rng, n, n)
    s = testmats.sigma_geometric(n, e) if kind == "geo" else testmats.sigma_log_uniform(rng, n, e)
    return testmats.compose(u, s, v)


CASES = [(1, 1), (2, 2), (5, 3), (16, 16), (33, 33), (64, 64), (100, 70), (130, 130), (200, 97)]


@pytest.mark.parametrize("mode", ["plain", "mixed"])
@pytest.mark.parametrize("shape", CASES)
def test_parity_small(lib, mode, shape):
    m, n = shape
    print(f"case mode={mode} shape={shape}", flush=True)
    A = known(m, n, seed=m * 1000 + n)
    Uo, So, Vo, io = oracle.svd(A)
    U, S, V, info = run(lib, A, mode)
    assert info["status"] == 0, info
    g = metrics.gates(A, U, S, V, So)
    assert g["pass"], (g, info)
    # sign rule agrees with the oracle's: compare vectors of well separated sigma
    gap = np.ones(n)
    if n > 1:
        rel = np.abs(np.diff(So)) / So[:-1]
        gap[:-1] = np.minimum(gap[:-1], rel)
        gap[1:] = np.minimum(gap[1:], rel)
    sep = gap > 1e-3
    if sep.any():
        assert np.max(np.abs(V[:, sep] - Vo[:, sep])) < 1e-8


@pytest.mark.parametrize("mode", ["plain", "mixed"])
def test_c1_config(lib, mode):
    A, s = testmats.config_c1()
    Uo, So, Vo, _ = oracle.svd(A)
    U, S, V, info = run(lib, A, mode)
    g = metrics.gates(A, U, S, V, So)
    assert info["status"] == 0 and g["pass"], (g, info)


@pytest.mark.parametrize("b_low,b_work", [(16, 16), (16, 32), (32, 16), (32, 32)])
def test_parity_block_widths(lib, b_low, b_work):
    """Every Jacobi block-width choice the tuning table may select (both
    stages) meets the gates: 300 x 300, five 64-column tiles with a ragged
    tail, log-uniform sigma over 10 decades."""
    print(f"case b_low={b_low} b_work={b_work}", flush=True)
    A = known(300, 300, seed=31, e=10.0, kind="log")
    Uo, So, Vo, _ = oracle.svd(A)
    for mode in ("mixed", "plain"):
        U, S, V, info = run(lib, A, mode, block_cols_low=b_low, block_cols_work=b_work)
        g = metrics.gates(A, U, S, V, So)
        assert info["status"] == 0 and g["pass"], (mode, g, info)


@pytest.mark.parametrize("mode", ["plain", "mixed"])
@pytest.mark.parametrize("inner_pairs", [0, 1])
def test_parity_inner_pairs(lib, mode, inner_pairs):
    """Both inner schedules of a block pair (all 2b columns every round, or
    only the pairs between the two blocks after a sweep's first round) meet
    the gates on a ragged size."""
    print(f"case inner_pairs={inner_pairs} mode={mode}", flush=True)
    A = known(330, 330, seed=91, e=10.0, kind="log")
    Uo, So, Vo, _ = oracle.svd(A)
    U, S, V, info = run(lib, A, mode, inner_pairs=inner_pairs)
    g = metrics.gates(A, U, S, V, So)
    assert info["status"] == 0 and g["pass"], (g, info)


@pytest.mark.parametrize("shape", [(300, 300), (200, 97)])
def test_parity_switch_method_2(lib, shape):
    """The switch through the QR of the accumulated FP32 V (method 2) meets
    the gates with the FP32 stage taken."""
    m, n = shape
    print(f"case switch_method=2 shape={shape}", flush=True)
    A = known(m, n, seed=41 + m, e=10.0, kind="log")
    Uo, So, Vo, _ = oracle.svd(A)
    U, S, V, info = run(lib, A, "mixed", switch_method=2, branch=1)
    g = metrics.gates(A, U, S, V, So)
    assert info["status"] == 0 and info["branch_taken"] == 1 and g["pass"], (g, info)
    U1, S1, V1, info1 = run(lib, A, "mixed", switch_method=1, branch=1)
    assert np.max(np.abs(S - S1) / S1) < 1e-12


@pytest.mark.parametrize("shape", [(300, 300), (200, 97)])
def test_parity_algorithm_3(lib, shape):
    """Algorithm 3 (switch_method = 3): the FP64 sweeps run on A1 Q with Q
    from the FP32 right vectors, V accumulated; it meets the gates, and its
    refinement takes at least as many sweeps as Algorithm 4's (Section 6)."""
    m, n = shape
    print(f"case switch_method=3 shape={shape}", flush=True)
    A = known(m, n, seed=43 + m, e=10.0, kind="log")
    Uo, So, Vo, _ = oracle.svd(A)
    U, S, V, info = run(lib, A, "mixed", switch_method=3, branch=1, diagnostics=1)
    g = metrics.gates(A, U, S, V, So)
    assert info["status"] == 0 and info["branch_taken"] == 1 and g["pass"], (g, info)
    assert info["v_method_taken"] == 0, info
    U1, S1, V1, info1 = run(lib, A, "mixed", switch_method=1, branch=1, diagnostics=1)
    assert info["sweeps_work"] >= info1["sweeps_work"], (info["sweeps_work"], info1["sweeps_work"])


def test_parity_tall_panel_fallback(lib):
    """66000 x 32: the tall QR's panels span more than 256 row groups, so the
    per-column panel launches (not the one-launch panel) factor them."""
    print("case tall 66000x32", flush=True)
    A = known(66000, 32, seed=7, e=6.0)
    Uo, So, Vo, _ = oracle.svd(A)
    for mode in ("mixed", "plain"):
        U, S, V, info = run(lib, A, mode)
        g = metrics.gates(A, U, S, V, So)
        assert info["status"] == 0 and g["pass"], (mode, g, info)


def test_large_n_pivot_step_fallback(lib):
    """n = 4160 > 4096: the pivot pass takes the step-by-step kernels (the
    one-launch pass holds at most 4096 rows per column in registers).  sigma
    geometric in [1e-3, 1], so the constructed sigma are exact to ~1e-13 and
    stand in for the oracle's; orthogonality and residual gates as always."""
    import torch
    n = 4160
    print(f"case square n={n}", flush=True)
    rng = np.random.default_rng(4160)
    s = testmats.sigma_geometric(n, 3.0)
    A = testmats.compose(testmats.haar(rng, n, n), s, testmats.haar(rng, n, n))
    At = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    eye = torch.eye(n, dtype=torch.float64, device="cuda")
    for mode in ("mixed", "plain"):
        U, S, V, info = lib.svd(At, mode, branch=1 if mode == "mixed" else 0)
        torch.cuda.synchronize()
        assert info["status"] == 0, info
        orth_u = torch.linalg.norm(U.t() @ U - eye).item()
        orth_v = torch.linalg.norm(V.t() @ V - eye).item()
        res = (torch.linalg.norm(At - (U * S) @ V.t()) / torch.linalg.norm(At)).item()
        rel = np.max(np.abs(S.cpu().numpy() - s) / s)
        assert orth_u <= 1e-13 * n and orth_v <= 1e-13 * n and res <= 1e-14 * n, (mode, orth_u, orth_v, res)
        assert rel < 1e-11, (mode, rel)


def test_gram_chunks_not_multiple_of_256(lib):
    """n = 1344: the Gram kernels take row chunks of N/4 = 320 rows (five
    64-row stripes over four wavefronts, ten 32-row FP64 stripes) and a last
    chunk of 64 rows.  sigma geometric in [1e-3, 1] stands in for the
    oracle's, as in the n = 4160 case."""
    import torch
    n = 1344
    print(f"case square n={n}", flush=True)
    rng = np.random.default_rng(1344)
    s = testmats.sigma_geometric(n, 3.0)
    A = testmats.compose(testmats.haar(rng, n, n), s, testmats.haar(rng, n, n))
    At = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    eye = torch.eye(n, dtype=torch.float64, device="cuda")
    for mode in ("mixed", "plain"):
        U, S, V, info = lib.svd(At, mode, branch=1 if mode == "mixed" else 0)
        torch.cuda.synchronize()
        assert info["status"] == 0, info
        orth_u = torch.linalg.norm(U.t() @ U - eye).item()
        orth_v = torch.linalg.norm(V.t() @ V - eye).item()
        res = (torch.linalg.norm(At - (U * S) @ V.t()) / torch.linalg.norm(At)).item()
        rel = np.max(np.abs(S.cpu().numpy() - s) / s)
        assert orth_u <= 1e-13 * n and orth_v <= 1e-13 * n and res <= 1e-14 * n, (mode, orth_u, orth_v, res)
        assert rel < 1e-11, (mode, rel)


def test_tall_ragged_large(lib):
    """5000 x 2100: a tall QR whose panels, in-block updates and 128 x 128
    GEMM tiles all end in partial tiles (5000 and 2100 are not multiples of
    64 or 128), the fused FP32 round on a padded 2112-column Y, and the
    switch's product on ragged tiles.  sigma geometric in [1e-3, 1] stands in
    for the oracle's, as in the n = 4160 case."""
    import torch
    m, n = 5000, 2100
    print(f"case tall m={m} n={n}", flush=True)
    rng = np.random.default_rng(5021)
    s = testmats.sigma_geometric(n, 3.0)
    A = testmats.compose(testmats.haar(rng, m, n), s, testmats.haar(rng, n, n))
    At = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    eye = torch.eye(n, dtype=torch.float64, device="cuda")
    for mode in ("mixed", "plain"):
        U, S, V, info = lib.svd(At, mode, branch=1 if mode == "mixed" else 0, fused_rounds=1)
        torch.cuda.synchronize()
        assert info["status"] == 0, info
        orth_u = torch.linalg.norm(U.t() @ U - eye).item()
        orth_v = torch.linalg.norm(V.t() @ V - eye).item()
        res = (torch.linalg.norm(At - (U * S) @ V.t()) / torch.linalg.norm(At)).item()
        rel = np.max(np.abs(S.cpu().numpy() - s) / s)
        print(mode, {"orth_u": orth_u, "orth_v": orth_v, "res": res, "rel": rel}, flush=True)
        assert orth_u <= 1e-13 * n and orth_v <= 1e-13 * n and res <= 1e-14 * n, (mode, orth_u, orth_v, res)
        assert rel < 1e-11, (mode, rel)


def graded(m, n, seed, e=8.0, d=4.0):
    """A = B diag(10^w), w ~ U(-d, 0): badly scaled columns over a B with
    log-uniform sigma (the A = B D family)."""
    rng = np.random.default_rng(seed)
    B = testmats.compose(testmats.haar(rng, m, n), testmats.sigma_log_uniform(rng, n, e),
                         testmats.haar(rng, n, n))
    return B * (10.0 ** rng.uniform(-d, 0.0, n))[None, :]


@pytest.mark.parametrize("mode", ["plain", "mixed"])
@pytest.mark.parametrize("case", ["square", "tall", "graded"])
def test_parity_v_solve(lib, mode, case):
    """V_X = X^{-1} Y by the triangular solve (Section 3.4) after FP64 sweeps
    without V: accepted on these preconditioned inputs and within the gates;
    sigma agree with the accumulated path's."""
    print(f"case v_method=1 mode={mode} {case}", flush=True)
    if case == "square":
        A = known(300, 300, seed=77, e=10.0, kind="log")
    elif case == "tall":
        A = known(200, 97, seed=78, e=10.0, kind="log")
    else:
        A = graded(260, 260, seed=79)
    Uo, So, Vo, _ = oracle.svd(A)
    U, S, V, info = run(lib, A, mode, v_method=1)
    g = metrics.gates(A, U, S, V, So)
    assert info["status"] == 0 and g["pass"], (g, info)
    assert info["v_method_taken"] == 1 and 0.0 <= info["orth_vx"] <= A.shape[1] * 2.0 ** -50, info
    U0, S0, V0, info0 = run(lib, A, mode, v_method=0)
    assert info0["v_method_taken"] == 0 and info0["orth_vx"] == -1.0
    assert np.max(np.abs(S - S0) / S0) < 1e-12


@pytest.mark.parametrize("mode", ["plain", "mixed"])
def test_v_solve_fallback(lib, mode):
    """A bound no solve can meet forces the other route of Section 3.4: V_X
    from the QR of X^T U_X, then FP64 sweeps with accumulation (one or two,
    the start being accurate)."""
    print(f"case v_method=1 fallback mode={mode}", flush=True)
    A = known(300, 300, seed=80, e=10.0, kind="log")
    Uo, So, Vo, _ = oracle.svd(A)
    U, S, V, info = run(lib, A, mode, v_method=1, tol_vsolve=1e-300)
    g = metrics.gates(A, U, S, V, So)
    assert info["status"] == 0 and g["pass"], (g, info)
    assert info["v_method_taken"] == 2 and 1 <= info["sweeps_vfix"] <= 3, info


def test_v_not_wanted(lib):
    """want_v = 0: no V work and no V output is touched."""
    import torch
    A = known(120, 90, seed=81)
    At = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    U, S, V, info = lib.svd(At, "mixed", want_v=0)
    torch.cuda.synchronize()
    So = oracle.svd(A)[1]
    assert info["v_method_taken"] == -1 and info["orth_vx"] == -1.0
    e = metrics.e_sigma(S.cpu().numpy(), So, metrics.kappa_s(A))
    assert e <= 1e-13, e
    assert metrics.orth_err(U.cpu().numpy()) <= 1e-13 * A.shape[1]


@pytest.mark.parametrize("method", [1, 2])
def test_orthogonality_of_y_after_switch(lib, method):
    """Diagnostics: how orthogonal Y is when the FP64 sweeps start, for both
    switch methods (Section 6 compares them).  Either way the FP32 stage has
    left its columns orthogonal to a few units of FP32 rounding, far from the
    O(1) of the unswitched X."""
    print(f"case orth_y switch_method={method}", flush=True)
    A = known(256, 256, seed=82, e=10.0, kind="log")
    U, S, V, info = run(lib, A, "mixed", branch=1, switch_method=method, diagnostics=1)
    assert info["status"] == 0 and info["branch_taken"] == 1
    assert 0.0 < info["orth_y"] < 1e-3, info
    U, S, V, info_x = run(lib, A, "plain", diagnostics=1)
    assert info_x["orth_y"] > 100 * info["orth_y"], (info_x, info)   # X itself


@pytest.mark.parametrize("v_method", [0, 1])
def test_y2_safeguard(lib, v_method):
    """Section 3.4's safeguard: by default it finds no badly orthogonal columns
    after the switch (Y2 empty); with the bound lowered it sweeps Y2 alone
    first (a part of the columns, then all of them) and the result still
    meets the gates."""
    print(f"case y2 safeguard v_method={v_method}", flush=True)
    A = known(300, 300, seed=95, e=10.0, kind="log")
    Uo, So, Vo, _ = oracle.svd(A)
    U, S, V, info = run(lib, A, "mixed", branch=1, diagnostics=1, v_method=v_method)
    assert info["status"] == 0 and info["n_y2"] == 0 and info["orth_y"] > 0, info
    for tol in (info["orth_y"] / 3, 1e-300):
        U, S, V, info2 = run(lib, A, "mixed", branch=1, tol_y2=tol, v_method=v_method)
        g = metrics.gates(A, U, S, V, So)
        assert info2["status"] == 0 and g["pass"], (tol, g, info2)
        assert info2["n_y2"] >= 2 and info2["sweeps_y2"] >= 1, info2
    assert info2["n_y2"] == 300
