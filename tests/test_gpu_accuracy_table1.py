"""The paper's accuracy experiment on the GPU (Section 7.3): the 16 matrix
types of Table 1 (pairs of XLATM1 modes for D and Sigma) at n = 1024 with
(kappa(D), kappa(B)) = (1e20, 1e2), through svd_mixed and svd_plain.

kappa_s of these matrices is about kappa(B), so the sigma gate is sharp here
(relative error <= 1e-13 kappa_s), and the column norms reach 1e-20: the FP32
copies (pivot pass and FP32 Jacobi stage) would square them below the FP32
range without the power-of-two scaling of the library.  Gates against the
oracle on the same stored matrix: e_sigma <= 1e-13 (oracle sigma),
||U^T U - I||_F and ||V^T V - I||_F <= 1e-13 n, and a columnwise backward
error no worse than twice the oracle's own (or 1e-13 when that is larger).
The oracle, plain FP64 one-sided Jacobi, reaches 3.4e-13 on type 2 (eleven
sweeps on a matrix with one large column), so a fixed 1e-13 would fail the
definition of the result itself; Proposition 1 asks for the accuracy of FP64
Jacobi, which is what the relative gate states.  The paper's printed maxima
(Section 7.3, its mixed algorithm against DGEJSV on the same family) are
printed beside the measured values as yardsticks.
"""
import concurrent.futures as cf
import json
import os

import numpy as np
import pytest

import oracle
import testmats
from testmats import metrics

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
N = 1024


def family():
    with open(os.path.join(HERE, "golden", "paper_values.json")) as f:
        paper = json.load(f)
    y = paper["accuracy_experiment"]
    mats = [testmats.graded(100 + i, N, N, ms, y["kappa_B"], md, y["kappa_D"])
            for i, (md, ms) in enumerate(paper["table1_modes"])]
    return mats, y


@pytest.fixture(scope="module")
def table1():
    mats, y = family()
    # the oracle runs single-threaded (cyclic order); the 16 matrices run side
    # by side on the host's cores (ctypes releases the interpreter lock)
    oracle.set_threads(1)

    def ref(A):
        U, S, V, _ = oracle.svd(A)
        return S, metrics.colwise_backward_err(A, U, S, V)

    with cf.ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        out = list(ex.map(ref, mats))
    sref = [o[0] for o in out]
    cwref = [o[1] for o in out]
    ks = [metrics.kappa_s(A) for A in mats]
    return mats, sref, cwref, ks, y


@pytest.mark.parametrize("mode", ["mixed", "plain"])
def test_table1_family_accuracy(lib, table1, mode):
    import torch
    mats, sref, cwref, ks, y = table1
    worst = {"rel_sigma": 0.0, "e_sigma": 0.0, "colwise": 0.0, "orth_u": 0.0, "orth_v": 0.0}
    branches, fails = [], []
    for i, A in enumerate(mats):
        print(f"case table1 type {i + 1} mode={mode}", flush=True)
        At = torch.from_numpy(np.ascontiguousarray(A)).cuda()
        U, S, V, info = lib.svd(At, mode)
        torch.cuda.synchronize()
        U, S, V = U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy()
        assert info["status"] == 0, (i, info)
        assert np.all(np.isfinite(S)) and np.all(np.isfinite(U)) and np.all(np.isfinite(V))
        rel = metrics.rel_sigma_err(S, sref[i])
        e = rel / max(1.0, ks[i])
        cw = metrics.colwise_backward_err(A, U, S, V)
        ou, ov = metrics.orth_err(U), metrics.orth_err(V)
        branches.append(info["branch_taken"])
        print(f"  type {i + 1}: kappa_s {ks[i]:.2e} rel_sigma {rel:.2e} colwise {cw:.2e} "
              f"(oracle {cwref[i]:.2e}) orth_u {ou:.2e} orth_v {ov:.2e} "
              f"branch {info['branch_taken']} sweeps {info['sweeps_low']}/{info['sweeps_work']}",
              flush=True)
        if not (e <= 1e-13 and cw <= max(2.0 * cwref[i], 1e-13) and ou <= 1e-13 * N
                and ov <= 1e-13 * N):
            fails.append(i + 1)
        for k, v in (("rel_sigma", rel), ("e_sigma", e), ("colwise", cw), ("orth_u", ou),
                     ("orth_v", ov)):
            worst[k] = max(worst[k], v)
    print(f"{mode}: worst {worst}; paper (mixed vs DGEJSV): rel_sigma "
          f"{y['max_rel_sigma_diff_vs_dgejsv']:.2e} colwise {y['max_colwise_backward_error']:.2e} "
          f"orth_u {y['max_orth_U_fro']:.2e} orth_v {y['max_orth_V_fro']:.2e}", flush=True)
    assert not fails, f"types outside the gates: {fails}"
    if mode == "mixed":
        # most types take the FP32 stage (MODE 1 of D leaves all but one
        # column below 2^-53 of the largest, which skips it)
        assert sum(b == lib.BRANCH_LOW for b in branches) >= 8, branches
