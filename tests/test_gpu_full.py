"""Full-size GPU parity, in the configuration bench.py times (default
options): the 1024^2 graded matrix, the 8192 x 2048 tall matrix and the
4096^2 matrix against the oracle's stored sigma (tests/golden, written by a
script that calls only the oracle), and the 2000-matrix ragged batch with
invariants on every matrix and the oracle on a sample."""
import os
import sys

import numpy as np
import pytest

import oracle
import testmats
from testmats import metrics

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
from make_oracle_sigma import fingerprint, load  # noqa: E402

GEN = {"C2": testmats.config_c2, "C3a": testmats.config_c3a, "C3b": testmats.config_c3b}


def gpu_gates(lib, A, mode):
    import torch
    At = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    U, S, V, info = lib.svd(At, mode)
    n = A.shape[1]
    eye = torch.eye(n, dtype=torch.float64, device="cuda")
    r = {
        "orth_u": torch.linalg.norm(U.t() @ U - eye).item(),
        "orth_v": torch.linalg.norm(V.t() @ V - eye).item(),
        "residual": (torch.linalg.norm(At - (U * S) @ V.t()) / torch.linalg.norm(At)).item(),
    }
    return S.cpu().numpy(), r, info


@pytest.mark.parametrize("mode", ["mixed", "plain"])
@pytest.mark.parametrize("name", ["C2", "C3a", "C3b"])
def test_full_size_against_stored_oracle_sigma(lib, name, mode):
    print(f"case {name} {mode}", flush=True)
    s_ref, kappa, fp, _ = load(name)
    A, _ = GEN[name]()
    # same seeded input up to the host's BLAS rounding
    assert np.allclose(fingerprint(A), fp, rtol=1e-12, atol=0)
    S, r, info = gpu_gates(lib, A, mode)
    n = A.shape[1]
    assert info["status"] == 0, info
    e = metrics.e_sigma(S, s_ref, kappa)
    print(name, mode, "e_sigma %.2e rel %.2e" % (e, metrics.rel_sigma_err(S, s_ref)), r, flush=True)
    assert e <= 1e-13
    assert r["orth_u"] <= 1e-13 * n and r["orth_v"] <= 1e-13 * n
    assert r["residual"] <= 1e-14 * n
    if mode == "mixed" and name != "C2":
        assert info["branch_taken"] == lib.BRANCH_LOW


def test_full_batch_c4(lib):
    import torch
    print("case C4 full batch", flush=True)
    shapes, mats, _ = testmats.config_c4()
    plan = lib.batched_plan(shapes)
    A = lib.pack_batch(mats, "cuda")
    S, U, V, info = lib.svd_batched(plan, A)
    torch.cuda.synchronize()
    info = info.cpu().numpy()
    assert np.all(info[:, 0] == 0)
    outs = lib.unpack_batch(plan, S, U, V)
    worst = {"orth_u": 0.0, "orth_v": 0.0, "residual": 0.0}
    rng = np.random.default_rng(0)
    sample = set(rng.choice(len(mats), 24, replace=False).tolist())
    for j, ((u, s, v), M) in enumerate(zip(outs, mats)):
        u, s, v = u.cpu().numpy(), s.cpu().numpy(), v.cpu().numpy()
        n = M.shape[1]
        ou, ov, res = metrics.orth_err(u), metrics.orth_err(v), metrics.residual(M, u, s, v)
        assert ou <= 1e-13 * n and ov <= 1e-13 * n and res <= 1e-14 * n, (j, shapes[j])
        assert np.all(np.diff(s) <= 0) and np.all(s >= 0)
        if j in sample:
            _, So, _, _ = oracle.svd(M)
            assert metrics.e_sigma(s, So, metrics.kappa_s(M)) <= 1e-13, (j, shapes[j])
