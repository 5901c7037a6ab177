"""GPU parity of the fused FP32 Jacobi round (Gram block, inner solve and
update of every block pair in one launch, the slot's rows split over several
workgroups that exchange partial Gram blocks), against the oracle.

- fused_rounds = 1 forces the fused round below its default size threshold,
  on square, tall and ragged sizes whose row splits give one to four
  workgroups per pair slot and one or two stripes per wavefront; the launch
  count of kernel class 9 shows the fused kernel ran.
- the graded 1024^2 matrix (column scaling over six orders) against its
  stored oracle sigma, fused.
- wait_polls = -1 makes the fused round's wait give up: the FP32 stage is run
  again with the separate kernels (info.fused_fallback) and the result still
  meets the gates (n = 256 keeps the Householder panels in one workgroup, so
  no other wait is involved).
- the three-precision variant (half_sweeps): the first FP32-stage sweeps with
  BF16 Gram products (and, with half_storage, a BF16 Y), then FP32, then
  FP64; the same gates
  against the oracle (Proposition 1: the low-precision stages change only the
  number of FP64 sweeps), eagerly and in the stream-ordered mode.
"""
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

ROUND32 = 9   # kernel class of the fused FP32 round
ROUND16 = 11  # the same round on BF16 storage


def run(lib, A, **kw):
    import torch
    At = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    U, S, V, info = lib.svd(At, "mixed", **kw)
    torch.cuda.synchronize()
    return U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy(), info


@pytest.mark.parametrize("shape", [(256, 256), (700, 640), (1000, 1000), (1300, 1090)])
def test_fused_round_parity(lib, shape):
    m, n = shape
    print(f"case fused round m={m} n={n}", flush=True)
    rng = np.random.default_rng(1000 + n)
    A = testmats.compose(testmats.haar(rng, m, n), testmats.sigma_log_uniform(rng, n, 8.0),
                         testmats.haar(rng, n, n))
    _, So, _, _ = oracle.svd(A)
    U, S, V, info = run(lib, A, fused_rounds=1, half_sweeps=0, branch=lib.BRANCH_LOW,
                        kernel_timing=100 + ROUND32)
    g = metrics.gates(A, U, S, V, So)
    print({k: g[k] for k in ("e_sigma", "orth_u", "orth_v", "residual")},
          {k: info[k] for k in ("status", "sweeps_low", "sweeps_work", "fused_fallback")},
          "fused launches", info["kern_calls"][ROUND32], flush=True)
    assert info["status"] == 0 and info["fused_fallback"] == 0, info
    assert info["kern_calls"][ROUND32] > 0
    assert info["sweeps_low"] >= 1
    assert g["pass"], g


def test_fused_round_graded_c2(lib):
    print("case fused round C2", flush=True)
    s_ref, kappa, fp, _ = load("C2")
    A, _ = testmats.config_c2()
    assert np.allclose(fingerprint(A), fp, rtol=1e-12, atol=0)
    U, S, V, info = run(lib, A, fused_rounds=1, half_sweeps=0, branch=lib.BRANCH_LOW,
                        kernel_timing=100 + ROUND32)
    n = A.shape[1]
    e = metrics.e_sigma(S, s_ref, kappa)
    print("e_sigma %.2e" % e, {k: info[k] for k in ("status", "sweeps_low", "sweeps_work")}, flush=True)
    assert info["status"] == 0 and info["kern_calls"][ROUND32] > 0, info
    assert e <= 1e-13
    assert metrics.orth_err(U) <= 1e-13 * n and metrics.orth_err(V) <= 1e-13 * n
    assert metrics.residual(A, U, S, V) <= 1e-14 * n


def test_fused_round_timeout_falls_back(lib):
    print("case fused round wait_polls=-1 n=256", flush=True)
    rng = np.random.default_rng(77)
    n = 256
    A = testmats.compose(testmats.haar(rng, n, n), testmats.sigma_log_uniform(rng, n, 6.0),
                         testmats.haar(rng, n, n))
    _, So, _, _ = oracle.svd(A)
    U, S, V, info = run(lib, A, fused_rounds=1, branch=lib.BRANCH_LOW, wait_polls=-1)
    # (the BF16 sweeps give up first, then the FP32 fused round: both fall back)
    g = metrics.gates(A, U, S, V, So)
    assert info["status"] == 0 and info["fused_fallback"] == 1, info
    assert g["pass"], g


@pytest.mark.parametrize("shape,storage", [((512, 512), 0), ((1000, 1000), 0), ((1300, 1090), 0),
                                           ((1000, 1000), 1)])
def test_bf16_sweeps_parity(lib, shape, storage):
    m, n = shape
    print(f"case bf16 sweeps m={m} n={n} storage={storage}", flush=True)
    rng = np.random.default_rng(3000 + n)
    A = testmats.compose(testmats.haar(rng, m, n), testmats.sigma_log_uniform(rng, n, 10.0),
                         testmats.haar(rng, n, n))
    _, So, _, _ = oracle.svd(A)
    U, S, V, info = run(lib, A, fused_rounds=1, half_sweeps=6, half_storage=storage,
                        branch=lib.BRANCH_LOW, kernel_timing=100 + ROUND16)
    g = metrics.gates(A, U, S, V, So)
    print({k: g[k] for k in ("e_sigma", "orth_u", "orth_v", "residual")},
          {k: info[k] for k in ("status", "sweeps_half", "sweeps_low", "sweeps_work")},
          "bf16 launches", info["kern_calls"][ROUND16], flush=True)
    assert info["status"] == 0 and info["fused_fallback"] == 0, info
    assert info["sweeps_half"] >= 1 and info["kern_calls"][ROUND16] > 0, info
    assert g["pass"], g


def test_bf16_sweeps_graded_c2_stream_ordered(lib):
    """The graded 1024^2 matrix (column scaling over six decades; the BF16
    copy keeps FP32's exponent range) with the BF16 sweeps, host-synchronised
    and stream-ordered: bit-identical results, stored oracle sigma."""
    print("case bf16 sweeps C2", flush=True)
    s_ref, kappa, fp, _ = load("C2")
    A, _ = testmats.config_c2()
    kw = dict(fused_rounds=1, half_sweeps=6, branch=lib.BRANCH_LOW, y2_safeguard=0)
    U, S, V, info = run(lib, A, **kw)
    U1, S1, V1, info1 = run(lib, A, capture=1, **kw)
    info1 = info1.read()
    print({k: (info[k], info1[k]) for k in ("status", "sweeps_half", "sweeps_low", "sweeps_work")},
          flush=True)
    assert np.array_equal(S, S1) and np.array_equal(U, U1) and np.array_equal(V, V1)
    assert info["sweeps_half"] == info1["sweeps_half"] >= 1
    n = A.shape[1]
    assert metrics.e_sigma(S, s_ref, kappa) <= 1e-13
    assert metrics.orth_err(U) <= 1e-13 * n and metrics.orth_err(V) <= 1e-13 * n
    assert metrics.residual(A, U, S, V) <= 1e-14 * n
