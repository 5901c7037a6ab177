"""GPU checks of the stream-ordered mode (svd_opts.capture = 1): no host
synchronisation inside svd_plain / svd_mixed, every decision (the branch
tests of Section 3.5, the stopping rules of each sweep stage, the acceptance
of the solved V of Section 3.4) taken on the device, svd_info written there.

- eager capture=1 against the host-synchronised call on the same input with
  the Y2 safeguard off (the one step the stream-ordered mode leaves out): the
  same kernels in the same order, so S, U and V must agree bit for bit, and
  the device-written info must report the same branch and sweep counts;
  both must meet the oracle's gates.  Square, tall and fused-round cases.
- a HIP graph (torch.cuda.CUDAGraph) holding one svd_mixed call, replayed on
  two different inputs copied into the captured input buffer, three replays
  in all with eager work and synchronisation between them; every replay is
  checked against the eager result of the same input and the oracle.
- the skip branch taken on the device (small cond_R): sweeps_low = 0, the
  result equals the host-synchronised skip result.
- status words on the device: non-finite input, a sweep cap, a zero column
  with the solved V (SVD_WARN_VSOLVE, S and U still valid).
"""
import numpy as np
import pytest

import oracle
import testmats
from testmats import metrics

pytestmark = pytest.mark.gpu


def known(m, n, seed, e=8.0):
    rng = np.random.default_rng(seed)
    return testmats.compose(testmats.haar(rng, m, n), testmats.sigma_log_uniform(rng, n, e),
                            testmats.haar(rng, n, n))


def run(lib, A, mode, **kw):
    import torch
    At = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    U, S, V, info = lib.svd(At, mode, **kw)
    if kw.get("capture"):
        info = info.read()          # synchronises
    torch.cuda.synchronize()
    return U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy(), info


SAME = ("branch_taken", "sweeps_low", "sweeps_work", "n_small", "v_method_taken", "status")


@pytest.mark.parametrize("mode,shape,kw", [
    ("mixed", (384, 384), {}),
    ("mixed", (700, 450), {}),
    ("mixed", (1000, 1000), {"fused_rounds": 1}),
    ("mixed", (320, 320), {"v_method": 0}),
    ("plain", (384, 384), {}),
])
def test_stream_ordered_matches_synchronised(lib, mode, shape, kw):
    m, n = shape
    print(f"case capture=1 vs 0 mode={mode} m={m} n={n} {kw}", flush=True)
    A = known(m, n, seed=100 + n)
    U0, S0, V0, i0 = run(lib, A, mode, y2_safeguard=0, **kw)
    U1, S1, V1, i1 = run(lib, A, mode, y2_safeguard=0, capture=1, **kw)
    print({k: (i0[k], i1[k]) for k in SAME}, flush=True)
    for k in SAME:
        assert i0[k] == i1[k], (k, i0, i1)
    assert i1["off_work"] == pytest.approx(i0["off_work"], rel=0, abs=0)
    assert np.array_equal(S0, S1) and np.array_equal(U0, U1) and np.array_equal(V0, V1)
    So = oracle.svd(A)[1]
    g = metrics.gates(A, U1, S1, V1, So)
    assert i1["status"] == 0 and g["pass"], (g, i1)
    if mode == "mixed":
        assert i1["branch_taken"] == lib.BRANCH_LOW and i1["sweeps_low"] >= 1


def test_graph_capture_replays(lib):
    import torch
    n = 512
    print(f"case graph capture svd_mixed n={n}", flush=True)
    A1 = known(n, n, seed=201)
    A2 = known(n, n, seed=202, e=10.0)
    dev = torch.device("cuda")
    o = lib.default_opts(True, capture=1, y2_safeguard=0, maxsweep_low=12, maxsweep_work=12)
    ws = lib.Workspace()
    ws.get(lib.workspace_size(n, n, o), dev)
    A_in = torch.from_numpy(np.ascontiguousarray(A1)).to(dev)
    # eager results of both inputs, for comparison
    ref = {}
    for key, A in (("A1", A1), ("A2", A2)):
        U, S, V, di = lib.svd(torch.from_numpy(np.ascontiguousarray(A)).to(dev), "mixed",
                              workspace=ws, opts=o)
        ref[key] = (U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy(), di.read())
    out = lib.svd(A_in, "mixed", workspace=ws, opts=o)        # buffers reused by the graph
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        lib.svd(A_in, "mixed", workspace=ws, opts=o, out=out)   # warm-up on the side stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        lib.svd(A_in, "mixed", workspace=ws, opts=o, out=out)
    torch.cuda.synchronize()
    So = {"A1": oracle.svd(A1)[1], "A2": oracle.svd(A2)[1]}
    for rep, (key, A) in enumerate((("A2", A2), ("A1", A1), ("A2", A2))):
        A_in.copy_(torch.from_numpy(np.ascontiguousarray(A)).to(dev))
        junk = torch.randn(256, 256, device=dev, dtype=torch.float64) @ torch.randn(
            256, 256, device=dev, dtype=torch.float64)        # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        U, S, V, di = out
        U, S, V, info = U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy(), di.read()
        Ur, Sr, Vr, ir = ref[key]
        print(f"replay {rep} {key}", {k: info[k] for k in SAME}, float(junk[0, 0]), flush=True)
        for k in SAME:
            assert info[k] == ir[k], (rep, k, info, ir)
        assert np.array_equal(S, Sr) and np.array_equal(U, Ur) and np.array_equal(V, Vr), rep
        gt = metrics.gates(A, U, S, V, So[key])
        assert info["status"] == 0 and gt["pass"], (rep, gt, info)


def test_skip_branch_on_device(lib):
    print("case capture=1 skip cond_R", flush=True)
    n = 256
    rng = np.random.default_rng(21)
    A = np.asfortranarray(np.eye(n) + 0.05 * rng.standard_normal((n, n)) / np.sqrt(n))
    U0, S0, V0, i0 = run(lib, A, "mixed", y2_safeguard=0)
    U1, S1, V1, i1 = run(lib, A, "mixed", y2_safeguard=0, capture=1)
    assert i0["branch_taken"] == i1["branch_taken"] == lib.BRANCH_SKIP, (i0, i1)
    assert i1["sweeps_low"] == 0 and i1["sweeps_work"] == i0["sweeps_work"]
    assert i1["orth"] >= 0.0          # all three tests are measured on the device
    assert np.array_equal(S0, S1) and np.array_equal(U0, U1) and np.array_equal(V0, V1)
    So = oracle.svd(A)[1]
    assert metrics.gates(A, U1, S1, V1, So)["pass"]


@pytest.mark.parametrize("mode", ["plain", "mixed"])
def test_device_status_nonfinite(lib, mode):
    print(f"case capture=1 NaN mode={mode}", flush=True)
    A = known(150, 120, seed=1)
    A[37, 91] = np.nan
    _, _, _, info = run(lib, A, mode, capture=1)
    assert info["status"] == lib.SVD_ERR_NONFINITE, info


@pytest.mark.parametrize("mode", ["plain", "mixed"])
def test_device_status_noconv(lib, mode):
    print(f"case capture=1 maxsweep_work=1 mode={mode}", flush=True)
    A = known(256, 256, seed=11, e=10.0)
    _, _, _, info = run(lib, A, mode, capture=1, maxsweep_work=1,
                        branch=1 if mode == "mixed" else 0)
    assert info["status"] == lib.SVD_WARN_NOCONV and info["sweeps_work"] == 1, info


def test_device_status_vsolve_rejected(lib):
    """A zero column makes l_nn = 0: the solve for V is rejected on the
    device; without the host-driven fallback the call reports
    SVD_WARN_VSOLVE, and S (with its exact zero) and U are still valid."""
    print("case capture=1 zero column v_method=1", flush=True)
    n = 200
    rng = np.random.default_rng(5)
    H = testmats.haar(rng, n, n)
    d = testmats.sigma_geometric(n, 4.0)
    d[-1] = 0.0
    A = np.asfortranarray(H * d)
    U, S, V, info = run(lib, A, "mixed", capture=1, branch=1)
    assert info["status"] == lib.SVD_WARN_VSOLVE and info["v_method_taken"] == 3, info
    ds = np.sort(d)[::-1]
    assert S[-1] == 0.0 and np.max(np.abs(S[:-1] - ds[:-1]) / ds[:-1]) < 1e-12
    assert np.all(np.isfinite(U)) and metrics.orth_err(U[:, :-1]) <= 1e-13 * n


def test_capture_rejects_host_only_options(lib):
    import torch
    A = torch.from_numpy(known(64, 64, seed=3)).cuda()
    for kw in ({"kernel_timing": 2}, {"switch_method": 3}):
        with pytest.raises(RuntimeError, match="returned -12"):
            lib.svd(A, "mixed", capture=1, **kw)
