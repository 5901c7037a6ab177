"""svd_backward_noalloc (the adjoint with the library's fixed scratch array
instead of a caller workspace) against svd_backward, through the C ABI.

Two calls in a row on the same process and GPU, the second with a smaller
batch and shape, so the second reuses the array the first left behind.  Each
result must equal svd_backward's on the same inputs bit for bit (the same
kernel runs on the same data), and a few matrices are checked against the
FP64 CPU formula at the adjoint's 1e-8 gate.  A problem larger than the array
is refused with SVD_ERR_SCRATCH_LIMIT before anything is launched.
"""
import ctypes

import numpy as np
import pytest

import oracle
import testmats

pytestmark = pytest.mark.gpu


def factors(batch, m, n, seed):
    """Exact SVD factors in the gradient workload's recipe: Haar U (m x n) and
    V (n x n), sigma ~ U(0.1, 10) sorted with relative gaps >= 1e-3, N(0, 1)
    cotangents."""
    rng = np.random.default_rng(seed)
    U = np.stack([testmats.haar(rng, m, n) for _ in range(batch)])
    V = np.stack([testmats.haar(rng, n, n) for _ in range(batch)])
    S = []
    for _ in range(batch):
        while True:
            s = np.sort(rng.uniform(0.1, 10.0, n))[::-1].copy()
            if n == 1 or np.min((s[:-1] - s[1:]) / s[:-1]) >= 1e-3:
                break
        S.append(s)
    S = np.stack(S)
    gU = rng.standard_normal((batch, m, n))
    gS = rng.standard_normal((batch, n))
    gV = rng.standard_normal((batch, n, n))
    return U, S, V, gU, gS, gV


def run_both(lib, batch, m, n, seed):
    import torch
    print(f"case noalloc batch={batch} m={m} n={n} seed={seed}", flush=True)
    U, S, V, gU, gS, gV = factors(batch, m, n, seed)
    t = [torch.from_numpy(x).cuda() for x in (U, S, V, gU, gS, gV)]
    ref = lib.svd_backward(*t)
    got = lib.svd_backward(*t, noalloc=True)
    torch.cuda.synchronize()
    ref, got = ref.cpu().numpy(), got.cpu().numpy()
    assert np.all(np.isfinite(got))
    assert np.array_equal(got, ref), float(np.max(np.abs(got - ref)))
    for b in (0, batch // 2, batch - 1):
        r = oracle.svd_backward_ref(U[b], S[b], V[b], gU[b], gS[b], gV[b])
        assert np.linalg.norm(got[b] - r) <= 1e-8 * np.linalg.norm(r), b


def test_noalloc_matches_workspace_entry_point_twice(lib):
    # gradient workload size (40 MiB of scratch), then a smaller ragged one
    run_both(lib, 256, 128, 64, seed=21)
    run_both(lib, 7, 45, 33, seed=22)


def test_noalloc_refuses_beyond_its_array(lib):
    import torch
    L = lib.load()
    m, n = 128, 64
    per = int(L.svd_backward_workspace_size(2, m, n)) - int(L.svd_backward_workspace_size(1, m, n))
    batch = lib.BACKWARD_NOALLOC_SCRATCH_BYTES // per + 1
    assert int(L.svd_backward_workspace_size(batch, m, n)) > lib.BACKWARD_NOALLOC_SCRATCH_BYTES
    # valid pointers are required up to the size check; nothing is launched,
    # so one small buffer stands for every operand
    buf = torch.zeros(16, dtype=torch.float64, device="cuda")
    p = buf.data_ptr()
    rc = L.svd_backward_noalloc(batch, m, n, p, m * n, p, n, p, n * n, None, None, None, p, m * n, 0.0,
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == lib.SVD_ERR_SCRATCH_LIMIT, rc
    assert b"scratch" in L.svd_last_error()
    torch.cuda.synchronize()
    assert torch.count_nonzero(buf).item() == 0
