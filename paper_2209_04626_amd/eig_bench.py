"""Timing and accuracy of the mixed-precision eigensolver (Algorithm 6).

Input: A = Q diag(lam) Q^T with Haar Q and lam = +-10^-u, u ~ U(0, E), random
signs (the eigenvalue analogue of the SVD workloads), built in FP64 on the host.
For each n it times eig_mixed (median of --reps, after one untimed call) and
torch.linalg.eigh on the same GPU (the library eigensolver, for scale), and
reports both against ||X^T X - I||_F / n and ||A X - X diag(w)||_F /
(||A||_F n), and the largest error of each eigenvalue relative to the lam the
matrix was built from (floored by the rounding of the construction, about
u ||A|| / |lam|, for the small ones).

    python3 -m paper_2209_04626_amd.eig_bench --sizes 512,1024,4096
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--sizes", default="512,1024,4096")
    ap.add_argument("--exp", type=float, default=12.0)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()

    import numpy as np
    import torch

    import paper_2209_04626_amd as mp
    import testmats

    ws = mp.Workspace()
    rows = []
    for n in [int(x) for x in args.sizes.split(",") if x]:
        rng = np.random.default_rng(1000 + n)
        lam = 10.0 ** -rng.uniform(0, args.exp, n) * np.where(rng.random(n) < 0.5, -1.0, 1.0)
        Q = testmats.haar(rng, n, n)
        A_np = (Q * lam) @ Q.T
        A_np = (A_np + A_np.T) / 2
        A = torch.from_numpy(np.ascontiguousarray(A_np)).cuda()
        eye = torch.eye(n, dtype=torch.float64, device=A.device)

        def check(W, X):
            orth = torch.linalg.norm(X.t() @ X - eye).item() / n
            res = (torch.linalg.norm(A @ X - X * W) / torch.linalg.norm(A)).item() / n
            return orth, res

        W, X, info = mp.eigh(A, workspace=ws)
        torch.cuda.synchronize()
        ts = []
        for _ in range(args.reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            mp.eigh(A, workspace=ws)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        ts.sort()
        t_mixed = ts[len(ts) // 2]
        Wt, Xt = torch.linalg.eigh(A)
        torch.cuda.synchronize()
        ts = []
        for _ in range(args.reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            torch.linalg.eigh(A)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        ts.sort()
        t_lib = ts[len(ts) // 2]
        row = {"n": n, "eig_mixed_ms": round(t_mixed * 1e3, 2), "torch_eigh_ms": round(t_lib * 1e3, 2),
               "info": info, "eig_mixed_orth_res": check(W, X), "torch_orth_res": check(Wt, Xt)}
        ref = np.sort(lam)
        row["eig_mixed_max_rel_err_vs_lam"] = float(np.max(np.abs(W.cpu().numpy() - ref) / np.abs(ref)))
        row["torch_max_rel_err_vs_lam"] = float(np.max(np.abs(Wt.cpu().numpy() - ref) / np.abs(ref)))
        rows.append(row)
        print(json.dumps(row), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
