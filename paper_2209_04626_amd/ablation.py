"""Ablations of the mixed path on one synthetic configuration (Section 6):

- the switch of precisions: method 1 (Algorithm 4, Q from the QR of X^T U_low),
  method 2 (Q from the QR of the FP32-accumulated V_low, Y = X Q) and
  method 3 (Algorithm 3: the FP64 sweeps on A1 Q, Q from the QR of the FP32
  right vectors of A);
- the right singular vectors: accumulated through the FP64 sweeps, or formed
  afterwards by the triangular solve of Section 3.4;
- the plain FP64 path with both V methods, for reference.

For each variant it reports the time per SVD (median of --reps), the stage
times, the sweep counts, the orthogonality of Y when the FP64 sweeps start
(max |D^-1 Y^T Y D^-1 - I|), the per-sweep off-diagonal trace, and the
orthogonality / residual gates; sigma is compared with the first variant's.

    python3 -m paper_2209_04626_amd.ablation --config c3b --reps 2
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

VARIANTS = [
    ("Alg. 4, switch 1, V solved (default)", "mixed", dict(switch_method=1, v_method=1)),
    ("Alg. 4, switch 1, V accumulated", "mixed", dict(switch_method=1, v_method=0)),
    ("switch 2 (QR of V_low), V accumulated", "mixed", dict(switch_method=2, v_method=0)),
    ("Alg. 3 (sweeps on A1 Q), V accumulated", "mixed", dict(switch_method=3, v_method=0)),
    ("plain, V accumulated (default)", "plain", dict(v_method=0)),
    ("plain, V solved", "plain", dict(v_method=1)),
]


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--config", default="c3b", choices=("c1", "c2", "c3a", "c3b"))
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--json", default=None, help="also write the rows as JSON here")
    args = ap.parse_args()

    import numpy as np
    import torch

    import paper_2209_04626_amd as mp
    import testmats

    A_np, _ = getattr(testmats, "config_" + args.config)()
    A = torch.from_numpy(np.ascontiguousarray(A_np)).cuda()
    m, n = A.shape
    eye = torch.eye(n, dtype=torch.float64, device=A.device)
    ws = mp.Workspace()
    rows, S_ref = [], None
    for name, mode, kw in VARIANTS:
        force = dict(branch=mp.BRANCH_LOW) if mode == "mixed" else {}
        U, S, V, info = mp.svd(A, mode, workspace=ws, diagnostics=1, **force, **kw)
        torch.cuda.synchronize()
        orth_u = torch.linalg.norm(U.t() @ U - eye).item()
        orth_v = torch.linalg.norm(V.t() @ V - eye).item()
        res = (torch.linalg.norm(A - (U * S) @ V.t()) / torch.linalg.norm(A)).item()
        if S_ref is None:
            S_ref = S.clone()
        dsig = (torch.abs(S - S_ref) / S_ref).max().item()
        ts = []
        for _ in range(args.reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            mp.svd(A, mode, workspace=ws, **force, **kw)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        ts.sort()
        row = {
            "variant": name, "ms": round(ts[len(ts) // 2] * 1e3, 1),
            "stage_ms": [round(x, 1) for x in info["stage_ms"]],
            "sweeps_low": info["sweeps_low"], "sweeps_work": info["sweeps_work"],
            "sweeps_vfix": info["sweeps_vfix"], "v_method_taken": info["v_method_taken"],
            "orth_y": info["orth_y"], "orth_vx": info["orth_vx"],
            "off_work": [float("%.2g" % x) for x in info["off_work"]],
            "orth_u_per_n": orth_u / n, "orth_v_per_n": orth_v / n, "residual_per_n": res / n,
            "gates": bool(orth_u <= 1e-13 * n and orth_v <= 1e-13 * n and res <= 1e-14 * n),
            "max_rel_sigma_vs_first": dsig, "status": info["status"],
        }
        rows.append(row)
        print(f"[ablation] {name}: {row['ms']} ms", file=sys.stderr, flush=True)

    print(f"| variant ({args.config}: {m}x{n}) | ms | FP32 sweeps | FP64 sweeps | orth(Y) at FP64 start "
          f"| FP64 off trace | stage ms (pivots, QR, LQ, FP32, switch, FP64+fin) | gates | rel. sigma vs row 1 |")
    print("|---|---:|---:|---:|---:|---|---|---|---:|")
    for r in rows:
        st = r["stage_ms"]
        print(f"| {r['variant']} | {r['ms']} | {r['sweeps_low']} | {r['sweeps_work']}"
              f"{' + ' + str(r['sweeps_vfix']) if r['sweeps_vfix'] else ''} | {r['orth_y']:.2e} | "
              f"{r['off_work']} | {st[1]}, {st[2]}, {st[3]}, {st[5]}, {st[6]}, {st[7]} | "
              f"{'pass' if r['gates'] else 'FAIL'} | {r['max_rel_sigma_vs_first']:.1e} |")
    if args.json:
        with open(args.json, "w") as fh:
            json.dump(rows, fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
