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

--switch-study compares the two switch methods of Theorem 4 on the
workload of the paper's switching test (Section 6): A = B D with
(kappa(D), kappa(B)) = (1e2, 1e12), the 16 mode pairs of Table 1.  For
each matrix and method it takes Y as the FP64 sweeps start (diagnostics = 2)
and reports the distribution of the off-diagonal |Y_c^T Y_c - I| (Y_c: Y with
unit columns; the quantity the paper plots), ||Y_c^T Y_c - I||_2, and
||Y Sigma^-1 - U||_2 of Theorem 4, with U, Sigma from a high-accuracy FP64
SVD of Y itself (svd_plain; Y = X Q has X's left vectors), each column of Y
matched to its singular vector through the right factor.

    python3 -m paper_2209_04626_amd.ablation --switch-study --n 1024
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


def switch_study(n: int) -> list:
    import numpy as np
    import torch

    import paper_2209_04626_amd as mp
    import testmats

    with open(os.path.join(os.path.dirname(HERE), "tests", "golden", "paper_values.json")) as fh:
        modes = json.load(fh)["table1_modes"]
    dev = torch.device("cuda")
    ws = mp.Workspace()
    N = -(-n // 64) * 64
    eye = torch.eye(n, dtype=torch.float64, device=dev)
    rows = []
    for t, (md, ms) in enumerate(modes):
        A_np = testmats.graded(600 + t, n, n, ms, 1e12, md, 1e2)
        A = torch.from_numpy(np.ascontiguousarray(A_np)).to(dev)
        for method in (1, 2):
            o = mp.default_opts(True, branch=mp.BRANCH_LOW, switch_method=method, v_method=0,
                                diagnostics=2, y2_safeguard=0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            U, S, V, info = mp.svd(A, "mixed", workspace=ws, opts=o)
            torch.cuda.synchronize()
            ms_call = (time.perf_counter() - t0) * 1e3
            off = mp.load().svd_diag_y_offset(n, n, o)
            Yst = ws.buf[off:off + N * N * 8].view(torch.float64).view(N, N)
            Y = Yst[:n, :n].t().contiguous()                     # column-major storage
            d = torch.linalg.norm(Y, dim=0)
            Yc = Y / d
            C = Yc.t() @ Yc - eye
            offd = C.abs()[~torch.eye(n, dtype=torch.bool, device=dev)]
            q = torch.quantile(offd[torch.randperm(offd.numel(), device=dev)[:1 << 22]],
                               torch.tensor([0.5, 0.9, 0.99], dtype=torch.float64, device=dev))
            c2 = torch.linalg.matrix_norm(C, ord=2).item()
            # Theorem 4's ||Y Sigma^-1 - U||_2 from an accurate SVD of Y
            Uy, Sy, Wy, _ = mp.svd(Y, "plain", workspace=mp.Workspace())
            pi = Wy.abs().argmax(dim=1)
            perm_ok = bool(torch.unique(pi).numel() == n)
            sg = torch.sign(Wy[torch.arange(n, device=dev), pi])
            E = Y / Sy[pi] - Uy[:, pi] * sg
            e4 = torch.linalg.matrix_norm(E, ord=2).item() if perm_ok else float("nan")
            rows.append({"type": t + 1, "modes": [md, ms], "method": method,
                         "sweeps_low": info["sweeps_low"], "sweeps_work": info["sweeps_work"],
                         "ms": round(ms_call, 1), "status": info["status"],
                         "offdiag_q50": q[0].item(), "offdiag_q90": q[1].item(),
                         "offdiag_q99": q[2].item(), "offdiag_max": offd.max().item(),
                         "orth2": c2, "thm4": e4, "perm_ok": perm_ok})
            print(f"[switch] type {t + 1} method {method}: sweeps {info['sweeps_work']}, "
                  f"max {rows[-1]['offdiag_max']:.2e}, thm4 {e4:.2e}", file=sys.stderr, flush=True)
    return rows


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--config", default="c3b", choices=("c1", "c2", "c3a", "c3b"))
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--json", default=None, help="also write the rows as JSON here")
    ap.add_argument("--switch-study", action="store_true",
                    help="Theorem 4's two switch methods on the Section 6 workload")
    ap.add_argument("--n", type=int, default=1024)
    args = ap.parse_args()
    if args.switch_study:
        rows = switch_study(args.n)
        print(f"| type (D mode, Sigma mode) | method | FP64 sweeps | off-diag median | 90% | 99% | max "
              f"| ||Yc^T Yc - I||_2 | ||Y Sigma^-1 - U||_2 |")
        print("|---|---:|---:|---:|---:|---:|---:|---:|---:|")
        for r in rows:
            print(f"| {r['type']} ({r['modes'][0]}, {r['modes'][1]}) | {r['method']} | {r['sweeps_work']} | "
                  f"{r['offdiag_q50']:.1e} | {r['offdiag_q90']:.1e} | {r['offdiag_q99']:.1e} | "
                  f"{r['offdiag_max']:.1e} | {r['orth2']:.1e} | {r['thm4']:.1e} |")
        import statistics
        for m in (1, 2):
            rr = [r for r in rows if r["method"] == m]
            print(f"| median over types | {m} | {statistics.median(r['sweeps_work'] for r in rr)} | "
                  f"{statistics.median(r['offdiag_q50'] for r in rr):.1e} | "
                  f"{statistics.median(r['offdiag_q90'] for r in rr):.1e} | "
                  f"{statistics.median(r['offdiag_q99'] for r in rr):.1e} | "
                  f"{statistics.median(r['offdiag_max'] for r in rr):.1e} | "
                  f"{statistics.median(r['orth2'] for r in rr):.1e} | "
                  f"{statistics.median(r['thm4'] for r in rr):.1e} |")
        if args.json:
            with open(args.json, "w") as fh:
                json.dump(rows, fh, indent=1)
        return 0

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
