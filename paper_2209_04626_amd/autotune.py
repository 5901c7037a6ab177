"""Autotuner for the tuning table the library reads (svd_set_tuning).

It measures, on the GPU it runs on:
- for each problem size n, the Jacobi block widths of the FP64 stage
  (timed on svd_plain) and then of the FP32 stage (timed on svd_mixed with
  the chosen FP64 width), each candidate checked against the accuracy gates;
- for a ragged batch of the batched workload's shape mix, the persistent
  grid of svd_batched (workgroups per compute unit), timed on graph replays.

Inputs are the seeded synthetic families of testmats (Haar U and V,
log-uniform singular values).  The table is written as JSON:

    python3 -m paper_2209_04626_amd.autotune --out paper_2209_04626_amd/tune_gfx950.json

--sizes, --reps and --batch shorten or widen the search.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))


def _gates_ok(torch, A, U, S, V) -> bool:
    n = A.shape[1]
    eye = torch.eye(n, dtype=torch.float64, device=A.device)
    orth_u = torch.linalg.norm(U.t() @ U - eye).item()
    orth_v = torch.linalg.norm(V.t() @ V - eye).item()
    res = (torch.linalg.norm(A - (U * S) @ V.t()) / torch.linalg.norm(A)).item()
    return orth_u <= 1e-13 * n and orth_v <= 1e-13 * n and res <= 1e-14 * n


def _time_svd(torch, mp, A, mode, ws, reps, **kw):
    opts = mp.default_opts(mode == "mixed", **kw)
    U, S, V, info = mp.svd(A, mode, workspace=ws, opts=opts)
    ok = info["status"] == 0 and _gates_ok(torch, A, U, S, V)
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mp.svd(A, mode, workspace=ws, opts=opts)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    ts.sort()
    return ts[len(ts) // 2] * 1e3, ok


def tune_single(torch, mp, np, testmats, sizes, reps, log):
    entries, measured = [], []
    ws = mp.Workspace()
    for n in sizes:
        A_np, _ = testmats.config_c3b(n=n)
        A = torch.from_numpy(np.ascontiguousarray(A_np)).cuda()
        work = {}
        for bw in (16, 32):
            work[bw] = _time_svd(torch, mp, A, "plain", ws, reps, block_cols_work=bw)
        ok_w = [b for b in work if work[b][1]] or list(work)
        b_work = min(ok_w, key=lambda b: work[b][0])
        low = {}
        for bl in (16, 32):
            low[bl] = _time_svd(torch, mp, A, "mixed", ws, reps, block_cols_low=bl, block_cols_work=b_work)
        ok_l = [b for b in low if low[b][1]] or list(low)
        b_low = min(ok_l, key=lambda b: low[b][0])
        entries.append({"nmax": n, "b_low": b_low, "b_work": b_work})
        rec = {"n": n, "plain_ms": {str(b): round(work[b][0], 2) for b in work},
               "mixed_ms": {str(b): round(low[b][0], 2) for b in low},
               "gates_ok": all(v[1] for v in list(work.values()) + list(low.values()))}
        measured.append(rec)
        log(f"[autotune] n={n}: b_work={b_work} b_low={b_low} {rec}")
        del A
    return entries, measured


def tune_batched(torch, mp, testmats, batch, reps, log):
    shapes, mats, _ = testmats.config_c4(batch=batch)
    Ap = mp.pack_batch(mats, torch.device("cuda:0"))
    nmax = max(n for _, n in shapes)
    ws = mp.Workspace()
    times = {}
    for w in (1, 2, 4):
        mp.set_tuning({"batched": [{"nmax": 4096, "wg_per_cu": w}]})
        plan = mp.batched_plan(shapes)
        mp.svd_batched(plan, Ap, workspace=ws)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            mp.svd_batched(plan, Ap, workspace=ws)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        ts.sort()
        times[w] = ts[len(ts) // 2] * 1e3
        log(f"[autotune] batched {batch} matrices, {w} workgroups per CU: {times[w]:.2f} ms")
        del plan
    mp.set_tuning(None)
    # the fewest workgroups per unit within 2 % of the fastest (each one holds
    # its own workspace slice)
    fastest = min(times.values())
    best = min(w for w, t in times.items() if t <= 1.02 * fastest)
    return [{"nmax": max(nmax, 256), "wg_per_cu": best}], {"batch": batch,
                                                          "ms": {str(k): round(v, 2) for k, v in times.items()}}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--out", default=os.path.join(HERE, "tune_gfx950.json"))
    ap.add_argument("--sizes", default="128,256,512,1024,2048,4096")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--batch", type=int, default=2000)
    args = ap.parse_args()

    import numpy as np
    import torch

    import paper_2209_04626_amd as mp
    import testmats

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    mp.load()
    mp.set_tuning(None)   # measure from the built-in choices
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    sizes = [int(x) for x in args.sizes.split(",") if x]
    single, meas_single = tune_single(torch, mp, np, testmats, sizes, args.reps, log)
    batched, meas_batched = tune_batched(torch, mp, testmats, args.batch, args.reps, log)
    table = {"arch": arch, "single": single, "batched": batched,
             "measured": {"single": meas_single, "batched": meas_batched}}
    with open(args.out, "w") as fh:
        json.dump(table, fh, indent=1)
        fh.write("\n")
    log(f"[autotune] wrote {args.out}")
    mp.set_tuning(table)
    return 0


if __name__ == "__main__":
    sys.exit(main())
