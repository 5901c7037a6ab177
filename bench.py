#!/usr/bin/env python3
"""Benchmark of the mixed-precision Jacobi SVD on one MI355X.

Metric: time of an n = 4096 SVD, svd_mixed (Algorithm 4) against svd_plain
(FP64 preconditioned Jacobi, Algorithm 2), on the same GPU, both with U and V
requested, both checked against the accuracy gates
(e_sigma <= 1e-13 after the column-scaled condition adjustment,
||U^T U - I||_F, ||V^T V - I||_F <= 1e-13 n, ||A - U S V^T||_F/||A||_F <=
1e-14 n).  value = T_plain / T_mixed; ms_per_step = T_mixed (one step = one
mixed SVD of the whole path).

Workload: 4096 x 4096 FP64 A = U diag(sigma) V^T, Haar U and V, sigma
log-uniform in [1e-12, 1], seed 4 (testmats.config_c3b).  Inputs are resident
in HBM before the timed region starts.

Prints one JSON line.  Options: --gpus (only 1), --steps K, --warmup W,
--n (size), --mode (both | mixed | plain: "both" is the metric, the others are
for profiling runs), --no-cpu-baseline, --cpu-sample-n.

Kernel classes: before the timed region, one SVD of each kind per kernel
class is run with HIP events on the launches of that class only (recorded by
the dispatch itself for the Jacobi kernels); the largest class of the mixed
step (GEMMs aside) is the dominant kernel, and the timed mixed SVDs clock it
(the pivot pass as one interval per pass).
roofline.traffic is the HBM traffic per launch of the dominant kernel from
the counter runs recorded in profiles/ (a <kernel>_n4096_traffic.md file); it
is reported only while the kernel's sources hash to the value recorded there.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
CLOCK_EVERY = 8                # sampled clocking of the dominant Jacobi class
FP64_PEAK_TF = 78.6            # dense FP64 (vector and MFMA)
FP32_PEAK_TF = 157.3           # dense FP32 (vector and MFMA)


def algorithmic_flops(n: int, info: dict, mixed: bool) -> float:
    """Algorithmic flop count of one SVD (square n, U and V formed), from the
    stage formulas: pivot pass 4n^3/3, QR of A1 P 4n^3/3, LQ 4n^3/3, branch
    SYRK n^3, FP32 sweeps 4n^2(n-1) each, switch 4.7 n^3, FP64 sweeps with V
    7n^2(n-1) each (without V 4n^2(n-1) each, then the triangular solve for
    V_X n^3; its fallback adds X^T U_X 2n^3, a QR 4n^3/3, X Q 2n^3 and sweeps
    with V), back-transforms 4n^3."""
    f = 4 * n ** 3 / 3 * 3 + 4 * n ** 3
    if mixed:
        f += n ** 3
        if info["branch_taken"] == 1:
            f += info["sweeps_low"] * 4 * n * n * (n - 1) + 4.7 * n ** 3
    if info.get("v_method_taken", 0) >= 1:
        f += info["sweeps_work"] * 4 * n * n * (n - 1) + n ** 3
        if info["v_method_taken"] == 2:
            f += 2 * n ** 3 + 4 * n ** 3 / 3 + 2 * n ** 3 + info["sweeps_vfix"] * 7 * n * n * (n - 1)
    else:
        f += info["sweeps_work"] * 7 * n * n * (n - 1)
    return f


# counter records (profiles/) of the kernels bench.py may report as dominant,
# with the sources whose hash the record carries
TRAFFIC = {
    "qrcp": ("qrcp_persist_f32_n4096_traffic.md",
             ["paper_2209_04626_amd/csrc/qrcp.hip", "paper_2209_04626_amd/csrc/common.hpp"]),
    "jac_update<f32>": ("jac_update_f32_n4096_traffic.md",
                        ["paper_2209_04626_amd/csrc/jacobi.hip", "paper_2209_04626_amd/csrc/common.hpp"]),
    "qr_panel": ("qr_panel_coop_n4096_traffic.md",
                 ["paper_2209_04626_amd/csrc/qr.hip", "paper_2209_04626_amd/csrc/common.hpp"]),
}


def kernel_source_hash(kernel: str = "qrcp") -> str:
    h = hashlib.sha256()
    for f in TRAFFIC[kernel][1]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(n: int, kernel: str = "qrcp"):
    """HBM bytes per launch of `kernel` measured with the FETCH_SIZE /
    WRITE_SIZE counters (copy-calibrated), or None when there is no record for
    this size or the kernel's sources have changed since."""
    if n != 4096 or kernel not in TRAFFIC:
        return None
    TRAFFIC_FILE = os.path.join(ROOT, "profiles", TRAFFIC[kernel][0])
    if not os.path.exists(TRAFFIC_FILE):
        return None
    rec = {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            m = re.match(r"^- (\w+): `?([^`\s]+)`?", line.strip())
            if m:
                rec[m.group(1)] = m.group(2)
    if rec.get("source_sha256") != kernel_source_hash(kernel):
        return None
    try:
        return float(rec["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# per-class roofline: which roof bounds the class and the peak it is priced
# against (HBM 8 TB/s; dense FP32 / FP64 157.3 / 78.6 TFLOP/s)
CLASS_ROOF = {
    "jac_gram<f32>": ("hbm", None), "jac_update<f32>": ("hbm", None),
    "jac_gram<f64>": ("hbm", None), "jac_update<f64>": ("hbm", None),
    "jac_inner<f32>": ("latency", FP64_PEAK_TF), "jac_inner<f64>": ("latency", FP64_PEAK_TF),
    "qrcp": ("hbm", None), "qr_panel": ("latency", FP64_PEAK_TF), "gemm": ("mfma", FP64_PEAK_TF),
}


def class_survey(mp, A, ws, mode: str, classes) -> dict:
    """One clocked SVD per kernel class, with HIP events around the launches of
    that class only (kernel_timing = 100 + class), so the other launches run
    as in an unclocked SVD.  Returns {class: (ms, launches, bytes, flops)}."""
    import torch
    out = {}
    for c in classes:
        o = mp.default_opts(mode == "mixed")
        o.kernel_timing = 100 + c
        info = mp.svd(A, mode, workspace=ws, opts=o)[3]
        torch.cuda.synchronize()
        if info["kern_calls"][c] > 0:
            out[c] = (info["kern_ms"][c], info["kern_calls"][c], info["kern_bytes"][c], info["kern_flops"][c])
    return out


def kernel_table(survey: dict, mp) -> list:
    """Per kernel class: launches, time, algorithmic bytes and flops per
    launch, achieved rates and the fraction of the roof that bounds the class
    (hbm: bytes against 8 TB/s; mfma: flops against the FP64 matrix peak;
    latency: flops against the FP64 peak, for scale only)."""
    rows = []
    for c, (ms, calls, byts, flops) in survey.items():
        name = mp.KERNEL_CLASSES[c]
        sec = ms / 1e3
        gbs = byts / sec / 1e9 if sec > 0 else 0.0
        tfs = flops / sec / 1e12 if sec > 0 else 0.0
        bound, fpk = CLASS_ROOF.get(name, ("hbm", None))
        frac = gbs / HBM_PEAK_GBS if bound == "hbm" else tfs / (fpk or FP64_PEAK_TF)
        rows.append({"kernel": name, "class": c, "launches": calls, "ms": round(ms, 3),
                     "avg_us": round(ms * 1e3 / calls, 2), "bytes_per_launch": round(byts / calls),
                     "flops_per_launch": round(flops / calls), "GB_s": round(gbs, 1),
                     "TFLOP_s": round(tfs, 3), "bound": bound, "frac": round(frac, 4)})
    rows.sort(key=lambda r: -r["ms"])
    return rows


def gates_gpu(A, U, S, V, s_ref, kappa_s):
    """The accuracy gates, evaluated with FP64 products on the GPU."""
    import torch
    n = A.shape[1]
    eye = torch.eye(n, dtype=torch.float64, device=A.device)
    orth_u = torch.linalg.norm(U.t() @ U - eye).item()
    orth_v = torch.linalg.norm(V.t() @ V - eye).item()
    res = (torch.linalg.norm(A - (U * S) @ V.t()) / torch.linalg.norm(A)).item()
    r = {"orth_u": orth_u, "orth_v": orth_v, "residual": res}
    if s_ref is not None:
        sref = torch.from_numpy(s_ref).to(A.device)
        rel = torch.max(torch.abs(S - sref) / sref).item()
        r["rel_sigma"] = rel
        r["e_sigma"] = rel / max(1.0, kappa_s)
    ok = orth_u <= 1e-13 * n and orth_v <= 1e-13 * n and res <= 1e-14 * n
    if "e_sigma" in r:
        ok = ok and r["e_sigma"] <= 1e-13
    r["pass"] = bool(ok)
    return r


def cpu_baseline(n_full: int, n_sample: int) -> dict:
    """The FP64 oracle timed on this host's cores on a bounded sample: the
    full oracle SVD (QRCP + LQ preconditioning, round-robin Jacobi on all
    cores) of the same construction at n_sample, scaled by (n_full /
    n_sample)^3 to one n_full SVD."""
    import oracle
    import testmats
    oracle.set_threads(os.cpu_count() or 1)
    A, _ = testmats.config_c3b(n=n_sample)
    t0 = time.perf_counter()
    _, _, _, info = oracle.svd(A, order="rr")
    dt = time.perf_counter() - t0
    scale = (n_full / n_sample) ** 3
    est = dt * scale
    return {
        "value": 1.0 / est, "unit": "SVD/s", "cores": oracle.max_threads(), "kind": "oracle",
        "sample": (f"full oracle SVD of the {n_sample}x{n_sample} instance of the same "
                   f"construction ({dt:.2f} s, {info['sweeps']} sweeps), scaled by "
                   f"({n_full}/{n_sample})^3 = {scale:.0f} to one {n_full}x{n_full} SVD"),
        "est_ms_per_svd": est * 1e3,
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--mode", choices=("both", "mixed", "plain"), default="both")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-survey", action="store_true",
                    help="skip the per-class clocked SVDs (no kernels table, no roofline)")
    ap.add_argument("--cpu-sample-n", type=int, default=1024)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr, flush=True)
        return 2

    import numpy as np
    import torch

    import paper_2209_04626_amd as mp
    import testmats

    n = args.n
    t0 = time.time()
    A_np, _ = testmats.config_c3b(n=n)
    print(f"[bench] generated {n}x{n} input in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    A = torch.from_numpy(np.ascontiguousarray(A_np)).to(dev)
    ws = mp.Workspace()
    opts_mixed = mp.default_opts(True)
    opts_plain = mp.default_opts(False)

    do_mixed = args.mode in ("both", "mixed")
    do_plain = args.mode in ("both", "plain")
    for _ in range(args.warmup):
        if do_mixed:
            mp.svd(A, "mixed", workspace=ws, opts=opts_mixed)
        if do_plain:
            mp.svd(A, "plain", workspace=ws, opts=opts_plain)
    torch.cuda.synchronize()
    print("[bench] warmup done", file=sys.stderr, flush=True)

    # per-class kernel times of one SVD of each kind (untimed): each class
    # clocked in an SVD of its own, HIP events around that class's launches
    # only; the GEMM class (many shapes) is listed but never picked
    survey = {}
    if do_mixed and not args.no_survey:
        survey["mixed"] = class_survey(mp, A, ws, "mixed", range(0, 8))
    if do_plain and not args.no_survey:
        survey["plain"] = class_survey(mp, A, ws, "plain", range(0, 9))
    kernels = {k: kernel_table(v, mp) for k, v in survey.items()}
    # the dominant kernel: the class with the largest total time in the mixed
    # step (the Jacobi kernels are clocked by events that their dispatch
    # records, so clocking them in the timed region costs no extra packets)
    dom_class = None
    if do_mixed and "mixed" in survey:
        dom_class = max(survey["mixed"].items(), key=lambda kv: kv[1][0])[0]
    print(f"[bench] class survey done; dominant class {dom_class}", file=sys.stderr, flush=True)

    # timed: K mixed SVDs (the step) with the dominant kernel clocked by HIP
    # events on the library's stream (the pivot pass as one interval per
    # pass); K plain SVDs without events
    opts_mixed.kernel_timing = 1 if dom_class == 6 else (100 + dom_class if dom_class is not None else 0)
    # a Jacobi class is clocked on every CLOCK_EVERY-th launch (a uniform
    # sample over rounds and sweeps) so that its events barely touch the step
    opts_mixed.kernel_timing_every = CLOCK_EVERY
    opts_plain.kernel_timing = 0
    infos, infos_p = [], []
    t_mixed = t_plain = None
    if do_mixed:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            Um, Sm, Vm, info = mp.svd(A, "mixed", workspace=ws, opts=opts_mixed)
            infos.append(info)
        torch.cuda.synchronize()
        t_mixed = (time.perf_counter() - t0) / args.steps
        print(f"[bench] mixed {t_mixed * 1e3:.1f} ms/SVD", file=sys.stderr, flush=True)

    # K plain SVDs on the same matrix
    if do_plain:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            Up, Sp, Vp, info_p = mp.svd(A, "plain", workspace=ws, opts=opts_plain)
            infos_p.append(info_p)
        torch.cuda.synchronize()
        t_plain = (time.perf_counter() - t0) / args.steps
        print(f"[bench] plain {t_plain * 1e3:.1f} ms/SVD", file=sys.stderr, flush=True)

    # context, not the metric: the plain path with the triangular-solve V of
    # Section 3.4 as well (a stronger FP64 baseline than accumulation)
    t_plain_vs, info_pv, g_plain_vs = None, None, None
    if do_plain and do_mixed:
        opts_pv = mp.default_opts(False, v_method=1)
        mp.svd(A, "plain", workspace=ws, opts=opts_pv)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            Upv, Spv, Vpv, info_pv = mp.svd(A, "plain", workspace=ws, opts=opts_pv)
        torch.cuda.synchronize()
        t_plain_vs = (time.perf_counter() - t0) / args.steps
        print(f"[bench] plain with solved V {t_plain_vs * 1e3:.1f} ms/SVD", file=sys.stderr, flush=True)

    # gates against the stored oracle sigma (when this size has one)
    s_ref, kappa = None, None
    if n == 4096:
        sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
        try:
            from make_oracle_sigma import fingerprint, load
            s_ref, kappa, fp, _ = load("C3b")
            if not np.allclose(fingerprint(A_np), fp, rtol=1e-12, atol=0):
                raise RuntimeError("regenerated input differs from the one the stored sigma is for")
        except FileNotFoundError:
            s_ref = None
    g_mixed = gates_gpu(A, Um, Sm, Vm, s_ref, kappa or 1.0) if do_mixed else None
    g_plain = gates_gpu(A, Up, Sp, Vp, s_ref, kappa or 1.0) if do_plain else None
    if t_plain_vs is not None:
        g_plain_vs = gates_gpu(A, Upv, Spv, Vpv, s_ref, kappa or 1.0)

    # roofline of the dominant kernel class of the mixed step, from the
    # clocked launches of the timed region
    roofline = None
    if do_mixed and dom_class is not None:
        c = dom_class
        ms = float(np.sum([i["kern_ms"][c] for i in infos]))
        calls = int(np.sum([i["kern_calls"][c] for i in infos]))
        byts = float(np.sum([i["kern_bytes"][c] for i in infos]))
        flops = float(np.sum([i["kern_flops"][c] for i in infos]))
        name = mp.KERNEL_CLASSES[c]
        avg_s = ms / 1e3 / max(calls, 1)
        bytes_per_launch = byts / max(calls, 1)
        bound, _ = CLASS_ROOF.get(name, ("hbm", None))
        traffic = recorded_traffic(n, name)
        if bound == "mfma":
            ach = flops / (ms / 1e3) / 1e12
            roofline = {"bound": "mfma", "achieved": round(ach, 2), "peak": FP64_PEAK_TF,
                        "unit": "TFLOP/s", "frac": round(ach / FP64_PEAK_TF, 4)}
        elif bound == "latency":
            # a chain of dependent LDS rounds: priced against the FP64 vector
            # ALU peak (256 CUs x 128 FP64 flop/clk x 2.4 GHz)
            ach = flops / (ms / 1e3) / 1e12
            roofline = {"bound": "alu", "achieved": round(ach, 3), "peak": FP64_PEAK_TF,
                        "unit": "TFLOP/s", "frac": round(ach / FP64_PEAK_TF, 4)}
        else:
            ach = bytes_per_launch / avg_s / 1e9
            roofline = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4)}
        roofline.update({
            "traffic": None if traffic is None else round(traffic),
            "kernel": name, "avg_us": round(avg_s * 1e6, 2), "launches": calls,
            "bytes_per_launch": round(bytes_per_launch),
            "measured": "timed region" + (f", every {CLOCK_EVERY}th launch" if c < 6 else ""),
        })

    line = {
        "metric": "n=4096 SVD time: mixed vs plain FP64 Jacobi, same GPU, sigma rel err <=1e-13",
        "value": round(t_plain / t_mixed, 4) if (t_plain and t_mixed) else None,
        "unit": "x (T_plain / T_mixed)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round((t_mixed or t_plain) * 1e3, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": f"C3b: {n}x{n} FP64, A = U diag(sigma) V^T, Haar U/V, "
                               f"sigma log-uniform in [1e-12, 1], seed 4; U and V formed",
                   "m": n, "n": n, "mode": args.mode},
    }
    if do_mixed:
        info = infos[-1]
        flops = algorithmic_flops(n, info, True)
        line.update({
            "mixed_ms": round(t_mixed * 1e3, 2), "mixed_svd_per_s": round(1.0 / t_mixed, 4),
            "mixed_gflops": round(flops / t_mixed / 1e9, 1),
            "mixed_info": {k: info[k] for k in ("status", "branch_taken", "sweeps_low", "sweeps_work",
                                                "orth", "cond_r", "v_method_taken", "orth_vx",
                                                "sweeps_vfix")},
            "mixed_off_trace": {"fp32": [float("%.3g" % x) for x in info["off_low"]],
                                "fp64": [float("%.3g" % x) for x in info["off_work"]]},
            "mixed_stage_ms": [round(x, 2) for x in info["stage_ms"]],
            "gates_mixed": g_mixed,
        })
    if do_plain:
        info_p = infos_p[-1]
        line.update({
            "plain_ms": round(t_plain * 1e3, 2), "plain_svd_per_s": round(1.0 / t_plain, 4),
            "plain_info": {k: info_p[k] for k in ("status", "sweeps_work")},
            "plain_stage_ms": [round(x, 2) for x in info_p["stage_ms"]],
            "gates_plain": g_plain,
        })
    if t_plain_vs is not None:
        line["plain_solved_v"] = {
            "ms": round(t_plain_vs * 1e3, 2), "ratio_to_mixed": round(t_plain_vs / t_mixed, 4),
            "info": {k: info_pv[k] for k in ("status", "sweeps_work", "v_method_taken", "orth_vx")},
            "stage_ms": [round(x, 2) for x in info_pv["stage_ms"]], "gates": g_plain_vs,
        }
    line["roofline"] = roofline
    line["kernels"] = kernels
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline ...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(n, args.cpu_sample_n)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
