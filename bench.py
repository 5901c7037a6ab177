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
CLOCK_EVERY = 8                # sampled clocking of the dominant kernel class
FP64_PEAK_TF = 78.6            # dense FP64 (vector and MFMA)
FP32_PEAK_TF = 157.3           # dense FP32 (vector and MFMA)


def algorithmic_flops(n: int, info: dict, mixed: bool, m: int | None = None) -> float:
    """Algorithmic flop count of one SVD (m x n, U and V formed), from the
    stage formulas: tall QR 2mn^2 - 2n^3/3 and its back-transform 4mn^2 - 2n^3
    (m > n only), pivot pass 4n^3/3, QR of A1 P 4n^3/3, LQ 4n^3/3, branch
    SYRK n^3, FP32 sweeps 4n^2(n-1) each, switch 4.7 n^3, FP64 sweeps with V
    7n^2(n-1) each (without V 4n^2(n-1) each, then the triangular solve for
    V_X n^3; its fallback adds X^T U_X 2n^3, a QR 4n^3/3, X Q 2n^3 and sweeps
    with V), back-transforms 4n^3."""
    f = 4 * n ** 3 / 3 * 3 + 4 * n ** 3
    if m is not None and m > n:
        f += 2 * m * n ** 2 - 2 * n ** 3 / 3 + 4 * m * n ** 2 - 2 * n ** 3
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
    "qr_panel": ("qr_panel_coop_n4096_traffic.md",
                 ["paper_2209_04626_amd/csrc/qr.hip", "paper_2209_04626_amd/csrc/common.hpp"]),
    "jac_round<f32>": ("jac_round_f32_n4096_traffic.md",
                       ["paper_2209_04626_amd/csrc/jacobi.hip", "paper_2209_04626_amd/csrc/common.hpp"]),
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
    # the fused FP32 round: its Gram and update products on the FP32 matrix
    # cores, its inner solve a chain of dependent LDS rounds
    "jac_round<f32>": ("mfma", FP32_PEAK_TF),
    "trsm_diag": ("latency", FP64_PEAK_TF),
    # the same round on BF16 storage (BF16 Gram products, FP32 update)
    "jac_round<bf16>": ("mfma", FP32_PEAK_TF),
}
GEMM_CLASS = 8                 # many shapes in one class: listed, never the dominant kernel
SURVEY_CLASSES = range(0, 12)


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
        peak = HBM_PEAK_GBS if bound == "hbm" else (fpk or FP64_PEAK_TF)
        rows.append({"kernel": name, "class": c, "launches": calls, "ms": round(ms, 3),
                     "avg_us": round(ms * 1e3 / calls, 2), "bytes_per_launch": round(byts / calls),
                     "flops_per_launch": round(flops / calls), "GB_s": round(gbs, 1),
                     "TFLOP_s": round(tfs, 3), "bound": bound, "peak": peak, "frac": round(frac, 4)})
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


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_full(n_full: int, n_one: int) -> dict:
    """The oracle measured without extrapolation: one full SVD of the n_full
    workload on all host cores (round-robin ordering, OpenMP over the pairs of
    a round), and one SVD of the n_one instance on one thread (row-cyclic
    ordering).  Minutes of CPU time: run separately (--cpu-full), not in the
    default bench line."""
    import oracle
    import testmats
    out = {"cpu_model": cpu_model(), "host_threads": os.cpu_count()}
    oracle.set_verbose(True)
    oracle.set_threads(os.cpu_count() or 1)
    A, _ = testmats.config_c3b(n=n_full)
    t0 = time.perf_counter()
    _, _, _, info = oracle.svd(A, order="rr")
    out["all_cores"] = {"n": n_full, "threads": oracle.max_threads(), "order": "round-robin",
                        "s": round(time.perf_counter() - t0, 2), "sweeps": info["sweeps"]}
    print(f"[bench] oracle n={n_full} all cores {out['all_cores']['s']} s", file=sys.stderr, flush=True)
    oracle.set_threads(1)
    A, _ = testmats.config_c3b(n=n_one)
    t0 = time.perf_counter()
    _, _, _, info = oracle.svd(A, order="cyclic")
    out["one_thread"] = {"n": n_one, "threads": 1, "order": "cyclic",
                         "s": round(time.perf_counter() - t0, 2), "sweeps": info["sweeps"]}
    return out


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
        "est_ms_per_svd": est * 1e3, "cpu_model": cpu_model(),
        "measured_full": recorded_cpu_full(),
    }


def recorded_cpu_full():
    """The oracle's full-size run on the same kind of host, measured once with
    --cpu-full and recorded in profiles/oracle_cpu_n4096.md (None if absent)."""
    path = os.path.join(ROOT, "profiles", "oracle_cpu_n4096.md")
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as fh:
        for line in fh:
            m = re.match(r"^- (\w+): `?([^`\s]+)`?", line.strip())
            if m:
                rec[m.group(1)] = m.group(2)
    try:
        return {"n4096_all_cores_s": float(rec["all_cores_s"]), "n1024_one_thread_s": float(rec["one_thread_s"]),
                "source": "profiles/oracle_cpu_n4096.md"}
    except (KeyError, ValueError):
        return None


def secondary(mp, ws, steps: int) -> dict:
    """The other workloads, timed the same way (inputs resident in HBM,
    synchronised around the timed calls): the 1024^2 graded matrix and the
    8192 x 2048 tall matrix (mixed and plain, gates against the stored oracle
    sigma), the ragged batch of 2000 (graph replays of the persistent
    kernel), and the adjoint of 256 128 x 64 SVDs."""
    import numpy as np
    import torch
    import testmats
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    from make_oracle_sigma import load
    out = {}
    gens = {"C2": testmats.config_c2, "C3a": testmats.config_c3a}
    for name, gen in gens.items():
        A_np, _ = gen()
        A = torch.from_numpy(np.ascontiguousarray(A_np)).cuda()
        m, n = A_np.shape
        s_ref, kappa, _, _ = load(name)
        row = {"m": m, "n": n}
        for mode in ("mixed", "plain"):
            mp.svd(A, mode, workspace=ws)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                U, S, V, info = mp.svd(A, mode, workspace=ws)
            torch.cuda.synchronize()
            t = (time.perf_counter() - t0) / steps
            g = gates_gpu(A, U, S, V, s_ref, kappa)
            row[mode] = {"ms": round(t * 1e3, 2), "svd_per_s": round(1.0 / t, 3),
                         "gflops": round(algorithmic_flops(n, info, mode == "mixed", m) / t / 1e9, 1),
                         "sweeps_low": info["sweeps_low"], "sweeps_work": info["sweeps_work"],
                         "branch_taken": info["branch_taken"], "gates_pass": g["pass"],
                         "e_sigma": g.get("e_sigma")}
        row["ratio"] = round(row["plain"]["ms"] / row["mixed"]["ms"], 4)
        out[name] = row
        print(f"[bench] {name}: mixed {row['mixed']['ms']} ms, plain {row['plain']['ms']} ms",
              file=sys.stderr, flush=True)
        del A
    # the ragged batch: one persistent launch per graph replay
    shapes, mats, _ = testmats.config_c4()
    plan = mp.batched_plan(shapes)
    Ab = mp.pack_batch(mats, "cuda")
    res = mp.svd_batched(plan, Ab)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = mp.svd_batched(plan, Ab, out=res)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    info = res[3].cpu().numpy()
    flops = 0.0
    for (m, n), inf in zip(shapes, info):
        sw_low, sw_work = int(inf[2]), int(inf[3])
        f = 4 * n ** 3 / 3 * 3 + n ** 3 + 4.7 * n ** 3 + 4 * n ** 3
        f += sw_low * 4 * n * n * (n - 1) + sw_work * 7 * n * n * (n - 1)
        if m > n:
            f += 2 * m * n * n - 2 * n ** 3 / 3 + 4 * m * n * n - 2 * n ** 3
        flops += f
    ach = flops / t / 1e12
    out["C4"] = {"batch": len(shapes), "ms": round(t * 1e3, 2), "svd_per_s": round(len(shapes) / t, 1),
                 "gflops": round(flops / t / 1e9, 1), "all_ok": bool(np.all(info[:, 0] == 0)),
                 "roofline": {"bound": "mfma", "achieved": round(ach, 3), "peak": FP64_PEAK_TF,
                              "unit": "TFLOP/s", "frac": round(ach / FP64_PEAK_TF, 4)}}
    print(f"[bench] C4: {out['C4']['ms']} ms per batch", file=sys.stderr, flush=True)
    # the adjoint of the gradient workload: forward by the batched path,
    # then svd_backward timed alone
    d = testmats.config_c5(batch=256, ndir=1)
    plan = mp.batched_plan([M.shape for M in d["A"]])
    S, U, V, _ = mp.svd_batched(plan, mp.pack_batch(d["A"], "cuda"))
    outs = mp.unpack_batch(plan, S, U, V)
    Ut = torch.stack([o[0] for o in outs]).contiguous()
    St = torch.stack([o[1] for o in outs]).contiguous()
    Vt = torch.stack([o[2] for o in outs]).contiguous()
    gU, gS, gV = (torch.from_numpy(d[k]).cuda() for k in ("gU", "gS", "gV"))
    mp.svd_backward(Ut, St, Vt, gU, gS, gV)
    torch.cuda.synchronize()
    reps = max(steps, 10)
    t0 = time.perf_counter()
    for _ in range(reps):
        mp.svd_backward(Ut, St, Vt, gU, gS, gV)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    B, m, n = Ut.shape
    flops = B * (6.0 * m * n * n + 2.0 * n ** 3)          # J, Z = U M, gA = Z V^T; K
    byts = B * (3.0 * m * n + 2.0 * n * n + 2.0 * n) * 8   # U, gU, gA; V, gV; S, gS
    out["C5"] = {"batch": B, "m": m, "n": n, "backward_us": round(t * 1e6, 1),
                 "gflops": round(flops / t / 1e9, 1), "GB_s": round(byts / t / 1e9, 1),
                 "roofline": {"bound": "mfma", "achieved": round(flops / t / 1e12, 3),
                              "peak": FP64_PEAK_TF, "unit": "TFLOP/s",
                              "frac": round(flops / t / 1e12 / FP64_PEAK_TF, 4)}}
    print(f"[bench] C5: backward {out['C5']['backward_us']} us per batch", file=sys.stderr, flush=True)
    return out


def graph_replay(mp, A, ws, steps: int, s_ref, kappa) -> dict:
    """The step's svd_mixed in the stream-ordered mode (capture=1: no host
    synchronisation, decisions on the device), eagerly and captured once in
    a HIP graph and replayed.  Every sweep up to the caps (30 and 30) is
    enqueued; those after the device-side stop exit at once."""
    import torch
    o = mp.default_opts(True, capture=1, y2_safeguard=0)
    out = mp.svd(A, "mixed", workspace=ws, opts=o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        mp.svd(A, "mixed", workspace=ws, opts=o, out=out)
    torch.cuda.synchronize()
    t_eager = (time.perf_counter() - t0) / steps
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        mp.svd(A, "mixed", workspace=ws, opts=o, out=out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        mp.svd(A, "mixed", workspace=ws, opts=o, out=out)
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    t_graph = (time.perf_counter() - t0) / steps
    info = out[3].read()
    gates = gates_gpu(A, out[0], out[1], out[2], s_ref, kappa or 1.0)
    del g
    print(f"[bench] stream-ordered mixed: eager {t_eager * 1e3:.1f} ms, graph replay "
          f"{t_graph * 1e3:.1f} ms", file=sys.stderr, flush=True)
    return {"eager_ms": round(t_eager * 1e3, 2), "graph_replay_ms": round(t_graph * 1e3, 2),
            "caps": [o.maxsweep_low, o.maxsweep_work],
            "info": {k: info[k] for k in ("status", "branch_taken", "sweeps_low", "sweeps_work",
                                          "v_method_taken")},
            "gates": gates}


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
    ap.add_argument("--cpu-sample-n", type=int, default=2048)
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the other workloads (1024^2 graded, 8192 x 2048, batch, adjoint)")
    ap.add_argument("--cpu-full", action="store_true",
                    help="only measure the oracle on the host: a full SVD at --n on all cores and "
                         "the 1024^2 instance on one thread (minutes); prints one JSON line")
    args = ap.parse_args()
    if args.cpu_full:
        print(json.dumps({"cpu_full": cpu_full(args.n, 1024)}), flush=True)
        return 0
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
        survey["mixed"] = class_survey(mp, A, ws, "mixed", SURVEY_CLASSES)
    if do_plain and not args.no_survey:
        survey["plain"] = class_survey(mp, A, ws, "plain", SURVEY_CLASSES)
    kernels = {k: kernel_table(v, mp) for k, v in survey.items()}
    # the dominant kernel: the class with the largest total time in the mixed
    # step (the Jacobi kernels are clocked by events that their dispatch
    # records, so clocking them in the timed region costs no extra packets)
    dom_class = None
    if do_mixed and "mixed" in survey:
        cand = {c: v for c, v in survey["mixed"].items() if c != GEMM_CLASS}
        dom_class = max(cand.items(), key=lambda kv: kv[1][0])[0]
    print(f"[bench] class survey done; dominant class {dom_class}", file=sys.stderr, flush=True)

    # timed: K mixed SVDs (the step) with the dominant kernel clocked by HIP
    # events on the library's stream (the pivot pass as one interval per
    # pass); K plain SVDs without events
    opts_mixed.kernel_timing = 1 if dom_class == 6 else (100 + dom_class if dom_class is not None else 0)
    # the class is clocked on every CLOCK_EVERY-th launch (a uniform sample
    # over rounds and sweeps, or over the panels of each QR) so that its
    # events barely touch the step
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

    # the three-precision variant: the first FP32-stage sweeps on a BF16 Y
    # (BF16 Gram products), at most k of them
    three = None
    if do_mixed and not args.no_secondary:
        three = {}
        for k, hs in ((0, 0), (6, 0), (4, 1)):
            o3 = mp.default_opts(True, half_sweeps=k, half_storage=hs)
            mp.svd(A, "mixed", workspace=ws, opts=o3)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                U3, S3, V3, i3 = mp.svd(A, "mixed", workspace=ws, opts=o3)
            torch.cuda.synchronize()
            t3 = (time.perf_counter() - t0) / args.steps
            three[f"half_sweeps={k}" + (",bf16_storage" if hs else "")] = {"ms": round(t3 * 1e3, 2),
                             "info": {q: i3[q] for q in ("status", "sweeps_half", "sweeps_low",
                                                         "sweeps_work", "n_y2", "sweeps_y2")},
                             "stage_ms": [round(x, 2) for x in i3["stage_ms"]],
                             "out": (U3, S3, V3)}
            print(f"[bench] three-precision half_sweeps={k} storage={hs}: {t3 * 1e3:.1f} ms/SVD",
                  file=sys.stderr, flush=True)

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
    if three:
        for v in three.values():
            v["gates"] = gates_gpu(A, *v.pop("out"), s_ref, kappa or 1.0)

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
        bound, fpk = CLASS_ROOF.get(name, ("hbm", None))
        traffic = recorded_traffic(n, name)
        if bound == "mfma":
            ach = flops / (ms / 1e3) / 1e12
            roofline = {"bound": "mfma", "achieved": round(ach, 2), "peak": fpk,
                        "unit": "TFLOP/s", "frac": round(ach / fpk, 4)}
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
            "measured": "timed region" + (f", every {CLOCK_EVERY}th launch" if c != 6 else ""),
        })
        if name == "qr_panel":
            # a chain of 32 dependent column steps, each ending in one
            # cross-workgroup exchange: the launch time per column step
            roofline["latency"] = {"steps_per_launch": 32, "us_per_step": round(avg_s * 1e6 / 32, 2)}

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
    if three:
        line["three_precision"] = three
    line["roofline"] = roofline
    line["kernels"] = kernels
    if do_mixed and do_plain and not args.no_secondary:
        line["secondary"] = secondary(mp, ws, args.steps)
        line["secondary"]["C3b_stream_ordered"] = graph_replay(mp, A, ws, args.steps, s_ref, kappa)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline ...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(n, args.cpu_sample_n)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
