"""Calibration run for the HBM byte counters: a plain device-to-device copy
of a known size (torch's elementwise copy kernel), repeated a few times.

Under ``rocprofv3 --pmc FETCH_SIZE`` (then ``WRITE_SIZE``) each copy should
read (write) ``--mib`` MiB; the ratio of the known size to the counter reading
is the factor that converts the counters into bytes for the other kernels
profiled the same way.

    python3 -m paper_2209_04626_amd.hbm_calib [--mib 1024] [--reps 3]
"""
from __future__ import annotations

import argparse
import sys


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    import torch
    n = args.mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(args.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {args.reps} x {args.mib} MiB ({n * 4} bytes read and written per copy)", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
