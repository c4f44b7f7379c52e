"""Micro-benchmark of the three launches of the FFT-convolution operator.

Times each stage of y = A x (eq. A_def) for one geometry and column-kernel
variant with HIP events on the launch stream, and copies a buffer of known
size with torch (a reference kernel whose HBM bytes are exact, used to scale
hardware counters).  Prints one JSON line.  Meant to run under a profiler:

    python -m paper_1708_01663_amd.opbench --n 256 --T 60 --reps 20
"""

from __future__ import annotations

import argparse
import json

import numpy as np
import torch

from .cisor import COL_VARIANTS, Cisor, plane_wave_dirs, ring


def stage_bytes(n, P, T, stage, real_bytes=4):
    """Algorithmic HBM bytes of one launch of a 2D operator stage (all T fields)."""
    c = 2 * real_bytes
    N = n * n
    if stage == 1:   # read x, f; write X1 [T][n][P]
        return T * N * c + N * real_bytes + T * n * P * c
    if stage == 2:   # read X1, write X2, read the kernel spectrum once
        return 2 * T * n * P * c + P * P * c
    return T * n * P * c + 2 * T * N * c + N * real_bytes   # read X2, x, f; write y


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--T", type=int, default=60)
    ap.add_argument("--h", type=float, default=0.1)
    ap.add_argument("--M", type=int, default=360, help="receivers of the projection timing")
    ap.add_argument("--variant", type=int, default=-1, help="column variant (-1: every variant)")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--copy-mib", type=int, default=512, help="size of the calibration copy (0: none)")
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    n, T = args.n, args.T
    op = Cisor(n, args.h, plane_wave_dirs(T), ring(8, n * args.h))
    rng = np.random.default_rng(0)
    f = torch.tensor(rng.uniform(0, 1, n * n), dtype=torch.float32, device="cuda")
    x = torch.tensor((rng.standard_normal((T, n * n)) + 1j * rng.standard_normal((T, n * n))).astype(np.complex64),
                     device="cuda")
    y = torch.empty_like(x)
    P = op.P
    variants = range(COL_VARIANTS) if args.variant < 0 else [args.variant]
    out = dict(n=n, T=T, P=P, reps=args.reps, stages={})
    for v in variants:
        op.set_col_variant(v)
        for stage in (1, 2, 3):
            if stage != 2 and v != list(variants)[0]:
                continue
            for _ in range(2):
                op.apply_A_stage(f, x, y, stage)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(args.reps):
                op.apply_A_stage(f, x, y, stage)
            e1.record()
            e1.synchronize()
            us = 1e3 * e0.elapsed_time(e1) / args.reps
            nb = stage_bytes(n, P, T, stage)
            key = f"stage{stage}" + (f"_v{v}" if stage == 2 else "")
            out["stages"][key] = dict(us=round(us, 2), bytes=nb, GBs=round(nb / us / 1e3, 1))
    # receiver projection (complex GEMM on matrix cores) and back-projection
    opm = Cisor(n, args.h, plane_wave_dirs(T), ring(args.M, n * args.h))
    w = torch.tensor((rng.standard_normal((T, args.M)) + 1j * rng.standard_normal((T, args.M))).astype(np.complex64),
                     device="cuda")
    for name, fn in (("project", lambda: opm.project(f, x)), ("backproject", lambda: opm.backproject(w))):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.reps):
            fn()
        e1.record()
        e1.synchronize()
        us = 1e3 * e0.elapsed_time(e1) / args.reps
        flop = 8.0 * args.M * n * n * T
        out["stages"][name] = dict(us=round(us, 2), TFLOPs=round(flop / us / 1e6, 1))
    if args.copy_mib > 0:
        a = torch.empty(args.copy_mib << 20, dtype=torch.uint8, device="cuda").fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        out["copy_bytes_each_way"] = args.copy_mib << 20
        # the runtime's device-to-device copy of the same buffer, timed like the
        # stages: a measured HBM rate (read + write) to set the stages against
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.reps):
            b.copy_(a)
        e1.record()
        e1.synchronize()
        us = 1e3 * e0.elapsed_time(e1) / args.reps
        out["copy_us"] = round(us, 2)
        out["copy_GBs"] = round(2.0 * (args.copy_mib << 20) / us / 1e3, 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
