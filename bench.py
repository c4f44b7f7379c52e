#!/usr/bin/env python3
"""Benchmark of the CISOR hot path on one MI355X.

A step is one relaxed-FISTA iteration (eqs. algo1-algo3) of the 256^2,
60-transmitter, 360-receiver strong-scattering workload: 60 forward
Lippmann-Schwinger solves to a true relative residual of 1e-6, the receiver
projection and misfit, the back-projection, 60 adjoint solves, the Prop. 1
gradient, the TV prox (100 FGP iterations) and the momentum update.  The
timed run is always the workload's whole reconstruction: its 100 steps from
f_0 = 0, whatever ``--steps`` asks (later iterations need more solver work, so
a shorter run would time a different workload; ``--iters`` truncates it for
profiling and the line then says so), after W untimed warm-up steps on a
separate state.  All inputs are seeded synthetic data resident on the GPU
before timing starts.

Headline value: CISOR iterations per second with every solve started from the
previous iterations' fields extrapolated along the FISTA path ("warm", start
mode 4).  The same K steps with the solves started from the previous
iteration's fields ("previous_fields", start mode 2) and from the first-Born
field ("plain") are timed beside it.  LS solves per second are
reported inside the run and, separately, for the hardest case: the 60 forward
solves on the true phantom from the zero and first-Born starts.

Further legs are reported inside the same JSON line (not in ``value``); a
leg that fails in Python is recorded as {"error": ...} and the line is still
printed:
  * ``expensive_regime``: the same starts compared from f_0 = f_true / 2,
    where every solve needs hundreds of BiCGSTAB iterations;
  * ``batched`` (only with ``--batched``): 32 independent problems with grids drawn from
    {64..512}^2 and 8-64 transmitters each, 50 relaxed-FISTA iterations
    stepped together through the batched API (grouped launches per grid,
    captured graphs, autotuned column kernels);
  * ``paper_geometry``: relaxed FISTA on the paper's layouts with point
    sources (a line of sources and two linear arrays; a ring with the
    receivers near each source switched off);
  * ``learned_warm_start``: the trained encoder-decoder's start against the
    zero and first-Born starts on held-out 128^2 phantoms (LS iterations and
    wall time to the same true residual), when its weights file is present.

Prints one JSON line.  ``--gpus`` above 1 is not supported (single-GPU build).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "CISOR iters/s and LS solves/s (256², 60 tx) at 1e-6 residual, plain vs warm-start"
HBM_PEAK_GBS = 8000.0
# Algorithmic HBM bytes of one BiCGSTAB iteration of one transmitter, in units
# of N = n^2 (complex64): stage A 72 (prologue reads s, t, x, p, v and writes
# x, p; the row FFTs write X1) + 32 (columns) + 40 (X2, p, rhat in; v out),
# stage B 48 (s, t, v in; s, X1 out) + 32 + 40 (X2, s, rhat in; t out).
SOLVE_BYTES_PER_TX_ITER_N = 264
FFT_LENGTHS = (64, 128, 192, 256, 384, 512, 768, 1024)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def stage_bytes(n, P, T, stage, real_bytes=4):
    """Algorithmic HBM bytes of one launch of a stage of y = A x (all T fields)."""
    c = 2 * real_bytes
    N = n * n
    if stage == 1:   # read x, f; write X1 [T][n][P]
        return T * N * c + N * real_bytes + T * n * P * c
    if stage == 2:   # read X1, write X2, read the kernel spectrum once
        return 2 * T * n * P * c + P * P * c
    return T * n * P * c + 2 * T * N * c + N * real_bytes   # read X2, x, f; write y


def column_stage_flops(n, P, T):
    """Algorithmic flops of one launch of the 2D column stage: for each of the
    P columns of every field, a forward and an inverse length-P FFT (counted
    as 5 P log2 P each, the usual convention, although the first and last
    passes are pruned) and the spectrum product (6 flops per entry)."""
    import math
    return T * P * (2 * 5 * P * math.log2(P) + 6 * P)


# FP32 vector peaks of the MI355X: published 157.3 TFLOP/s counts packed
# FP32 (two lanes per instruction); without packed instructions, which this
# library does not emit, one FMA per lane per clock on 256 CUs x 4 SIMDs x 16
# lanes at 2.4 GHz gives 78.6 TFLOP/s.
FP32_PEAK_TFLOPS = 157.3
FP32_NONPACKED_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12

# The full 32-problem batched run is kept off the GPU: its last run ended in a
# host segmentation fault, and no cause has been shown (the host orchestration
# is clean under AddressSanitizer and the stream/graph rule checks of
# tests/test_host_orchestration.py on the same recipe).
BATCHED_DISABLED = ("the 32-problem batched leg is disabled: its last full run ended in a host segmentation "
                    "fault whose cause is not identified (host orchestration clean on the CPU harness)")

COUNTER_PROFILE = os.path.join(ROOT, "profiles", "operator_stage_counters_strong_256.md")
KERNEL_SOURCES = ["paper_1708_01663_amd/csrc/conv_kernels.hpp", "paper_1708_01663_amd/csrc/conv_cfg.hpp",
                  "paper_1708_01663_amd/csrc/fft.hpp", "paper_1708_01663_amd/csrc/conv_p.hip"]


def measured_traffic(variant, n, T, key="traffic_bytes_per_launch_by_variant"):
    """HBM bytes per launch of the column stage from the committed counter
    profile (FETCH_SIZE + WRITE_SIZE, scaled by a copy of known size), if it
    was taken on this workload, this column variant and these kernel sources
    (key="valu_insts_per_launch_by_variant": its SQ_INSTS_VALU per launch)."""
    import hashlib
    try:
        text = open(COUNTER_PROFILE).read()
        block = json.loads(text.split("```json")[1].split("```")[0])
    except (OSError, IndexError, ValueError):
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if block.get("source_hash") != h.hexdigest()[:16] or (n, T) != (256, 60):
        return None
    return block.get(key, {}).get(str(variant))


def time_stages(op, f, x, reps=20):
    """Average duration (s) of each stage of y = A x, timed with HIP events
    recorded on the stream the stages are launched on (torch's current stream)."""
    import torch
    y = torch.empty_like(x)
    out = {}
    for stage in (1, 2, 3):
        for _ in range(3):
            op.apply_A_stage(f, x, y, stage)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(reps):
            op.apply_A_stage(f, x, y, stage)
        ev1.record()
        ev1.synchronize()
        out[stage] = ev0.elapsed_time(ev1) / 1e3 / reps
    return out


def cpu_baseline(w, f_state, y_meas_np, ftrue, tx=0, with_vec3d=False, with_apg=False):
    """The FP64 oracle, single-threaded, on a bounded sample of the workload:
    (a) one transmitter's share of a CISOR iteration at the mid-run state (forward
    and adjoint solves, projection, back-projection, G^H v) plus one full TV
    prox, scaled to the 60 transmitters; (b) one forward solve on the true
    phantom from the first-Born start."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import cisor as ocisor, operators, tv as otv
    with threadpool_limits(limits=1):
        prob = ocisor.make_problem_2d(w.n, w.h, w.T, w.M, w.rx_radius, eps_b=w.eps_b)
        sub = ocisor.Problem(n=w.n, h=w.h, dim=2, u_in=prob.u_in[tx:tx + 1], H=prob.H,
                             Ghat=prob.Ghat, k=prob.k, eps_b=w.eps_b)
        f = f_state.reshape(w.n, w.n).astype(np.float64)
        t0 = time.perf_counter()
        u, its_f = ocisor.solve_fields(sub, f, x0=sub.u_in, tol=w.ls_tol)
        y = ocisor.project(sub, f, u)
        wv = y - y_meas_np[tx:tx + 1]
        q = (np.conj(sub.H).T @ wv.T).T.reshape(u.shape)
        v, its_a = ocisor.solve_fields(sub, f, rhs=f * q, tol=w.ls_tol, adjoint=True)
        g = np.real(np.conj(u) * (q + operators.apply_GH(sub.Ghat, v))).sum(0)
        t1 = time.perf_counter()
        otv.prox_tv_box(f - 1e-3 * g, 1e-3 * w.tau, w.lo, w.hi, 100)
        t2 = time.perf_counter()
        _, its_t = ocisor.solve_fields(sub, ftrue, x0=sub.u_in, tol=w.ls_tol)
        t3 = time.perf_counter()
    per_tx = t1 - t0
    per_iter = w.T * per_tx + (t2 - t1)
    return dict(value=round(1.0 / per_iter, 6), unit="CISOR iter/s", cores=1, kind="oracle",
                sample=(f"FP64 numpy oracle, 1 thread: 1 of {w.T} transmitters of a CISOR iteration at "
                        f"the mid-run state (Born-start forward + zero-start adjoint BiCGSTAB to "
                        f"{w.ls_tol:g}: {int(its_f[0])} + {int(its_a[0])} iterations, projection, "
                        f"back-projection, G^H v) = {per_tx:.2f} s, plus one 100-iteration TV prox "
                        f"= {t2 - t1:.2f} s; per iteration {w.T} x {per_tx:.2f} + {t2 - t1:.2f} s. "
                        f"Hardest solve: 1 forward solve on the true phantom, Born start, "
                        f"{int(its_t[0])} iterations, {t3 - t2:.2f} s"),
                ls_solves_per_s_ftrue=round(1.0 / (t3 - t2), 4), seconds=round(t3 - t0, 2),
                vectorial_3d=cpu_baseline_vec3d() if with_vec3d else None,
                monotone_apg=cpu_baseline_apg(w, sub, f, y_meas_np[tx:tx + 1]) if with_apg else None)


def cpu_baseline_apg(w, sub, f, y_meas_1):
    """The FP64 oracle's monotone APG: one iteration on one transmitter's
    share (two gradients, two objective solves) and its two TV proxes, scaled
    to all transmitters."""
    from threadpoolctl import threadpool_limits

    from oracle import apg as oapg, tv as otv
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        oapg.cisor_apg(sub, y_meas_1, 1e-3, 1e-3, w.tau, K=1, lo=w.lo, hi=w.hi, inner=100, tol=w.ls_tol, f0=f)
        t1 = time.perf_counter()
        for _ in range(2):
            otv.prox_tv_box(f, 1e-3 * w.tau, w.lo, w.hi, 100)
        t2 = time.perf_counter()
    prox = t2 - t1
    per_iter = w.T * (t1 - t0 - prox) + prox
    return dict(value=round(1.0 / per_iter, 6), unit="APG iter/s", cores=1, kind="oracle",
                sample=(f"FP64 numpy oracle, 1 thread: one monotone APG iteration (gradients at y and x, objective "
                        f"at z and v, LS to {w.ls_tol:g}) on 1 of {w.T} transmitters from the mid-run state = "
                        f"{t1 - t0 - prox:.2f} s without its two TV proxes ({prox:.2f} s); per iteration "
                        f"{w.T} x {t1 - t0 - prox:.2f} + {prox:.2f} s"))


def cpu_baseline_vec3d(tx=0):
    """The FP64 oracle, single-threaded, on one transmitter of the vectorial
    3D workload (the same layout, mask row and object as the GPU leg; data
    y_meas = 0, which changes no step's cost), scaled to the 81 transmitters."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import vec3d as ovec
    from synth import fresnel3d_like_geometry, fresnel3d_like_sources, two_spheres_3d
    n, h, dirs, rx, mask = fresnel3d_like_geometry()
    with threadpool_limits(limits=1):
        prob = ovec.make_problem(n, h, None, rx, mask=mask[tx:tx + 1], src=fresnel3d_like_sources()[tx:tx + 1])
        f = 0.5 * two_spheres_3d(n, h)
        t0 = time.perf_counter()
        ovec.gradient(prob, f, np.zeros((1, rx.shape[0]), dtype=np.complex128), tol=1e-6)
        dt = time.perf_counter() - t0
    T = dirs.shape[0]
    return dict(value=round(1.0 / (T * dt), 6), unit="gradients/s", cores=1, kind="oracle",
                sample=(f"FP64 numpy oracle, 1 thread: the vectorial gradient (forward and adjoint BiCGSTAB to "
                        f"1e-6 from zero, projection, back-projection, G0^H (k^2 + D) V) for 1 of {T} "
                        f"transmitters on 32^3 = {dt:.2f} s, scaled x{T}"))


def batched_leg(steps, warmup, log):
    """The batched uneven workload: setup, data, autotune, then `steps` steps of
    every problem timed together."""
    import numpy as np
    import torch

    from paper_1708_01663_amd.cisor import Batch, SolveOpts, plane_wave_dirs, ring
    from synth import batched_uneven, complex_normal
    from synth.workloads import make_phantom

    ws = batched_uneven()
    specs = [dict(n=w.n, h=w.h, tx_dir=plane_wave_dirs(w.T), rx_pos=ring(w.M, w.rx_radius)) for w in ws]
    t0 = time.perf_counter()
    b = Batch(specs, precision="c64", autotune=True, reps=5)
    setup = time.perf_counter() - t0
    log(f"[batched] {len(ws)} problems in {b.groups} grid groups, setup {setup:.1f} s, column variants "
        f"{b.variants}")
    fs = [torch.tensor(make_phantom(w).ravel(), dtype=torch.float32, device="cuda") for w in ws]
    _, ys, its, code = b.forward(fs, SolveOpts(tol=1e-7, maxit=20000, start=1))
    log(f"[batched] data: forward on f_true, mean iterations {np.mean(np.concatenate(its)):.0f}, status {code}")
    data = []
    for p, w in enumerate(ws):
        y = ys[p].cpu().numpy().astype(np.complex128)
        sigma = np.linalg.norm(y) / np.sqrt(y.size) * 10 ** (-w.snr_db / 20.0)
        y_meas = torch.tensor(y + sigma * complex_normal(y.shape, w.seed + 1), dtype=torch.complex64, device="cuda")
        data.append((y_meas, 1.0 / b.born_lipschitz(p, 50), w.tau))

    def reset():
        for p, (y_meas, gamma, tau) in enumerate(data):
            b.set_problem(p, y_meas, gamma, tau)

    opts = SolveOpts(tol=1e-6, maxit=20000, start=2)
    reset()
    for _ in range(warmup):
        b.step(opts=opts)
    reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [b.step(opts=opts) for _ in range(steps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    solves = 2 * sum(w.T for w in ws) * steps
    ls_iters = sum(i["fwd_sum"] + i["adj_sum"] for st in infos for i in st)
    worst = max(i["relres"] for st in infos for i in st)
    log(f"[batched] {steps} steps of {len(ws)} problems in {dt:.2f} s: {len(ws) * steps / dt:.1f} problem-iterations/s, "
        f"{solves / dt:.0f} LS solves/s, mean LS iterations/solve {ls_iters / solves:.1f}, worst relres {worst:.1e}")
    from collections import Counter
    out = dict(problems=len(ws), grid_groups=b.groups, steps=steps, seconds=round(dt, 3),
               problem_iters_per_s=round(len(ws) * steps / dt, 3), ls_solves_per_s=round(solves / dt, 1),
               mean_ls_iters=round(ls_iters / solves, 2), max_true_relres=worst, setup_s=round(setup, 2),
               grids=dict(sorted(Counter(w.n for w in ws).items())), transmitters=sum(w.T for w in ws),
               column_variants=b.variants, start=opts.start,
               workload="32 problems, grids from {64,96,128,192,256,384,512}^2, 8-64 plane-wave Tx, M = 4T ring "
                        "receivers, random disks eps in [1.05,1.8], lambda/10, 30 dB, tau 5e-4, 50 iterations")
    b.close()
    return out


def paper_geometry_leg(log, steps=50):
    """The paper's experimental layouts (point sources; two linear arrays, or a
    ring with the receivers near each source switched off): relaxed FISTA from
    f_0 = 0 with the extrapolated start, timed like the headline run."""
    import numpy as np
    import torch

    from paper_1708_01663_amd.cisor import Cisor, Fista, SolveOpts
    from synth import complex_normal, ellipses_2d, fresnel_like_geometry, paper_sim_geometry

    out = {}
    n, h, tx, rx = paper_sim_geometry()
    setups = {"paper_sim_128": (n, h, tx, rx, None,
                                "128x128 at lambda/8 (120 cm at 7.49 cm), 25 line sources on x = -19.2 lambda at "
                                "-60..60 deg, two 169-sensor arrays at x = +-12.8 lambda; ellipse phantom eps in "
                                "[1, 1.5]")}
    n, h, tx, rx, mask = fresnel_like_geometry()
    setups["fresnel_like_128"] = (n, h, tx, rx, mask,
                                  "128x128 pixels of 1.2 mm at lambda 99.9 mm (the 150 mm region), 8 sources and 360 "
                                  "receivers on a 16.7-lambda circle, 119 receivers nearest each source off; ellipse "
                                  "phantom eps in [1, 1.5]")
    for name, (n, h, tx, rx, mask, desc) in setups.items():
        op = Cisor(n, h, None, rx, tx_pos=tx)
        op.autotune(reps=5)
        if mask is not None:
            op.set_rx_mask(mask)
        f_t = torch.tensor(ellipses_2d(n, 0, inner=5, eps_range=(1.0, 1.5)).ravel(), dtype=torch.float32,
                           device="cuda")
        _, y, _, code = op.forward(f_t, SolveOpts(tol=1e-7, maxit=20000, start=1))
        y_np = y.cpu().numpy().astype(np.complex128)
        sigma = np.linalg.norm(y_np) / np.sqrt(y_np.size) * 10 ** (-30.0 / 20.0)
        y_meas = torch.tensor(y_np + sigma * complex_normal(y_np.shape, 7), dtype=torch.complex64, device="cuda")
        gamma = 1.0 / op.born_lipschitz(50)
        opts = SolveOpts(tol=1e-6, maxit=20000, start=4)
        # three untimed steps: the extrapolated start's three depths (0, 1, 2)
        # capture their solver graphs outside the timed run
        warm = Fista(op, y_meas, gamma, 5e-4, opts=opts)
        for _ in range(3):
            warm.step()
        fi = Fista(op, y_meas, gamma, 5e-4, opts=opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        recs = [fi.step() for _ in range(steps)]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        iters = sum(r["fwd_sum"] + r["adj_sum"] for r in recs) / (2 * op.T * steps)
        out[name] = dict(iters_per_s=round(steps / dt, 2), ms_per_step=round(1e3 * dt / steps, 3), steps=steps,
                         T=op.T, M=op.M, mean_ls_iters=round(iters, 2), D_first=round(recs[0]["D"], 6),
                         D_last=round(recs[-1]["D"], 6), worst_status=max(r["status"] for r in recs),
                         workload=desc)
        log(f"[paper-geometry] {name}: {steps / dt:.1f} CISOR it/s, mean LS iterations {iters:.1f}, "
            f"D {recs[0]['D']:.4e} -> {recs[-1]['D']:.4e}")
    return out


def vec_bytes_per_tx_iteration(n, P, N):
    """Modelled HBM bytes of one BiCGSTAB iteration of one transmitter's
    vectorial system (3N complex128 unknowns): two convolutions of the three
    component fields and 23 field streams of the fused vector kernels (p update
    + f p: 5, v = A p with <rhat, v>: 4, s update + f s: 4, t = A s with its
    dots: 3, x and r update with its dots: 7).  A convolution streams 2 + 4 rho
    field-sized arrays (rho = P / n) where the y- and x-passes run fused per kz
    plane (power-of-two P up to 64 in FP64: the z-transforms in and out, the
    plane kernel's n^2 P read and write), else 2 + 4 rho + 4 rho^2 (the y- and
    x-passes through HBM on the padded grid)."""
    rho = P / n
    plane = P in (64,)
    conv = 2 + 4 * rho + (0 if plane else 4 * rho * rho)
    return int(3 * N * 16 * (2 * conv + 23))


def vectorial_3d_leg(log, reps=5):
    """The 3D vectorial model on the 3D experimental layout (81 plane waves from
    a sphere, 36 receivers on the azimuthal circle, receivers within 50 degrees
    of the transmitter off) with a two-spheres object on a 32^3 grid: gradient
    evaluations (forward and adjoint solves, projection, back-projection,
    gradient) from the first-Born start, complex128."""
    import numpy as np
    import torch

    from paper_1708_01663_amd.cisor import SolveOpts
    from paper_1708_01663_amd.vec3d import VecCisor
    from synth import complex_normal, fresnel3d_like_geometry, fresnel3d_like_sources, two_spheres_3d

    n, h, dirs, rx, mask = fresnel3d_like_geometry()
    op = VecCisor(n, h, None, rx, tx_pos=fresnel3d_like_sources())
    op.set_rx_mask(mask)
    ftrue = two_spheres_3d(n, h)
    fd_true = torch.tensor(ftrue.ravel(), dtype=torch.float64, device="cuda")
    _, y, its_true, code, _ = op.forward(fd_true, SolveOpts(tol=1e-8, maxit=20000, start=1))
    y_np = y.cpu().numpy()
    sigma = np.linalg.norm(y_np) / np.sqrt(y_np.size) * 10 ** (-30.0 / 20.0)
    y_meas = torch.tensor(y_np + sigma * complex_normal(y_np.shape, 11), dtype=torch.complex128, device="cuda")
    f = torch.tensor(0.5 * ftrue.ravel(), dtype=torch.float64, device="cuda")
    opts = SolveOpts(tol=1e-6, maxit=20000, start=1)
    op.grad(f, y_meas, opts)                       # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = [op.grad(f, y_meas, opts) for _ in range(reps)]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    its = recs[-1][2]
    tx_iters = int(its.sum())
    P = 64 if n <= 32 else 2 * n
    bpi = vec_bytes_per_tx_iteration(n, P, n ** 3)
    gbs = bpi * tx_iters / dt / 1e9
    g2 = op.grad(f, y_meas, SolveOpts(tol=1e-6, maxit=20000, start=2))
    # CISOR iterations on the vectorial model: relaxed FISTA with the 3D TV/box
    # prox from f_0 = 0, step half the Cauchy step of the Born linearisation at
    # 0 (gamma = ||g0||^2 / ||J g0||^2 / 2 with J g0 = Ht (g0 E_in))
    from paper_1708_01663_amd.vec3d import VecFista
    g0, D0, *_ = op.grad(torch.zeros_like(f), y_meas, opts)
    Jg = op.project(g0.contiguous(), op.uin())
    gamma = 0.5 * float(torch.sum(g0 * g0)) / float(torch.sum(torch.abs(Jg) ** 2))
    # tau scaled to the data (the dipoles' amplitude is arbitrary): tau TV(f_true) = D(0) / 100
    tv_true = float(np.sum(np.sqrt(sum(np.diff(ftrue, axis=a, append=ftrue.take([-1], axis=a)) ** 2
                                       for a in range(3)))))
    tau = 0.01 * D0 / tv_true
    K = 10
    VecFista(op, y_meas, gamma, tau, opts=SolveOpts(tol=1e-6, maxit=20000, start=2)).step()   # warm-up
    fi = VecFista(op, y_meas, gamma, tau, opts=SolveOpts(tol=1e-6, maxit=20000, start=2))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    frecs = [fi.step() for _ in range(K)]
    torch.cuda.synchronize()
    dtf = (time.perf_counter() - t0) / K
    out = dict(grad_evals_per_s=round(1.0 / dt, 3), ms_per_grad=round(1e3 * dt, 2), reps=reps,
               n=n, T=op.T, M=op.M, active_rx_per_tx=float(mask.sum(1).mean()),
               mean_ls_iters_fwd=round(float(its[:op.T].mean()), 2),
               mean_ls_iters_adj=round(float(its[op.T:].mean()), 2),
               max_ls_iters=int(its.max()), ls_iters_true_object=round(float(its_true.mean()), 2),
               D=recs[-1][1], status=int(max(r[3] for r in recs)),
               solve_path=dict(bytes_per_tx_iteration=bpi, tx_iterations=tx_iters, achieved_GBs=round(gbs, 1),
                               frac=round(gbs / HBM_PEAK_GBS, 4),
                               note="modelled bytes of the active systems' iterations over the whole gradient time"),
               restart_from_previous_fields_iters=int(g2[2].sum()),
               cisor=dict(iters_per_s=round(1.0 / dtf, 3), ms_per_iter=round(1e3 * dtf, 2), steps=K, gamma=gamma,
                          tau=tau, alpha=0.96, start=2,
                          mean_ls_iters=round(sum(r["fwd_sum"] + r["adj_sum"] for r in frecs) / (2 * op.T * K), 2),
                          D_first=frecs[0]["D"], D_last=frecs[-1]["D"], worst_status=max(r["status"] for r in frecs)),
               workload=("3D vectorial, 32^3 voxels of lambda/15.9 (4.7 mm at 74.9 mm), 81 electric dipoles on the "
                         "1.769 m sphere (azimuth 20..340/40, polar 30..150/15), 36 z-polarised Rx on the azimuthal "
                         "circle, Rx within 50 deg of the Tx off; two touching spheres eps 2.6 (f = 1.6); "
                         "gradient at f = f_true / 2, true residual 1e-6, first-Born start, complex128"))
    log(f"[vec3d] CISOR (relaxed FISTA, 3D TV prox): {1.0 / dtf:.2f} it/s, D {frecs[0]['D']:.4e} -> "
        f"{frecs[-1]['D']:.4e}, mean LS iterations {out['cisor']['mean_ls_iters']}")
    log(f"[vec3d] {1.0 / dt:.2f} gradients/s ({1e3 * dt:.1f} ms), LS iterations fwd {out['mean_ls_iters_fwd']} "
        f"adj {out['mean_ls_iters_adj']}, solve path {gbs:.0f} GB/s modelled ({100 * gbs / HBM_PEAK_GBS:.1f}% of 8 TB/s)")
    return out


def apg_comparison_leg(op, y_meas, gamma, w, opts_of, inner, steps, log):
    """Relaxed FISTA against the monotone APG of Li and Lin (the comparison of
    the paper's "Proposed Method" section) on the headline problem: the same
    gamma, tau and solve tolerance, both from f_0 = 0; wall time per iteration,
    solve passes and BiCGSTAB iterations per iteration, and the objective
    F = D + tau TV reached (FISTA's iterates are scored after the timed run)."""
    import torch

    from paper_1708_01663_amd.cisor import Apg, Fista, SolveOpts
    from paper_1708_01663_amd.diagnostics import objective
    checkpoints = sorted({k for k in (10, 25, steps // 2, steps) if 1 <= k <= steps})
    fi = Fista(op, y_meas, gamma, w.tau, alpha=w.alpha, lo=w.lo, hi=w.hi, inner=inner, opts=opts_of(4))
    saved, t_f, its_f = {}, [], 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(1, steps + 1):
        r = fi.step()
        its_f += r["fwd_sum"] + r["adj_sum"]
        t_f.append(time.perf_counter() - t0)
        if k in checkpoints:
            saved[k] = fi.f.clone()
    ap = Apg(op, y_meas, gamma, w.tau, lo=w.lo, hi=w.hi, inner=inner, opts=opts_of(1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_a, recs = [], []
    for k in range(1, steps + 1):
        recs.append(ap.step())
        t_a.append(time.perf_counter() - t0)
    F_f = {k: objective(op, saved[k], y_meas, w.tau, SolveOpts(tol=w.ls_tol, maxit=20000, start=1))[0]
           for k in checkpoints}
    F_a = [r["F"] for r in recs]
    k_t = max(1, steps // 2)
    target = F_f[k_t]
    k_a = next((k + 1 for k, F in enumerate(F_a) if F <= target), None)
    out = dict(
        steps=steps, target=dict(F=target, what=f"relaxed FISTA's F after {k_t} iterations"),
        relaxed_fista=dict(ms_per_iter=round(1e3 * t_f[-1] / steps, 3), solve_passes_per_iter=dict(fwd=1, adj=1),
                           ls_iters_per_iter=round(its_f / steps / w.T, 2),
                           F={str(k): F_f[k] for k in checkpoints},
                           seconds_to_target=round(t_f[k_t - 1], 4)),
        monotone_apg=dict(ms_per_iter=round(1e3 * t_a[-1] / steps, 3),
                          solve_passes_per_iter=dict(fwd=recs[-1]["fwd_solves"], adj=recs[-1]["adj_solves"]),
                          ls_iters_per_iter=round(sum(r["fwd_sum"] + r["adj_sum"] for r in recs) / steps / w.T, 2),
                          F={str(k): F_a[k - 1] for k in checkpoints},
                          took_accelerated=sum(r["took_z"] for r in recs),
                          iterations_to_target=k_a,
                          seconds_to_target=None if k_a is None else round(t_a[k_a - 1], 4)),
        note="BiCGSTAB iterations per iteration count forward + adjoint, per transmitter")
    ra, rf = out["monotone_apg"], out["relaxed_fista"]
    log(f"[apg] relaxed FISTA {rf['ms_per_iter']} ms/it, F({steps}) {F_f[steps]:.5e}, target reached in "
        f"{rf['seconds_to_target']} s; monotone APG {ra['ms_per_iter']} ms/it, F({steps}) {F_a[-1]:.5e}, "
        f"target after {k_a} iterations / {ra['seconds_to_target']} s; z taken {ra['took_accelerated']}/{steps}")
    return out


def cisor_3d_leg(log, steps=10):
    """CISOR on the scalar 3D workload (64^3 voxels at lambda/6, 16 plane waves
    on a 45-degree cone, 1024 receivers on a 32 x 32 plane below, random
    ellipsoids eps in [1, 1.3], 30 dB): relaxed FISTA with the 3D TV/box prox
    from f_0 = 0, start mode 4, complex64."""
    import numpy as np
    import torch

    from paper_1708_01663_amd.cisor import Cisor, Fista, SolveOpts, cone_dirs, plane_rx
    from synth import complex_normal, ellipsoids_3d
    n, h, T = 64, 1 / 6, 16
    hw = n * h / 2
    op = Cisor(n, h, cone_dirs(T), plane_rx(32, 2 * hw, -2 * hw))
    f_t = torch.tensor(ellipsoids_3d(n, 0).ravel(), dtype=torch.float32, device="cuda")
    _, y, its, _ = op.forward(f_t, SolveOpts(tol=1e-7, maxit=20000, start=1))
    y_np = y.cpu().numpy().astype(np.complex128)
    sigma = np.linalg.norm(y_np) / np.sqrt(y_np.size) * 10 ** (-30.0 / 20.0)
    y_meas = torch.tensor(y_np + sigma * complex_normal(y_np.shape, 5), dtype=torch.complex64, device="cuda")
    gamma = 1.0 / op.born_lipschitz(50)
    opts = SolveOpts(tol=1e-6, maxit=20000, start=4)
    warm = Fista(op, y_meas, gamma, 5e-4, opts=opts)       # untimed: the extrapolation depths 0, 1, 2
    for _ in range(3):
        warm.step()
    fi = Fista(op, y_meas, gamma, 5e-4, opts=opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = [fi.step() for _ in range(steps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    iters = sum(r["fwd_sum"] + r["adj_sum"] for r in recs) / (2 * T * steps)
    out = dict(iters_per_s=round(steps / dt, 3), ms_per_iter=round(1e3 * dt / steps, 2), steps=steps, T=T, M=op.M,
               mean_ls_iters=round(iters, 2), D_first=recs[0]["D"], D_last=recs[-1]["D"],
               worst_status=max(r["status"] for r in recs),
               workload="64^3 at lambda/6, 16 plane waves on a 45-degree cone, 1024 Rx on a 32x32 plane, random "
                        "ellipsoids eps in [1, 1.3], 30 dB, tau 5e-4, gamma 1/L_Born, LS 1e-6, c64")
    log(f"[cisor-3d] {steps / dt:.2f} CISOR it/s ({1e3 * dt / steps:.1f} ms), mean LS iterations {iters:.1f}, "
        f"D {recs[0]['D']:.4e} -> {recs[-1]['D']:.4e}")
    return out


def warm_start_leg(log, phantoms=64):
    """The learned warm start on held-out phantoms (see warmstart.evaluate)."""
    from paper_1708_01663_amd import warmstart
    if not os.path.exists(warmstart.DEFAULT_WEIGHTS):
        log("[warm-start] no weights file; leg skipped")
        return None
    op = warmstart.make_op()
    net = warmstart.WarmStartNet.load(warmstart.DEFAULT_WEIGHTS)
    warmstart.evaluate(op, net, range(200000, 200004))      # warm-up (allocation, first launches)
    res = warmstart.evaluate(op, net, range(100000, 100000 + phantoms))
    log(f"[warm-start] mean LS iterations zero {res['zero']['mean_iters']:.1f}, born {res['born']['mean_iters']:.1f}, "
        f"net {res['net']['mean_iters']:.1f}; net field error {res['net_rel_error_of_scattered_field']:.3f}")
    res["inference"] = warmstart.time_inference(op, net)
    log(f"[warm-start] inference on {res['inference']['batch']} fields: {res['inference']['ms']} ms, "
        f"{res['inference']['TFLOPs']} TFLOP/s BF16 ({100 * res['inference']['frac_bf16_peak']:.1f}% of 2.5 PFLOP/s)")
    res["workload"] = ("128x128, lambda/10, 16 plane-wave Tx, held-out seeded disk/ellipse phantoms eps in [1,2], "
                       "true residual 1e-6")
    return res


def _device_failure(e):
    """True for errors that mean the GPU itself failed (these end the run)."""
    code = getattr(e, "code", None)
    if code == -3:                                  # CISOR_E_DEVICE
        return True
    msg = str(e)
    return any(k in msg for k in ("HIP error", "hipError", "device-side", "Memory access fault"))


def guarded(name, fn, *a, **kw):
    """Run a side leg; a Python-level failure is recorded as {"error": ...}
    in the JSON instead of ending the run (a device failure still ends it)."""
    import traceback
    try:
        return fn(*a, **kw)
    except Exception as e:                          # noqa: BLE001
        if _device_failure(e):
            raise
        log(f"[bench] leg {name} failed: {type(e).__name__}: {e}")
        traceback.print_exc(file=sys.stderr)
        return {"error": f"{type(e).__name__}: {e}"}


def warm_vs_plain(legs, wsn, expensive):
    """The plain-vs-warm comparison in one place: LS solves/s and BiCGSTAB
    iterations per solve at the same 1e-6 true residual for every start, in the
    headline run (256^2 x 60), in the expensive regime, and for the learned
    network start with its fallback (128^2 x 16, the grid it is trained on)."""
    def pick(d, keys):
        if not isinstance(d, dict) or "error" in d:
            return None
        return {k: d[k] for k in keys if k in d}
    fista_keys = ("start", "ls_solves_per_s", "mean_ls_iters", "iters_per_s")
    out = {"headline_256": {k: pick(v, fista_keys) for k, v in legs.items()}}
    if isinstance(expensive, dict) and "error" not in expensive:
        out["expensive_regime_256"] = {k: pick(expensive.get(k), fista_keys)
                                       for k in ("warm", "previous_fields", "plain", "plain_zero")}
    if isinstance(wsn, dict) and "error" not in wsn:
        out["network_start_128"] = {k: {"ls_solves_per_s": round(wsn[k]["solves_per_s"], 1),
                                        "mean_ls_iters": round(wsn[k]["mean_iters"], 2)}
                                    for k in ("net", "zero", "born") if k in wsn}
        out["network_start_128"]["inference_ms_per_16_fields"] = wsn.get("inference", {}).get("ms")
    out["note"] = ("warm = starts from earlier solves (extrapolated fields, start 4; previous fields, start 2) "
                   "or from the trained network with the zero-start fallback (start 5); plain = first-Born "
                   "and zero starts; every solve ends at the same FP64 true residual 1e-6")
    return out


def sig(v, digits=4):
    """Round to significant digits (keeps small residuals such as 9.99e-07)."""
    if not isinstance(v, float) or v == 0.0 or v != v:
        return v
    return float(f"{v:.{digits}g}")


def sig_dict(d):
    return None if d is None else {k: sig(v, 6) for k, v in d.items()}


def column_stage_flops_pruned(n, P, T):
    """Flops of one launch of the 2D column stage in the textbook radix-2
    accounting with the pruning the kernels do: per column, a forward length-P
    FFT whose upper half input is zero (5 P log2 P - 2 P: the first stage's
    butterflies reduce to their twiddle products), the spectrum product (6 P)
    and an inverse FFT of which only n = P/2 outputs are kept (5 P log2 P - P:
    the last stage computes one output per butterfly)."""
    import math
    return T * P * (10 * P * math.log2(P) - 3 * P + 6 * P)


def expensive_regime_leg(op, y_meas, gamma, w, ftrue, inner, check_every, steps, log):
    """CISOR iterations where every solve is expensive: relaxed FISTA started
    at f_0 = f_true / 2 (solves from the zero start there take hundreds of
    BiCGSTAB iterations), with the extrapolated start (mode 4), the previous
    fields (mode 2) and the plain first-Born and zero starts; the same steps,
    the same true-residual tolerance.  Reports the reconstruction SNR beside
    the rates."""
    import numpy as np
    import torch

    from paper_1708_01663_amd.cisor import Fista, SolveOpts
    f0 = torch.tensor(0.5 * ftrue.ravel(), dtype=op.rdtype, device=op.device)
    nt = np.linalg.norm(ftrue)
    snr0 = 20 * np.log10(nt / np.linalg.norm(0.5 * ftrue))
    out = dict(steps=steps, f0="f_true / 2", recon_snr_db_at_f0=round(float(snr0), 3), gamma=gamma)
    for start, label in ((4, "warm"), (2, "previous_fields"), (1, "plain"), (0, "plain_zero")):
        fi = Fista(op, y_meas, gamma, w.tau, alpha=w.alpha, lo=w.lo, hi=w.hi, inner=inner, f0=f0,
                   opts=SolveOpts(tol=w.ls_tol, maxit=20000, start=start, check_every=check_every))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        recs = [fi.step() for _ in range(steps)]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        solves = 2 * w.T * steps
        its = sum(r["fwd_sum"] + r["adj_sum"] for r in recs)
        f = fi.f.cpu().numpy().astype(np.float64)
        snr = 20 * np.log10(nt / np.linalg.norm(f - ftrue.ravel()))
        out[label] = dict(start=start, iters_per_s=sig(steps / dt), ms_per_step=sig(1e3 * dt / steps),
                          ls_solves_per_s=sig(solves / dt), mean_ls_iters=sig(its / solves),
                          max_true_relres=sig(max(r["relres"] for r in recs)), D_first=sig(recs[0]["D"], 6),
                          D_last=sig(recs[-1]["D"], 6), recon_snr_db=sig(float(snr)),
                          worst_status=max(r["status"] for r in recs))
        log(f"[expensive] {label}: {steps / dt:.2f} CISOR it/s, mean LS iterations/solve {its / solves:.1f}, "
            f"D {recs[0]['D']:.4e} -> {recs[-1]['D']:.4e}, recon SNR {snr:.2f} dB")
    out["workload"] = (f"{w.name} from f_0 = f_true/2 ({steps} relaxed-FISTA iterations, gamma 1/L_Born, "
                       f"LS true residual {w.ls_tol:g})")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100,
                    help="requested step count; the headline always times the workload's whole reconstruction "
                         "(100 relaxed-FISTA iterations for strong_256), see --iters")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--iters", type=int, default=None,
                    help="override the headline iteration count (profiling only: the line then names a "
                         "truncated workload)")
    ap.add_argument("--workload", default="strong_256")
    ap.add_argument("--inner", type=int, default=100, help="FGP iterations per prox")
    ap.add_argument("--gamma-scale", type=float, default=1.0, help="gamma = scale / L_Born")
    ap.add_argument("--check-every", type=int, default=10, help="LS iterations between true-residual checks")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--start", type=int, default=4, choices=(1, 2, 4),
                    help="start mode of the headline run (4 extrapolated, 2 previous fields, 1 first-Born)")
    ap.add_argument("--no-plain", action="store_true", help="skip the comparison runs with the other starts")
    ap.add_argument("--batched", action="store_true",
                    help="the 32-problem batched workload: disabled (its last full run ended in a host "
                         "segmentation fault whose cause is not identified; the leg records why instead)")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched uneven workload")
    ap.add_argument("--batched-steps", type=int, default=50)
    ap.add_argument("--expensive-steps", type=int, default=10,
                    help="steps of the expensive-regime leg (from f_true / 2)")
    ap.add_argument("--no-expensive", action="store_true", help="skip the expensive-regime leg")
    ap.add_argument("--no-warm-start-net", action="store_true", help="skip the learned warm-start leg")
    ap.add_argument("--no-paper-geometry", action="store_true", help="skip the point-source geometries leg")
    ap.add_argument("--no-vec3d", action="store_true", help="skip the 3D vectorial leg")
    ap.add_argument("--no-apg", action="store_true", help="skip the monotone APG comparison")
    ap.add_argument("--vec3d-only", action="store_true",
                    help="run only the 3D vectorial leg and print its JSON (profiling hook)")
    ap.add_argument("--only", choices=("cisor3d", "paper-geometry"),
                    help="run only this leg and print its JSON (profiling hook)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only; --gpus {args.gpus} is not supported (the multi-GPU layout, "
              "transmitters sharded with one gradient all-reduce per iteration, is not implemented)",
              file=sys.stderr)
        sys.exit(2)
    if args.vec3d_only:
        print(json.dumps(vectorial_3d_leg(log, reps=args.steps)), flush=True)
        return
    if args.only:
        leg = cisor_3d_leg if args.only == "cisor3d" else paper_geometry_leg
        print(json.dumps(leg(log)), flush=True)
        return

    import numpy as np
    import torch

    from paper_1708_01663_amd.cisor import Cisor, Fista, SolveOpts, plane_wave_dirs, ring
    from synth import complex_normal
    from synth.workloads import WORKLOADS, make_phantom

    w = WORKLOADS[args.workload]
    K = w.iters if args.iters is None else args.iters
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    log(f"[bench] workload {w.name}: n={w.n} T={w.T} M={w.M} tol={w.ls_tol}; headline {K} iterations "
        f"(requested --steps {args.steps})")
    op = Cisor(w.n, w.h, plane_wave_dirs(w.T), ring(w.M, w.rx_radius), eps_b=w.eps_b,
               precision=w.precision, device=dev)
    variant, tune_ms = op.autotune(reps=10)
    log(f"[bench] column-stage autotune: variant {variant}, ms per launch {[round(t, 4) for t in tune_ms]}")
    ftrue = make_phantom(w)
    f_t = torch.tensor(ftrue.ravel(), dtype=op.rdtype, device=dev)
    _, y_clean, its, code = op.forward(f_t, SolveOpts(tol=w.ls_tol * 0.1, maxit=20000, start=1))
    log(f"[bench] data: forward on f_true, {its.mean():.0f} mean / {its.max()} max iterations, status {code}")
    y_np = y_clean.cpu().numpy().astype(np.complex128)
    sigma = np.linalg.norm(y_np) / np.sqrt(y_np.size) * 10 ** (-w.snr_db / 20.0)
    y_meas_np = y_np + sigma * complex_normal(y_np.shape, w.seed + 1)
    y_meas = torch.tensor(y_meas_np, dtype=op.cdtype, device=dev)
    L = op.born_lipschitz(50)
    gamma = args.gamma_scale / L
    log(f"[bench] L_Born = {L:.4e}, gamma = {gamma:.4e}")

    def fista(start):
        return Fista(op, y_meas, gamma, w.tau, alpha=w.alpha, lo=w.lo, hi=w.hi, inner=args.inner,
                     opts=SolveOpts(tol=w.ls_tol, maxit=20000, start=start, check_every=args.check_every))

    warm_fi = fista(args.start)
    for k in range(args.warmup):
        rec = warm_fi.step()
        log(f"[bench] warmup {k}: D={rec['D']:.5e}")
    del warm_fi

    mid = {}

    def run(start, label):
        fi = fista(start)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        recs = []
        for k in range(K):
            recs.append(fi.step())
            if k == max(1, K // 2) - 1 and "s" not in mid:
                mid["s"] = fi.s.clone()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        solves = 2 * w.T * K
        iters = sum(r["fwd_sum"] + r["adj_sum"] for r in recs)
        f = fi.f.cpu().numpy().astype(np.float64)
        snr = 20 * np.log10(np.linalg.norm(ftrue) / np.linalg.norm(f - ftrue.ravel()))
        log(f"[bench] {label}: {K} steps in {dt:.3f} s, D {recs[0]['D']:.4e} -> {recs[-1]['D']:.4e}, "
            f"mean LS iterations/solve {iters / solves:.2f}, worst relres {max(r['relres'] for r in recs):.2e}, "
            f"recon SNR {snr:.2f} dB")
        return dict(iters_per_s=K / dt, ms_per_step=1e3 * dt / K, seconds=dt,
                    ls_solves_per_s=solves / dt, mean_ls_iters=iters / solves,
                    max_true_relres=max(r["relres"] for r in recs), D_first=recs[0]["D"], D_last=recs[-1]["D"],
                    recon_snr_db=float(snr), worst_status=max(r["status"] for r in recs))

    labels = {4: "warm (extrapolated start)", 2: "previous-fields start", 1: "plain (first-Born start)",
              0: "plain (zero start)"}
    warm = run(args.start, labels[args.start])
    previous = None if args.no_plain or args.start == 2 else guarded("previous", run, 2, labels[2])
    plain = None if args.no_plain or args.start == 1 else guarded("plain", run, 1, labels[1])
    plain_zero = None if args.no_plain else guarded("plain_zero", run, 0, labels[0])
    apg_cmp = None if args.no_apg else guarded("apg", apg_comparison_leg,
        op, y_meas, gamma, w,
        lambda start: SolveOpts(tol=w.ls_tol, maxit=20000, start=start, check_every=args.check_every),
        args.inner, K, log)
    expensive = None if args.no_expensive else guarded("expensive", expensive_regime_leg, op, y_meas, gamma, w,
                                                       ftrue, args.inner, args.check_every, args.expensive_steps, log)

    # hardest solves: the 60 forward solves on the true phantom
    hard = {}
    for start, label in ((0, "zero"), (1, "born")):
        so = SolveOpts(tol=w.ls_tol, maxit=20000, start=start, check_every=args.check_every)
        op.forward(f_t, so, project=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, its, code = op.forward(f_t, so, project=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        hard[label] = dict(ls_solves_per_s=round(w.T / dt, 2), mean_iters=round(float(its.mean()), 1),
                           max_iters=int(its.max()), seconds=round(dt, 4), status=code,
                           tx_iterations=int(its.sum()))
        log(f"[bench] f_true solves, {label} start: {w.T / dt:.1f} solves/s, {its.mean():.0f} mean iterations")

    # roofline of the dominant operator stage, measured live with HIP events on
    # the stream it runs on: algorithmic bytes per launch / average launch time
    x = op.uin()
    st = time_stages(op, mid["s"], x)
    P = next(p for p in FFT_LENGTHS if p >= 2 * w.n)
    dom = max(st, key=st.get)
    rb = 4 if w.precision == "c64" else 8
    nbytes = stage_bytes(w.n, P, w.T, dom, rb)
    achieved = nbytes / st[dom] / 1e9
    colk = {0: "k_col", 1: "k_col", 2: "k_col", 3: "k_col", 4: "k_colw", 5: "k_colw", 6: "k_colb", 7: "k_colb",
            8: "k_colbn", 9: "k_colbw"}.get(variant, "k_col")
    names = {1: "k_row_fwd (stage 1: contrast x row FFTs)",
             2: f"{colk} (stage 2: column FFTs, x Ghat, inverse column FFTs; column variant {variant})",
             3: "k_row_inv (stage 3: inverse row FFTs, x - conv)"}
    log("[bench] stage times (us): " + ", ".join(f"{k}: {1e6 * v:.1f}" for k, v in st.items()))
    traffic = measured_traffic(variant, w.n, w.T) if dom == 2 else None
    roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic, kernel=names[dom],
                bytes_per_launch=nbytes, avg_launch_us=round(1e6 * st[dom], 2),
                stage_us={str(k): round(1e6 * v, 2) for k, v in st.items()},
                stage_frac={str(k): round(stage_bytes(w.n, P, w.T, k, rb) / v / 1e9 / HBM_PEAK_GBS, 4)
                            for k, v in st.items()},
                matvec_GBs=round(sum(stage_bytes(w.n, P, w.T, s, rb) for s in (1, 2, 3)) / sum(st.values()) / 1e9, 1),
                column_variant=variant, column_variant_ms=[round(t, 4) for t in tune_ms])
    if dom == 2 and w.precision == "c64":
        # secondary view: the column stage's FP32 vector arithmetic (pruned
        # transforms) against the published FP32 peak and the non-packed rate
        fl = column_stage_flops_pruned(w.n, P, w.T)
        tf = fl / st[dom] / 1e12
        roof["alu"] = dict(achieved=round(tf, 2), unit="TFLOP/s", flops_per_launch=int(fl),
                           peak=FP32_PEAK_TFLOPS, frac=round(tf / FP32_PEAK_TFLOPS, 4),
                           peak_nonpacked=round(FP32_NONPACKED_PEAK_TFLOPS, 1),
                           frac_nonpacked=round(tf / FP32_NONPACKED_PEAK_TFLOPS, 4),
                           note="pruned radix-2 accounting: 10 P log2 P + 3 P flops per column (forward with zero "
                                "upper half, spectrum product, inverse keeping n outputs); the library emits no "
                                "packed FP32, so the non-packed rate is the attainable one")
        valu = measured_traffic(variant, w.n, w.T, key="valu_insts_per_launch_by_variant")
        if valu:
            # VALU issue time of the launch (SQ_INSTS_VALU from the counter
            # profile, 4 cycles per wave64 instruction on 1024 SIMDs at 2.4 GHz)
            # as a fraction of the measured launch time
            issue_s = valu * 4 / (256 * 4) / 2.4e9
            roof["alu"].update(valu_insts_per_launch=valu, valu_issue_us=round(1e6 * issue_s, 2),
                               valu_issue_frac=round(issue_s / st[dom], 4))
        log(f"[bench] column stage: {achieved:.0f} GB/s ({100 * achieved / HBM_PEAK_GBS:.1f}% of 8 TB/s); "
            f"{tf:.1f} TFLOP/s pruned ({100 * tf / FP32_PEAK_TFLOPS:.0f}% of 157.3, "
            f"{100 * tf / FP32_NONPACKED_PEAK_TFLOPS:.0f}% of the non-packed rate)")

    # the whole solve path (BiCGSTAB iterations with their fused vector updates,
    # scalar steps, FP64 residual checks, masked tails) on the hardest solves:
    # modelled bytes per transmitter-iteration / wall time
    sb = SOLVE_BYTES_PER_TX_ITER_N * w.N * (1 if w.precision == "c64" else 2)
    hb = hard["born"]
    solve_gbs = sb * hb["tx_iterations"] / hb["seconds"] / 1e9
    solve_path = dict(bytes_per_tx_iteration=sb, tx_iterations=hb["tx_iterations"], seconds=hb["seconds"],
                      achieved_GBs=round(solve_gbs, 1), frac=round(solve_gbs / HBM_PEAK_GBS, 4),
                      solves="60 forward solves on the true phantom, first-Born start")
    log(f"[bench] solve path: {solve_gbs:.0f} GB/s modelled ({100 * solve_gbs / HBM_PEAK_GBS:.1f}% of 8 TB/s)")
    batched = None if args.no_batched else dict(disabled=BATCHED_DISABLED)
    wsn = None if args.no_warm_start_net else guarded("learned_warm_start", warm_start_leg, log)
    pgeo = None if args.no_paper_geometry else guarded("paper_geometry", paper_geometry_leg, log)
    vec3d = None if args.no_vec3d else guarded("vectorial_3d", vectorial_3d_leg, log)
    c3d = None if args.no_vec3d else guarded("cisor_3d", cisor_3d_leg, log)

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on a bounded sample ...")
        cpu = guarded("cpu_baseline", cpu_baseline, w, mid["s"].cpu().numpy(), y_meas_np, ftrue,
                      with_vec3d=isinstance(vec3d, dict) and "error" not in vec3d,
                      with_apg=isinstance(apg_cmp, dict) and "error" not in apg_cmp)
        if cpu and "sample" in cpu:
            log(f"[bench] oracle: {cpu['sample']}")

    truncated = "" if K == w.iters else f" (TRUNCATED: {K} of the workload's {w.iters} iterations)"
    out = {
        "metric": METRIC,
        "value": round(warm["iters_per_s"], 3),
        "unit": "CISOR iter/s",
        "n_gpus": 1,
        "steps": K,
        "steps_requested": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(warm["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64" if w.precision == "c64" else "c128",
        "data": "synthetic (seeded random-ellipse phantom, plane waves, ring receivers, 30 dB noise)",
        "config": {"workload": f"{w.name}: {w.n}x{w.n} grid, pixel lambda/{round(1 / w.h)}, {w.T} plane-wave Tx, "
                               f"{w.M} Rx ring, eps in [1,2], tau {w.tau:g}, alpha {w.alpha}, "
                               f"LS true residual {w.ls_tol:g}, FGP {args.inner}, {K} relaxed-FISTA iterations "
                               f"from f0=0{truncated}",
                   "n": w.n, "T": w.T, "M": w.M, "ls_tol": w.ls_tol, "gamma": gamma, "iterations": K},
        "ls_solves_per_s": round(warm["ls_solves_per_s"], 2),
        "warm": dict(sig_dict(warm), start=args.start),
        "previous_fields": sig_dict(previous) if previous is None or "error" not in previous else previous,
        "plain": sig_dict(plain) if plain is None or "error" not in plain else plain,
        "plain_zero": sig_dict(plain_zero) if plain_zero is None or "error" not in plain_zero else plain_zero,
        "expensive_regime": expensive,
        "apg_comparison": apg_cmp,
        "solve_path": solve_path,
        "ftrue_solves": hard,
        "warm_vs_plain": warm_vs_plain({"warm": warm, "previous_fields": previous, "plain": plain,
                                        "plain_zero": plain_zero}, wsn, expensive),
        "batched": batched,
        "learned_warm_start": wsn,
        "paper_geometry": pgeo,
        "vectorial_3d": vec3d,
        "cisor_3d": c3d,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
