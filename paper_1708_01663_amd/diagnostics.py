"""Convergence diagnostics of relaxed FISTA (Prop. 3), computed on the GPU.

* ``objective``: F(f) = D(f) + tau TV(f) (eq. objective_func; the box
  indicator is zero on the iterates, which the prox keeps in the box), from
  one forward solve, the projection's FP64 misfit (eq. D_def) and
  ``cisor_tv_value``.
* ``gradient_mapping_norm``: ||G_gamma(f)|| with
  G_gamma(f) = (f - prox_{gamma R}(f - gamma grad D(f))) / gamma
  (eq. gradient_mapping_def), from one gradient evaluation (forward and
  adjoint solves) and one prox.  It vanishes exactly at stationary points.
* ``rate_bound``: the right-hand side of eq. convergence_rate.
* ``alpha_sweep``: relaxed FISTA for several alpha with F and ||G_gamma||
  recorded along the run.  This is the alpha comparison the paper makes on
  measured data, run here on a synthetic workload.

The diagnostics cost extra solves per evaluation (the paper's point about
methods that need them at every iteration), so they run beside the iteration,
every ``every`` steps, and their time is reported separately.

    python -m paper_1708_01663_amd.diagnostics --workload strong_256 --K 100 --every 10
"""

from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from .cisor import Cisor, Fista, SolveOpts, plane_wave_dirs, ring


def objective(op: Cisor, f, y_meas, tau, opts=None):
    """(F, D, TV) at f."""
    opts = opts or SolveOpts(tol=1e-6, start=1)
    u, _, _, _ = op.forward(f, opts, project=False)
    _, D = op.project(f, u, y_meas)
    tv = op.tv_value(f)
    return D + tau * tv, D, tv


def gradient_mapping_norm(op: Cisor, f, y_meas, gamma, tau, lo=0.0, hi=2.0, inner=100, opts=None):
    g, _, _, _, _, _ = op.grad(f, y_meas, opts or SolveOpts(tol=1e-6, start=1))
    x = op.tv_prox((f - gamma * g).contiguous(), gamma * tau, lo, hi, inner)
    return float(torch.linalg.vector_norm((f - x).double()) / gamma)


def rate_bound(L, gamma, F0, Fstar, K):
    """Bound on min_{k <= K} ||G_gamma(f_k)||^2 for gamma <= (1 - alpha^2)/(2L)."""
    return 2 * L * (3 + gamma * L) ** 2 * (F0 - Fstar) / (K * gamma * L * (1 - gamma * L))


def alpha_sweep(op: Cisor, y_meas, gamma, tau, alphas, K, every=10, lo=0.0, hi=2.0, inner=100, tol=1e-6, start=4):
    """{alpha: {"history": [{k, F, D, TV, gmap}], "step_seconds", "diag_seconds"}}."""
    dopts = SolveOpts(tol=tol, start=1)
    out = {}
    for a in alphas:
        fi = Fista(op, y_meas, gamma, tau, alpha=a, lo=lo, hi=hi, inner=inner, opts=SolveOpts(tol=tol, start=start))
        hist, t_step, t_diag = [], 0.0, 0.0
        for k in range(1, K + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rec = fi.step()
            torch.cuda.synchronize()
            t_step += time.perf_counter() - t0
            if k == 1 or k % every == 0:
                t0 = time.perf_counter()
                F, D, tv = objective(op, fi.f, y_meas, tau, dopts)
                gm = gradient_mapping_norm(op, fi.f, y_meas, gamma, tau, lo, hi, inner, dopts)
                torch.cuda.synchronize()
                t_diag += time.perf_counter() - t0
                hist.append(dict(k=k, F=F, D=D, TV=tv, gmap=gm, D_at_s=rec["D"]))
        out[a] = dict(history=hist, step_seconds=t_step, diag_seconds=t_diag)
    return out


def main(argv=None):
    from synth import complex_normal
    from synth.workloads import WORKLOADS, make_phantom
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="strong_256")
    ap.add_argument("--K", type=int, default=100)
    ap.add_argument("--every", type=int, default=10)
    ap.add_argument("--alphas", default="0,0.5,0.9,0.96")
    args = ap.parse_args(argv)
    log = lambda m: print(m, file=sys.stderr, flush=True)
    torch.cuda.set_device(0)
    w = WORKLOADS[args.workload]
    op = Cisor(w.n, w.h, plane_wave_dirs(w.T), ring(w.M, w.rx_radius), eps_b=w.eps_b, precision=w.precision)
    op.autotune(reps=5)
    f_t = torch.tensor(make_phantom(w).ravel(), dtype=op.rdtype, device=op.device)
    _, y, _, _ = op.forward(f_t, SolveOpts(tol=w.ls_tol * 0.1, maxit=20000, start=1))
    y_np = y.cpu().numpy().astype(np.complex128)
    sigma = np.linalg.norm(y_np) / np.sqrt(y_np.size) * 10 ** (-w.snr_db / 20.0)
    y_meas = torch.tensor(y_np + sigma * complex_normal(y_np.shape, w.seed + 1), dtype=op.cdtype, device=op.device)
    gamma = 1.0 / op.born_lipschitz(50)
    alphas = [float(a) for a in args.alphas.split(",")]
    res = alpha_sweep(op, y_meas, gamma, w.tau, alphas, args.K, args.every, w.lo, w.hi, 100, w.ls_tol)
    for a, r in res.items():
        h = r["history"]
        log(f"[diag] alpha {a}: F {h[0]['F']:.4e} -> {h[-1]['F']:.4e}, ||G|| {h[0]['gmap']:.3e} -> "
            f"{h[-1]['gmap']:.3e}, min ||G|| {min(x['gmap'] for x in h):.3e}; steps {r['step_seconds']:.3f} s, "
            f"diagnostics {r['diag_seconds']:.3f} s")
    print(json.dumps(dict(workload=w.name, K=args.K, every=args.every, gamma=gamma, tau=w.tau,
                          sweep={str(a): r for a, r in res.items()})), flush=True)


if __name__ == "__main__":
    main()
