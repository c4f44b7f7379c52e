"""Learned warm start of the Lippmann-Schwinger solves.

``WarmStartNet`` wraps the library's BF16-MFMA encoder-decoder (``cisor_net_*``)
that predicts the total field u of ``A u = u_in`` from ``(f, u_in)``; besides f
and u_in it reads the first-Born scattered field u_B = u_in - A u_in, one
application of the library's operator.  The
module also holds the data generator (fields produced by the library's own
solver on seeded disk/ellipse phantoms), the training loop, and the
evaluation that compares LS iterations and wall time from the network start
(with a per-transmitter zero-start fallback) against the zero and first-Born
starts at the same true residual.

Command line (on a GPU):
    python -m paper_1708_01663_amd.warmstart train --out weights.npz
    python -m paper_1708_01663_amd.warmstart eval --weights weights.npz
"""

from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys
import time

import numpy as np
import torch

from . import _lib
from .cisor import Cisor, SolveOpts, plane_wave_dirs, ring

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "warmstart_128.npz")


def _p(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class WarmStartNet:
    """The encoder-decoder on an ``H x W`` grid (parameters live on the GPU)."""

    def __init__(self, H=128, W=128, base=32, max_batch=16, seed=0, device="cuda"):
        self.lib = _lib.load()
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.H, self.W, self.base, self.max_batch = H, W, base, max_batch
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(self.lib.cisor_net_create(H, W, base, max_batch, seed, self._stream(), C.byref(h)),
                       "cisor_net_create", allow_not_converged=False)
        self.handle = h
        n = C.c_longlong()
        _lib.check(self.lib.cisor_net_num_params(self.handle, C.byref(n)), "cisor_net_num_params")
        self.nparams = int(n.value)

    def _stream(self):
        return C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def _sync(self):
        _lib.check(self.lib.cisor_net_set_stream(self.handle, self._stream()), "cisor_net_set_stream")

    def params(self):
        out = torch.empty(self.nparams, dtype=torch.float32, device=self.device)
        self._sync()
        _lib.check(self.lib.cisor_net_get_params(self.handle, _p(out)), "cisor_net_get_params")
        return out

    def set_params(self, p):
        p = torch.as_tensor(p, dtype=torch.float32).to(self.device).contiguous()
        assert p.numel() == self.nparams
        self._sync()
        _lib.check(self.lib.cisor_net_set_params(self.handle, _p(p)), "cisor_net_set_params")
        torch.cuda.current_stream(self.device).synchronize()

    def predict(self, f, u_in, u_born=None):
        """f: float32 [B, H*W]; u_in, u_born: complex64 [B, H*W] -> u0 complex64 [B, H*W]."""
        f, u_in = f.contiguous(), u_in.contiguous()
        ub = u_born.contiguous() if u_born is not None else None
        u0 = torch.empty_like(u_in)
        self._sync()
        _lib.check(self.lib.cisor_net_forward(self.handle, _p(f), _p(u_in), _p(ub), _p(u0), f.shape[0]),
                   "cisor_net_forward")
        return u0

    def loss_grad(self, f, u_in, u, u_born=None):
        g = torch.empty(self.nparams, dtype=torch.float32, device=self.device)
        L = C.c_double()
        ub = u_born.contiguous() if u_born is not None else None
        self._sync()
        _lib.check(self.lib.cisor_net_loss_grad(self.handle, _p(f.contiguous()), _p(u_in.contiguous()), _p(ub),
                                                _p(u.contiguous()), f.shape[0], C.byref(L), _p(g)),
                   "cisor_net_loss_grad")
        return L.value, g

    def train_step(self, f, u_in, u, lr, u_born=None, clip=0.0):
        L = C.c_double()
        ub = u_born.contiguous() if u_born is not None else None
        self._sync()
        _lib.check(self.lib.cisor_net_train_step(self.handle, _p(f), _p(u_in), _p(ub), _p(u), f.shape[0], float(lr),
                                                 float(clip), C.byref(L)), "cisor_net_train_step")
        return L.value

    def save(self, path):
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        np.savez(path, params=self.params().cpu().numpy(), H=self.H, W=self.W, base=self.base)

    @classmethod
    def load(cls, path, max_batch=16, device="cuda"):
        z = np.load(path, allow_pickle=False)
        net = cls(int(z["H"]), int(z["W"]), int(z["base"]), max_batch=max_batch, device=device)
        net.set_params(z["params"])
        return net

    def close(self):
        if getattr(self, "handle", None):
            self.lib.cisor_net_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ data
def geometry(n=128, T=16):
    """Workload of the learned warm start: h = lambda/10, T plane waves, ring receivers."""
    h = 0.1
    return dict(n=n, h=h, T=T, M=4 * T, rx_radius=n * h)


def make_op(n=128, T=16, device="cuda"):
    g = geometry(n, T)
    return Cisor(g["n"], g["h"], plane_wave_dirs(g["T"]), ring(g["M"], g["rx_radius"]), device=device)


def born_field(op: Cisor, f, u_in=None):
    """First-Born scattered field u_B = G diag(f) u_in = u_in - A u_in for all
    transmitters (one library launch sequence, ``cisor_born_field``)."""
    return op.born_field(f)


def generate(op: Cisor, seeds, tol=1e-6, log=None):
    """Fields of the plain solver (first-Born start, true residual tol) for seeded
    disk/ellipse phantoms: returns f [S, N] float32, u [S, T, N] and the
    first-Born scattered fields u_B [S, T, N] (complex64) on the GPU."""
    from synth import mixed_2d
    fs, us, bs = [], [], []
    u_in = op.uin()
    for i, s in enumerate(seeds):
        f = torch.tensor(mixed_2d(op.n, int(s)).ravel(), dtype=torch.float32, device=op.device)
        u, _, its, code = op.forward(f, SolveOpts(tol=tol, maxit=20000, start=1), project=False)
        fs.append(f)
        us.append(u)
        bs.append(born_field(op, f, u_in))
        if log and i % 100 == 0:
            log(f"[data] {i}/{len(seeds)} mean iterations {its.mean():.0f}")
    return torch.stack(fs), torch.stack(us), torch.stack(bs)


def dihedral(x, n, g):
    """Apply the g-th symmetry of the square grid (g = 0..7: g % 4 quarter
    turns, then a transpose when g >= 4) to fields x [B, n*n]."""
    y = torch.rot90(x.view(-1, n, n), g % 4, dims=(1, 2))
    if g >= 4:
        y = y.transpose(1, 2)
    return y.contiguous().view(x.shape[0], n * n)


def train(net: WarmStartNet, f, u, u_in, u_b=None, epochs=10, batch=16, lr=5e-4, clip=1.0, warmup=500, seed=0,
          log=None, augment=False):
    """Adam on the relative-L2 loss over all (phantom, transmitter) pairs:
    linear warm-up over ``warmup`` steps, cosine decay, global-norm clipping.
    With ``augment`` each batch is mapped by a random symmetry of the square
    grid (rotations by quarter turns and reflections): the centred grid and the
    isotropic Green's function make the mapped contrast, incident and total
    fields an exact solution pair of the mapped problem."""
    S, T, N = u.shape
    n = int(round(N ** 0.5))
    rng = np.random.default_rng(seed)
    hist = []
    steps_per_epoch = (S * T) // batch
    total = epochs * steps_per_epoch
    step = 0
    for ep in range(epochs):
        perm = rng.permutation(S * T)
        losses = []
        for k in range(steps_per_epoch):
            idx = torch.as_tensor(perm[k * batch:(k + 1) * batch], device=u.device)
            s_i, t_i = idx // T, idx % T
            fb = f[s_i].contiguous()
            ub = u[s_i, t_i].contiguous()
            ib = u_in[t_i].contiguous()
            bb = u_b[s_i, t_i].contiguous() if u_b is not None else None
            if augment:
                g = int(rng.integers(8))
                fb, ub, ib = dihedral(fb, n, g), dihedral(ub, n, g), dihedral(ib, n, g)
                bb = dihedral(bb, n, g) if bb is not None else None
            cur = lr * min(1.0, (step + 1) / warmup) * 0.5 * (1 + np.cos(np.pi * step / total))
            losses.append(net.train_step(fb, ib, ub, cur, u_born=bb, clip=clip))
            step += 1
        hist.append(float(np.mean(losses)))
        if log:
            log(f"[train] epoch {ep}: mean relative-L2 loss {hist[-1]:.4f}")
    return hist


def forward_flops(H, W, base=32, batch=1):
    """Multiply-add FLOPs (2 per product) of the network's 15 3x3 convolutions
    on a batch: encoder levels at full, 1/2, 1/4 resolution, the bottleneck at
    1/8, the decoder back up (channel counts as the library builds them)."""
    c1, c2, c3, c4 = base, 2 * base, 4 * base, 8 * base
    layers = [(32, c1, 1), (c1, c1, 1), (c1, c2, 2), (c2, c2, 2), (c2, c3, 4), (c3, c3, 4), (c3, c4, 8),
              (c4, c4, 8), (c3 + c4, c3, 4), (c3, c3, 4), (c2 + c3, c2, 2), (c2, c2, 2), (c1 + c2, c1, 1),
              (c1, c1, 1), (c1, 32, 1)]
    return sum(2 * 9 * ci * co * (H // d) * (W // d) for ci, co, d in layers) * batch


def time_inference(op: Cisor, net: WarmStartNet, reps=20, seed=300000):
    """Average wall time of one network forward on a batch of op.T fields,
    timed with HIP events on the launch stream, and its rate against the
    dense BF16 matrix peak of the MI355X (2.5 PFLOP/s)."""
    from synth import mixed_2d
    u_in = op.uin()
    f = torch.tensor(mixed_2d(op.n, seed).ravel(), dtype=torch.float32, device=op.device)
    fb = f.expand(op.T, -1).contiguous()
    ub = born_field(op, f, u_in)
    for _ in range(3):
        net.predict(fb, u_in, ub)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        net.predict(fb, u_in, ub)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    flops = forward_flops(net.H, net.W, net.base, op.T)
    tflops = flops / (ms * 1e-3) / 1e12
    return dict(ms=round(ms, 4), batch=op.T, gflop=round(flops / 1e9, 3), TFLOPs=round(tflops, 1),
                frac_bf16_peak=round(tflops / 2500.0, 4))


def evaluate(op: Cisor, net: WarmStartNet, seeds, tol=1e-6):
    """LS iterations and wall time to the true residual tol from the zero, the
    first-Born and the network start, and the network field error against the
    converged solve.  The network leg's time covers the first-Born input field,
    the inference and the solve; its solve keeps the network's field per
    transmitter unless its starting residual is larger than the zero start's
    (start mode 5, a check that costs no operator application)."""
    from synth import mixed_2d
    u_in = op.uin()
    out = {"zero": [0, 0.0], "born": [0, 0.0], "net": [0, 0.0]}
    errs, fallbacks = [], 0
    for s in seeds:
        f = torch.tensor(mixed_2d(op.n, int(s)).ravel(), dtype=torch.float32, device=op.device)
        for label, start in (("zero", 0), ("born", 1)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            u, _, its, _ = op.forward(f, SolveOpts(tol=tol, maxit=20000, start=start), project=False)
            torch.cuda.synchronize()
            out[label][0] += int(its.sum())
            out[label][1] += time.perf_counter() - t0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u0 = net.predict(f.expand(op.T, -1).contiguous(), u_in, born_field(op, f, u_in))
        un, _, its, _ = op.forward(f, SolveOpts(tol=tol, maxit=20000, start=5), u0=u0, project=False)
        torch.cuda.synchronize()
        out["net"][0] += int(its.sum())
        out["net"][1] += time.perf_counter() - t0
        choice = (C.c_int * op.T)()
        _lib.check(op.lib.cisor_get_start_choice(op.handle, choice), "cisor_get_start_choice")
        fallbacks += int(sum(choice))
        sc = (u - u_in)
        errs.append(float(torch.linalg.vector_norm(u0 - u) / torch.linalg.vector_norm(sc)))
    nsolves = len(seeds) * op.T
    res = {k: dict(mean_iters=v[0] / nsolves, solves_per_s=nsolves / v[1], seconds=v[1]) for k, v in out.items()}
    res["net_rel_error_of_scattered_field"] = float(np.mean(errs))
    res["fallback_fraction"] = fallbacks / nsolves
    res["solves"] = nsolves
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["train", "eval", "infer"])
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--weights", default=DEFAULT_WEIGHTS)
    ap.add_argument("--phantoms", type=int, default=1250, help="training phantoms (x16 transmitters)")
    ap.add_argument("--epochs", type=int, default=10)
    ap.add_argument("--lr", type=float, default=5e-4)
    ap.add_argument("--clip", type=float, default=1.0)
    ap.add_argument("--eval-phantoms", type=int, default=64)
    ap.add_argument("--augment", action="store_true", help="random grid symmetries per batch")
    args = ap.parse_args(argv)
    log = lambda m: print(m, file=sys.stderr, flush=True)
    torch.cuda.set_device(0)
    op = make_op()
    if args.cmd == "infer":   # inference timing only (profiling entry point)
        net = WarmStartNet.load(args.weights)
        print(json.dumps(time_inference(op, net)), flush=True)
        return
    if args.cmd == "train":
        t0 = time.perf_counter()
        f, u, ub = generate(op, range(args.phantoms), log=log)
        log(f"[data] {f.shape[0]} phantoms x {op.T} transmitters in {time.perf_counter() - t0:.1f} s")
        net = WarmStartNet(op.n, op.n, 32, max_batch=16)
        t0 = time.perf_counter()
        hist = train(net, f, u, op.uin(), ub, epochs=args.epochs, lr=args.lr, clip=args.clip, log=log,
                     augment=args.augment)
        log(f"[train] {time.perf_counter() - t0:.1f} s")
        net.save(args.out)
        res = evaluate(op, net, range(100000, 100000 + args.eval_phantoms))
        print(json.dumps(dict(train_loss=hist, eval=res)), flush=True)
    else:
        net = WarmStartNet.load(args.weights)
        res = evaluate(op, net, range(100000, 100000 + args.eval_phantoms))
        print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
