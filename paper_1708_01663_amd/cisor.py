"""Thin Python front end of the CISOR HIP library.

``Cisor`` owns one library context.  Arrays are torch tensors on the GPU; the
wrapper only checks shapes and dtypes and passes raw device pointers and the
current HIP stream to the C ABI.  PyTorch provides device memory and streams;
every step of the reconstruction runs in the library's kernels.
"""

from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib

COL_VARIANTS = 10  # compiled column-stage variants (see cisor_autotune)


@dataclass
class SolveOpts:
    tol: float = 1e-6
    maxit: int = 5000
    start: int = 0            # 0 zero, 1 first-Born (x0 = rhs), 2 caller x0, 3 better of 1 and 2,
                              # 4 (FISTA steps only) previous fields extrapolated along the path,
                              # 5 caller x0 with a zero-start fallback (no extra operator application)
    replace_every: int = 50
    check_every: int = 10

    def c(self):
        return _lib.LsOpts(self.tol, self.maxit, self.start, self.replace_every, self.check_every)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class Cisor:
    """One scattering geometry on the GPU: plane-wave transmitters (tx_dir) or
    unit point sources (tx_pos, with tx_dir None), point receivers."""

    def __init__(self, n, h, tx_dir, rx_pos, wavelength=1.0, eps_b=1.0, precision="c64",
                 device="cuda", tx_pos=None):
        self.lib = _lib.load()
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        tx_kind = 0 if tx_pos is None else 1
        tx_dir = np.asarray(tx_dir if tx_pos is None else tx_pos, dtype=np.float64)
        self.dim = int(tx_dir.shape[-1]) if tx_dir.ndim == 2 else 2
        tx = np.ascontiguousarray(tx_dir.reshape(-1, self.dim))
        rx = np.ascontiguousarray(np.asarray(rx_pos, dtype=np.float64).reshape(-1, self.dim))
        self.n, self.N, self.T, self.M = int(n), int(n) ** self.dim, tx.shape[0], rx.shape[0]
        self.precision = 0 if precision == "c64" else 1
        self.rdtype = torch.float32 if self.precision == 0 else torch.float64
        self.cdtype = torch.complex64 if self.precision == 0 else torch.complex128
        self._tx, self._rx = tx, rx
        txp = tx.ctypes.data_as(C.POINTER(C.c_double))
        g = _lib.Geometry(self.dim, self.n, float(h), float(wavelength), float(eps_b), self.T, self.M,
                          txp if tx_kind == 0 else None, rx.ctypes.data_as(C.POINTER(C.c_double)), self.precision,
                          tx_kind, txp if tx_kind == 1 else None)
        handle = C.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(self.lib.cisor_create(C.byref(g), self._stream(), C.byref(handle)), "cisor_create",
                       allow_not_converged=False)
        self.handle = handle
        self.h, self.wavelength, self.eps_b = h, wavelength, eps_b
        Pv = C.c_int()
        _lib.check(self.lib.cisor_get_sizes(self.handle, None, None, None, C.byref(Pv), None), "cisor_get_sizes")
        self.P = Pv.value

    # -- helpers -----------------------------------------------------------
    def _stream(self):
        return C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def _sync_stream(self):
        _lib.check(self.lib.cisor_set_stream(self.handle, self._stream()), "cisor_set_stream")

    def _field(self, x, name, rows=None):
        rows = self.T if rows is None else rows
        if x.dtype != self.cdtype or x.device != self.device or not x.is_contiguous() \
                or x.numel() != rows * self.N:
            raise ValueError(f"{name}: expected contiguous {self.cdtype} [{rows}, {self.N}] on {self.device}")
        return x

    def _real(self, x, name):
        if x.dtype != self.rdtype or x.device != self.device or not x.is_contiguous() or x.numel() != self.N:
            raise ValueError(f"{name}: expected contiguous {self.rdtype} [{self.N}] on {self.device}")
        return x

    def _data(self, y, name):
        if y.dtype != self.cdtype or y.device != self.device or not y.is_contiguous() \
                or y.numel() != self.T * self.M:
            raise ValueError(f"{name}: expected contiguous {self.cdtype} [{self.T}, {self.M}]")
        return y

    def empty_fields(self):
        return torch.empty((self.T, self.N), dtype=self.cdtype, device=self.device)

    def empty_data(self):
        return torch.empty((self.T, self.M), dtype=self.cdtype, device=self.device)

    # -- API ---------------------------------------------------------------
    def uin(self):
        out = self.empty_fields()
        self._sync_stream()
        _lib.check(self.lib.cisor_get_uin(self.handle, _ptr(out)), "cisor_get_uin")
        return out

    def H(self):
        out = torch.empty((self.M, self.N), dtype=self.cdtype, device=self.device)
        self._sync_stream()
        _lib.check(self.lib.cisor_get_H(self.handle, _ptr(out)), "cisor_get_H")
        return out

    def apply_A(self, f, x, adjoint=False):
        self._real(f, "f")
        self._field(x, "x")
        y = torch.empty_like(x)
        self._sync_stream()
        _lib.check(self.lib.cisor_apply_A(self.handle, _ptr(f), _ptr(x), _ptr(y), int(adjoint)), "cisor_apply_A")
        return y

    def born_field(self, f):
        """First-Born scattered fields G diag(f) u_in,t of every transmitter (``cisor_born_field``)."""
        self._real(f, "f")
        y = self.empty_fields()
        self._sync_stream()
        _lib.check(self.lib.cisor_born_field(self.handle, _ptr(f), _ptr(y)), "cisor_born_field")
        return y

    def apply_A_stage(self, f, x, y, stage, adjoint=False):
        """Launch one of the three stages of ``apply_A`` (timing / profiling hook)."""
        self._sync_stream()
        _lib.check(self.lib.cisor_apply_A_stage(self.handle, _ptr(f) if f is not None else None,
                                                _ptr(x) if x is not None else None,
                                                _ptr(y) if y is not None else None, int(adjoint), int(stage)),
                   "cisor_apply_A_stage")

    def solve(self, f, b, adjoint=False, opts=None, x0=None):
        opts = opts or SolveOpts()
        self._real(f, "f")
        self._field(b, "b")
        x = x0.clone() if x0 is not None else torch.empty_like(b)
        iters = (C.c_int * self.T)()
        o = opts.c()
        self._sync_stream()
        code = _lib.check(self.lib.cisor_solve(self.handle, _ptr(f), _ptr(b), _ptr(x), int(adjoint), C.byref(o),
                                               iters), "cisor_solve")
        return x, np.array(iters[:]), code

    def forward(self, f, opts=None, u0=None, project=True):
        opts = opts or SolveOpts()
        self._real(f, "f")
        u = u0.clone() if u0 is not None else self.empty_fields()
        y = self.empty_data() if project else None
        iters = (C.c_int * self.T)()
        o = opts.c()
        self._sync_stream()
        code = _lib.check(self.lib.cisor_forward(self.handle, _ptr(f), _ptr(u), _ptr(y) if project else None,
                                                 C.byref(o), iters), "cisor_forward")
        return u, y, np.array(iters[:]), code

    def project(self, f, u, y_meas=None):
        self._real(f, "f")
        self._field(u, "u")
        y = self.empty_data()
        D = C.c_double(0.0)
        self._sync_stream()
        _lib.check(self.lib.cisor_project(self.handle, _ptr(f), _ptr(u), _ptr(y_meas) if y_meas is not None else None,
                                          _ptr(y), C.byref(D) if y_meas is not None else None), "cisor_project")
        return (y, D.value) if y_meas is not None else y

    def backproject(self, w):
        self._data(w, "w")
        q = self.empty_fields()
        self._sync_stream()
        _lib.check(self.lib.cisor_backproject(self.handle, _ptr(w), _ptr(q)), "cisor_backproject")
        return q

    def grad(self, f, y_meas, opts=None, u_ws=None, v_ws=None):
        opts = opts or SolveOpts()
        self._real(f, "f")
        self._data(y_meas, "y_meas")
        u = u_ws if u_ws is not None else self.empty_fields()
        v = v_ws if v_ws is not None else self.empty_fields()
        g = torch.empty(self.N, dtype=self.rdtype, device=self.device)
        D = C.c_double(0.0)
        iters = (C.c_int * (2 * self.T))()
        o = opts.c()
        self._sync_stream()
        code = _lib.check(self.lib.cisor_grad(self.handle, _ptr(f), _ptr(y_meas), _ptr(g), C.byref(D), _ptr(u),
                                              _ptr(v), C.byref(o), iters), "cisor_grad")
        return g, D.value, u, v, np.array(iters[:]), code

    def vjp(self, f, u, w, opts=None, v_ws=None):
        """grad = Re{J^H w} for the data map f -> y at the fields u (see ``cisor_vjp``)."""
        opts = opts or SolveOpts()
        self._real(f, "f")
        self._field(u, "u")
        self._data(w, "w")
        v = v_ws if v_ws is not None else self.empty_fields()
        g = torch.empty(self.N, dtype=self.rdtype, device=self.device)
        iters = (C.c_int * self.T)()
        o = opts.c()
        self._sync_stream()
        code = _lib.check(self.lib.cisor_vjp(self.handle, _ptr(f), _ptr(u), _ptr(w), _ptr(g), _ptr(v), C.byref(o),
                                             iters), "cisor_vjp")
        return g, np.array(iters[:]), code

    def tv_prox(self, z, lam, lo=0.0, hi=2.0, inner=100):
        self._real(z, "z")
        x = torch.empty_like(z)
        self._sync_stream()
        _lib.check(self.lib.cisor_tv_prox(self.handle, _ptr(z), _ptr(x), float(lam), float(lo), float(hi),
                                          int(inner)), "cisor_tv_prox")
        return x

    def set_rx_mask(self, mask):
        """mask: [T, M] (nonzero = receiver active for the transmitter) or None."""
        if mask is None:
            _lib.check(self.lib.cisor_set_rx_mask(self.handle, None), "cisor_set_rx_mask")
            return
        m = np.ascontiguousarray(np.asarray(mask).reshape(self.T, self.M) != 0, dtype=np.uint8)
        self._sync_stream()
        _lib.check(self.lib.cisor_set_rx_mask(self.handle, m.ctypes.data_as(C.c_void_p)), "cisor_set_rx_mask")

    def tv_value(self, x):
        """Isotropic TV of x (FP64 sum), the regulariser of the objective."""
        self._real(x, "x")
        v = C.c_double(0.0)
        self._sync_stream()
        _lib.check(self.lib.cisor_tv_value(self.handle, _ptr(x), C.byref(v)), "cisor_tv_value")
        return v.value

    def autotune(self, reps=10):
        """Time the column-stage variants on this context and keep the fastest:
        returns (variant, mean ms per launch of each variant)."""
        v = C.c_int()
        times = (C.c_float * COL_VARIANTS)()
        self._sync_stream()
        _lib.check(self.lib.cisor_autotune(self.handle, int(reps), C.byref(v), times), "cisor_autotune")
        return v.value, list(times)

    def set_col_variant(self, v):
        _lib.check(self.lib.cisor_set_col_variant(self.handle, int(v)), "cisor_set_col_variant")

    def born_lipschitz(self, iters=50):
        L = C.c_double(0.0)
        self._sync_stream()
        _lib.check(self.lib.cisor_born_lipschitz(self.handle, int(iters), C.byref(L)), "cisor_born_lipschitz")
        return L.value

    def close(self):
        if getattr(self, "handle", None):
            self.lib.cisor_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Fista:
    """Relaxed-FISTA driver over ``cisor_fista_step`` (state lives on the GPU)."""

    def __init__(self, op: Cisor, y_meas, gamma, tau, alpha=0.96, lo=0.0, hi=2.0, inner=100,
                 opts=None, f0=None):
        self.op, self.y = op, op._data(y_meas, "y_meas")
        self.gamma, self.tau, self.alpha, self.lo, self.hi, self.inner = gamma, tau, alpha, lo, hi, inner
        self.opts = opts or SolveOpts(start=4)
        z = torch.zeros(op.N, dtype=op.rdtype, device=op.device) if f0 is None else f0.clone()
        self.f, self.f_prev, self.s = z.clone(), z.clone(), z.clone()
        self.state = _lib.FistaState(self.f.data_ptr(), self.f_prev.data_ptr(), self.s.data_ptr(), 1.0, 0)
        self.history = []

    def step(self):
        info = _lib.StepInfo()
        o = self.opts.c()
        self.op._sync_stream()
        code = _lib.check(self.op.lib.cisor_fista_step(
            self.op.handle, C.byref(self.state), _ptr(self.y), self.gamma, self.tau, self.alpha, self.lo, self.hi,
            self.inner, C.byref(o), C.byref(info)), "cisor_fista_step")
        rec = dict(k=self.state.k, D=info.D, fwd_max=info.fwd_iters_max, adj_max=info.adj_iters_max,
                   fwd_sum=info.fwd_iters_sum, adj_sum=info.adj_iters_sum, relres=info.max_true_relres,
                   status=info.status, code=code)
        self.history.append(rec)
        return rec


class Apg:
    """Monotone APG (Li and Lin) driver over ``cisor_apg_step``: the comparison
    method that keeps the better of an accelerated and a proximal-gradient
    estimate each iteration (state lives on the GPU)."""

    def __init__(self, op: Cisor, y_meas, gamma, tau, gamma_x=None, lo=0.0, hi=2.0, inner=100, opts=None,
                 f0=None):
        self.op, self.y = op, op._data(y_meas, "y_meas")
        self.gamma_y, self.gamma_x = gamma, gamma if gamma_x is None else gamma_x
        self.tau, self.lo, self.hi, self.inner = tau, lo, hi, inner
        self.opts = opts or SolveOpts(start=1)
        z = torch.zeros(op.N, dtype=op.rdtype, device=op.device) if f0 is None else f0.clone()
        self.x, self.x_prev, self.z = z.clone(), z.clone(), z.clone()
        self.state = _lib.ApgState(self.x.data_ptr(), self.x_prev.data_ptr(), self.z.data_ptr(), 1.0, 0.0, 0)
        self.history = []

    def step(self):
        info = _lib.ApgInfo()
        o = self.opts.c()
        self.op._sync_stream()
        code = _lib.check(self.op.lib.cisor_apg_step(
            self.op.handle, C.byref(self.state), _ptr(self.y), self.gamma_y, self.gamma_x, self.tau, self.lo,
            self.hi, self.inner, C.byref(o), C.byref(info)), "cisor_apg_step")
        rec = dict(k=self.state.k, F=info.F, F_z=info.F_z, F_v=info.F_v, D_y=info.D_y, D_x=info.D_x,
                   took_z=bool(info.took_z), fwd_solves=info.fwd_solves, adj_solves=info.adj_solves,
                   fwd_sum=info.fwd_iters_sum, adj_sum=info.adj_iters_sum, relres=info.max_true_relres,
                   status=info.status, code=code)
        self.history.append(rec)
        return rec


class Batch:
    """Many 2D problems with uneven grids and transmitter counts stepped
    together (``cisor_batch_*``).  ``problems``: sequence of dicts with keys
    n, h, tx_dir [T, 2] (or tx_pos [T, 2] for point sources), rx_pos [M, 2] and
    optionally wavelength, eps_b."""

    def __init__(self, problems, precision="c64", device="cuda", autotune=True, reps=5):
        self.lib = _lib.load()
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.precision = 0 if precision == "c64" else 1
        self.rdtype = torch.float32 if self.precision == 0 else torch.float64
        self.cdtype = torch.complex64 if self.precision == 0 else torch.complex128
        self._keep = []
        geoms = (_lib.Geometry * len(problems))()
        for i, pr in enumerate(problems):
            kind = 1 if pr.get("tx_pos") is not None else 0
            tx = np.ascontiguousarray(np.asarray(pr["tx_pos"] if kind else pr["tx_dir"], dtype=np.float64).reshape(-1, 2))
            rx = np.ascontiguousarray(np.asarray(pr["rx_pos"], dtype=np.float64).reshape(-1, 2))
            self._keep += [tx, rx]
            txp = tx.ctypes.data_as(C.POINTER(C.c_double))
            geoms[i] = _lib.Geometry(2, int(pr["n"]), float(pr["h"]), float(pr.get("wavelength", 1.0)),
                                     float(pr.get("eps_b", 1.0)), tx.shape[0], rx.shape[0],
                                     txp if kind == 0 else None, rx.ctypes.data_as(C.POINTER(C.c_double)),
                                     self.precision, kind, txp if kind == 1 else None)
        handle = C.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(self.lib.cisor_batch_create(geoms, len(problems), self._stream(), C.byref(handle)),
                       "cisor_batch_create", allow_not_converged=False)
        self.handle = handle
        self.count = len(problems)
        self.sizes = []
        for p in range(self.count):
            N, T, M, P, g = (C.c_int() for _ in range(5))
            _lib.check(self.lib.cisor_batch_get_sizes(self.handle, p, C.byref(N), C.byref(T), C.byref(M), C.byref(P),
                                                      C.byref(g)), "cisor_batch_get_sizes")
            self.sizes.append(dict(N=N.value, T=T.value, M=M.value, P=P.value, group=g.value))
        ng = C.c_int()
        _lib.check(self.lib.cisor_batch_num_groups(self.handle, C.byref(ng)), "cisor_batch_num_groups")
        self.groups = ng.value
        self.variants, self.tune_ms = None, None
        if autotune:
            self.autotune(reps)

    def _stream(self):
        return C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def _sync_stream(self):
        _lib.check(self.lib.cisor_batch_set_stream(self.handle, self._stream()), "cisor_batch_set_stream")

    def autotune(self, reps=5):
        v = (C.c_int * self.groups)()
        t = (C.c_float * (COL_VARIANTS * self.groups))()
        self._sync_stream()
        _lib.check(self.lib.cisor_batch_autotune(self.handle, int(reps), v, t), "cisor_batch_autotune")
        self.variants = list(v)
        self.tune_ms = np.array(t[:]).reshape(self.groups, COL_VARIANTS)
        return self.variants

    def born_lipschitz(self, p, iters=50):
        L = C.c_double(0.0)
        self._sync_stream()
        _lib.check(self.lib.cisor_batch_born_lipschitz(self.handle, int(p), int(iters), C.byref(L)),
                   "cisor_batch_born_lipschitz")
        return L.value

    def set_problem(self, p, y_meas, gamma, tau):
        s = self.sizes[p]
        if y_meas.dtype != self.cdtype or y_meas.device != self.device or not y_meas.is_contiguous() \
                or y_meas.numel() != s["T"] * s["M"]:
            raise ValueError(f"y_meas of problem {p}: expected contiguous {self.cdtype} [{s['T']}, {s['M']}]")
        self._sync_stream()
        _lib.check(self.lib.cisor_batch_set_problem(self.handle, int(p), _ptr(y_meas), float(gamma), float(tau)),
                   "cisor_batch_set_problem")

    def step(self, alpha=0.96, lo=0.0, hi=2.0, inner=100, opts=None):
        opts = opts or SolveOpts(start=2)
        info = (_lib.StepInfo * self.count)()
        o = opts.c()
        self._sync_stream()
        _lib.check(self.lib.cisor_batch_fista_step(self.handle, float(alpha), float(lo), float(hi), int(inner),
                                                   C.byref(o), info), "cisor_batch_fista_step")
        return [dict(D=i.D, fwd_max=i.fwd_iters_max, adj_max=i.adj_iters_max, fwd_sum=i.fwd_iters_sum,
                     adj_sum=i.adj_iters_sum, relres=i.max_true_relres, status=i.status) for i in info]

    def f(self, p):
        out = torch.empty(self.sizes[p]["N"], dtype=self.rdtype, device=self.device)
        self._sync_stream()
        _lib.check(self.lib.cisor_batch_get_f(self.handle, int(p), _ptr(out)), "cisor_batch_get_f")
        return out

    def forward(self, fs, opts=None, u0=None, project=True):
        """Forward solves of every problem: fs[p] real [N_p] -> (u list, y list, iters list, code)."""
        opts = opts or SolveOpts()
        fa = (C.c_void_p * self.count)()
        ua = (C.c_void_p * self.count)()
        ya = (C.c_void_p * self.count)()
        us, ys = [], []
        for p, s in enumerate(self.sizes):
            f = fs[p]
            if f.dtype != self.rdtype or f.device != self.device or not f.is_contiguous() or f.numel() != s["N"]:
                raise ValueError(f"f of problem {p}: expected contiguous {self.rdtype} [{s['N']}]")
            u = u0[p].clone() if u0 is not None else torch.empty((s["T"], s["N"]), dtype=self.cdtype,
                                                                  device=self.device)
            y = torch.empty((s["T"], s["M"]), dtype=self.cdtype, device=self.device) if project else None
            fa[p], ua[p] = f.data_ptr(), u.data_ptr()
            ya[p] = y.data_ptr() if project else None
            us.append(u)
            ys.append(y)
        total = sum(s["T"] for s in self.sizes)
        iters = (C.c_int * total)()
        o = opts.c()
        self._sync_stream()
        code = _lib.check(self.lib.cisor_batch_forward(self.handle, fa, ua, ya if project else None, C.byref(o),
                                                       iters), "cisor_batch_forward")
        its, off = [], 0
        for s in self.sizes:
            its.append(np.array(iters[off:off + s["T"]]))
            off += s["T"]
        return us, ys, its, code

    def close(self):
        if getattr(self, "handle", None):
            self.lib.cisor_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cone_dirs(T, half_angle_deg=45.0):
    """3D plane-wave directions on a downward cone of the given half-angle."""
    a = np.deg2rad(half_angle_deg)
    ph = 2 * np.pi * np.arange(T) / T
    return np.stack([np.sin(a) * np.cos(ph), np.sin(a) * np.sin(ph), -np.cos(a) * np.ones(T)], axis=1)


def plane_rx(side, extent, z):
    """side x side receivers on the plane z spanning [-extent, extent]^2."""
    c = np.linspace(-extent, extent, side)
    X, Y = np.meshgrid(c, c, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), np.full(side * side, z)], axis=1)


def plane_wave_dirs(T):
    th = 2 * np.pi * np.arange(T) / T
    return np.stack([np.cos(th), np.sin(th)], axis=1)


def ring(M, radius):
    ph = 2 * np.pi * np.arange(M) / M
    return radius * np.stack([np.cos(ph), np.sin(ph)], axis=1)
