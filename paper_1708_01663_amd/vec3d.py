"""Python front end of the library's 3D vectorial (electromagnetic) model.

``VecCisor`` owns one ``cisor_vec_ctx``: three-component fields
``E = (E_x, E_y, E_z)`` on an ``n^3`` grid (the appendix on 3D imaging),
complex128 tensors of shape ``[T, 3, N]`` on the GPU.  Argument marshalling
only: the solves, the grad-div stencil, the dyadic projection and the
gradient run in the library's kernels.
"""

from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from .cisor import SolveOpts, _ptr


class VecCisor:
    """Plane-wave transmitters along ``tx_dir``, or electric dipoles at
    ``tx_pos`` (with ``tx_dir`` None), polarised along z projected transverse to
    the direction of travel; receivers polarised along z at ``rx_pos`` (outside
    the grid's cube); background permittivity 1."""

    def __init__(self, n, h, tx_dir, rx_pos, wavelength=1.0, device="cuda", tx_pos=None):
        self.lib = _lib.load()
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        kind = 0 if tx_pos is None else 1
        tx = np.ascontiguousarray(np.asarray(tx_dir if tx_pos is None else tx_pos, dtype=np.float64).reshape(-1, 3))
        rx = np.ascontiguousarray(np.asarray(rx_pos, dtype=np.float64).reshape(-1, 3))
        self.n, self.N, self.T, self.M = int(n), int(n) ** 3, tx.shape[0], rx.shape[0]
        self._tx, self._rx = tx, rx
        txp = tx.ctypes.data_as(C.POINTER(C.c_double))
        g = _lib.Geometry(3, self.n, float(h), float(wavelength), 1.0, self.T, self.M,
                          txp if kind == 0 else None, rx.ctypes.data_as(C.POINTER(C.c_double)), 1,
                          kind, txp if kind == 1 else None)
        handle = C.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(self.lib.cisor_vec_create(C.byref(g), self._stream(), C.byref(handle)), "cisor_vec_create",
                       allow_not_converged=False)
        self.handle = handle
        self.h, self.wavelength = h, wavelength

    def _stream(self):
        return C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def _sync_stream(self):
        _lib.check(self.lib.cisor_vec_set_stream(self.handle, self._stream()), "cisor_vec_set_stream")

    def _fields(self, x, name):
        if x.dtype != torch.complex128 or x.device != self.device or not x.is_contiguous() \
                or x.numel() != self.T * 3 * self.N:
            raise ValueError(f"{name}: expected contiguous complex128 [{self.T}, 3, {self.N}] on {self.device}")
        return x

    def _real(self, f, name):
        if f.dtype != torch.float64 or f.device != self.device or not f.is_contiguous() or f.numel() != self.N:
            raise ValueError(f"{name}: expected contiguous float64 [{self.N}] on {self.device}")
        return f

    def _data(self, y, name):
        if y.dtype != torch.complex128 or y.device != self.device or not y.is_contiguous() \
                or y.numel() != self.T * self.M:
            raise ValueError(f"{name}: expected contiguous complex128 [{self.T}, {self.M}]")
        return y

    def empty_fields(self):
        return torch.empty((self.T, 3, self.N), dtype=torch.complex128, device=self.device)

    def empty_data(self):
        return torch.empty((self.T, self.M), dtype=torch.complex128, device=self.device)

    def uin(self):
        out = self.empty_fields()
        self._sync_stream()
        _lib.check(self.lib.cisor_vec_get_uin(self.handle, _ptr(out)), "cisor_vec_get_uin")
        return out

    def H(self):
        out = torch.empty((self.M, 3 * self.N), dtype=torch.complex128, device=self.device)
        self._sync_stream()
        _lib.check(self.lib.cisor_vec_get_H(self.handle, _ptr(out)), "cisor_vec_get_H")
        return out

    def set_rx_mask(self, mask):
        """Receivers active per transmitter (host ``[T, M]`` 0/1, or None for all)."""
        if mask is None:
            _lib.check(self.lib.cisor_vec_set_rx_mask(self.handle, None), "cisor_vec_set_rx_mask")
            return
        m = np.ascontiguousarray(np.asarray(mask).reshape(self.T, self.M) != 0, dtype=np.uint8)
        self._sync_stream()
        _lib.check(self.lib.cisor_vec_set_rx_mask(self.handle, m.ctypes.data_as(C.c_void_p)), "cisor_vec_set_rx_mask")

    def apply_A(self, f, x, adjoint=False):
        self._real(f, "f")
        self._fields(x, "x")
        y = torch.empty_like(x)
        self._sync_stream()
        _lib.check(self.lib.cisor_vec_apply_A(self.handle, _ptr(f), _ptr(x), _ptr(y), int(adjoint)),
                   "cisor_vec_apply_A")
        return y

    def forward(self, f, opts=None, E0=None, project=True):
        """Returns ``(E, y, iters, code, max_rel)``; ``E0`` is the start when
        ``opts.start == 3``."""
        opts = opts or SolveOpts(tol=1e-10, start=0)
        self._real(f, "f")
        if opts.start == 3 and E0 is None:
            raise ValueError("start 3 needs a starting guess E0")
        E = self._fields(E0, "E0").clone() if E0 is not None else self.empty_fields()
        y = self.empty_data() if project else None
        iters = (C.c_int * self.T)()
        mr = C.c_double(0.0)
        o = opts.c()
        self._sync_stream()
        code = _lib.check(self.lib.cisor_vec_forward(self.handle, _ptr(f), C.byref(o), _ptr(E),
                                                     _ptr(y) if project else None, iters, C.byref(mr)),
                          "cisor_vec_forward")
        return E, y, np.array(iters[:]), code, mr.value

    def project(self, f, E):
        self._real(f, "f")
        self._fields(E, "E")
        y = self.empty_data()
        self._sync_stream()
        _lib.check(self.lib.cisor_vec_project(self.handle, _ptr(f), _ptr(E), _ptr(y)), "cisor_vec_project")
        return y

    def grad(self, f, y_meas, opts=None):
        """Returns ``(grad, D, iters[2T], code, max_rel)``."""
        opts = opts or SolveOpts(tol=1e-10, start=1)
        self._real(f, "f")
        self._data(y_meas, "y_meas")
        g = torch.empty(self.N, dtype=torch.float64, device=self.device)
        D = C.c_double(0.0)
        iters = (C.c_int * (2 * self.T))()
        mr = C.c_double(0.0)
        o = opts.c()
        self._sync_stream()
        code = _lib.check(self.lib.cisor_vec_grad(self.handle, _ptr(f), _ptr(y_meas), _ptr(g), C.byref(D),
                                                  C.byref(o), iters, C.byref(mr)), "cisor_vec_grad")
        return g, D.value, np.array(iters[:]), code, mr.value

    def close(self):
        if getattr(self, "handle", None):
            self.lib.cisor_vec_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class VecFista:
    """Relaxed-FISTA driver of the vectorial model over ``cisor_vec_fista_step``
    (3D TV/box prox; the state lives on the GPU)."""

    def __init__(self, op: VecCisor, y_meas, gamma, tau, alpha=0.96, lo=0.0, hi=2.0, inner=100, opts=None,
                 f0=None):
        self.op, self.y = op, op._data(y_meas, "y_meas")
        self.gamma, self.tau, self.alpha, self.lo, self.hi, self.inner = gamma, tau, alpha, lo, hi, inner
        self.opts = opts or SolveOpts(tol=1e-6, start=2)
        z = torch.zeros(op.N, dtype=torch.float64, device=op.device) if f0 is None else f0.clone()
        self.f, self.f_prev, self.s = z.clone(), z.clone(), z.clone()
        self.state = _lib.FistaState(self.f.data_ptr(), self.f_prev.data_ptr(), self.s.data_ptr(), 1.0, 0)
        self.history = []

    def step(self):
        info = _lib.StepInfo()
        o = self.opts.c()
        self.op._sync_stream()
        code = _lib.check(self.op.lib.cisor_vec_fista_step(
            self.op.handle, C.byref(self.state), _ptr(self.y), self.gamma, self.tau, self.alpha, self.lo, self.hi,
            self.inner, C.byref(o), C.byref(info)), "cisor_vec_fista_step")
        rec = dict(k=self.state.k, D=info.D, fwd_max=info.fwd_iters_max, adj_max=info.adj_iters_max,
                   fwd_sum=info.fwd_iters_sum, adj_sum=info.adj_iters_sum, relres=info.max_true_relres,
                   status=info.status, code=code)
        self.history.append(rec)
        return rec
