"""Isotropic total variation and its proximal map with a box constraint (FP64).

Regulariser (eq. R_def): ``R(f) = tau sum_n sqrt(sum_d |[D_d f]_n|^2) + chi_C(f)``.
Readings: ``D_d`` is the forward difference along axis d, zero at the last
index (Neumann boundary); ``C`` is the box ``[lo, hi]`` (the paper only says a
bounded closed convex set).

The proximal map in eq. algo1, ``prox_{gamma R}(z) = argmin_{x in C}
1/2 ||x - z||^2 + lam TV(x)`` with ``lam = gamma tau``, is computed by the fast
gradient projection (FGP) method of Beck and Teboulle (2009, "Fast
gradient-based algorithms for constrained total variation image denoising"),
which the paper cites for this step.  Derivation used here:

  ``TV(x) = max_{|p_n| <= 1} <p, grad x>``.  For fixed dual ``p`` the primal
  minimiser over the box is ``x(p) = P_C(z + lam div p)`` with
  ``div = -grad^T``; the dual objective is concave with a gradient
  ``lam grad x(p)`` whose Lipschitz constant is ``lam^2 ||grad||^2 <=
  lam^2 4d``.  FGP runs projected gradient ascent on the dual with step
  ``1/(4 d lam^2)`` -- i.e. ``p <- P_disk(r + grad x(r) / (4 d lam))`` --
  plus Nesterov momentum on the dual iterates (``t_1 = 1``), starting from
  ``p = 0``, and returns ``P_C(z + lam div p)``.

Pinned by: closed-form special cases (lam = 0, constant images, very large
lam), the exact 1-D TV prox of images that vary along one axis (its dual is a
bound-constrained least-squares problem, solved with ``scipy``), and the
primal-dual gap.
"""

from __future__ import annotations

import numpy as np


def grad(x):
    """Forward differences along every axis, zero at the last index."""
    g = np.zeros((x.ndim,) + x.shape)
    for d in range(x.ndim):
        sl_hi = [slice(None)] * x.ndim
        sl_lo = [slice(None)] * x.ndim
        sl_hi[d] = slice(1, None)
        sl_lo[d] = slice(0, -1)
        g[d][tuple(sl_lo)] = x[tuple(sl_hi)] - x[tuple(sl_lo)]
    return g


def div(p):
    """Negative adjoint of ``grad``: ``<grad x, p> = -<x, div p>``."""
    nd = p.shape[0]
    out = np.zeros(p.shape[1:])
    for d in range(nd):
        pd = p[d].copy()
        sl_last = [slice(None)] * nd
        sl_last[d] = -1
        pd[tuple(sl_last)] = 0.0          # the last-index component never couples
        out += pd
        sl_hi = [slice(None)] * nd
        sl_lo = [slice(None)] * nd
        sl_hi[d] = slice(1, None)
        sl_lo[d] = slice(0, -1)
        out[tuple(sl_hi)] -= pd[tuple(sl_lo)]
    return out


def tv_value(x):
    """Isotropic TV ``sum_n ||(grad x)_n||_2``."""
    return float(np.sum(np.sqrt(np.sum(grad(x) ** 2, axis=0))))


def _project_disk(p):
    nrm = np.sqrt(np.sum(p * p, axis=0))
    return p / np.maximum(1.0, nrm)


def prox_tv_box(z, lam, lo=-np.inf, hi=np.inf, iters=100, return_dual=False):
    """FGP for ``argmin_{lo <= x <= hi} 1/2||x - z||^2 + lam TV(x)``."""
    z = np.asarray(z, dtype=np.float64)
    if lam <= 0:
        x = np.clip(z, lo, hi)
        return (x, np.zeros((z.ndim,) + z.shape)) if return_dual else x
    L = 4.0 * z.ndim
    p = np.zeros((z.ndim,) + z.shape)
    r = p.copy()
    t = 1.0
    for _ in range(iters):
        x = np.clip(z + lam * div(r), lo, hi)
        p_new = _project_disk(r + grad(x) / (L * lam))
        t_new = (1.0 + np.sqrt(1.0 + 4.0 * t * t)) / 2.0
        r = p_new + ((t - 1.0) / t_new) * (p_new - p)
        p, t = p_new, t_new
    x = np.clip(z + lam * div(p), lo, hi)
    return (x, p) if return_dual else x


def primal_value(x, z, lam):
    return 0.5 * float(np.sum((x - z) ** 2)) + lam * tv_value(x)


def dual_value(p, z, lam, lo=-np.inf, hi=np.inf):
    """Dual objective ``min_{x in C} 1/2||x-z||^2 - lam <div p, x>`` (a lower bound)."""
    x = np.clip(z + lam * div(p), lo, hi)
    return 0.5 * float(np.sum((x - z) ** 2)) - lam * float(np.sum(div(p) * x))
