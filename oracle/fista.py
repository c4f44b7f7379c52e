"""Relaxed FISTA (eqs. algo1-algo3), FP64.

  ``f_k     = prox_{gamma R}(s_k - gamma grad D(s_k))``                 (algo1)
  ``t_{k+1} = (sqrt(4 t_k^2 + 1) + 1) / 2``                             (algo2)
  ``s_{k+1} = f_k + alpha ((t_k - 1)/t_{k+1}) (f_k - f_{k-1})``          (algo3)

Readings: the paper starts from "some initialisation" with ``s_1 = f_0`` and
writes ``t_0 = 1`` although the first update uses ``t_1``; here ``t_1 = 1`` (so
the first momentum weight is zero, as in Beck-Teboulle FISTA, which the paper
says alpha = 1 reproduces) and ``f_{-1} = f_0`` (as the convergence proof
assumes).  ``f_0 = 0`` unless given.  The step ``gamma`` is an input: the paper
tunes it by hand; Prop. 3 guarantees convergence for
``gamma <= (1 - alpha^2) / (2 L)``.

Pinned by: convergence to the least-squares solution of a linear model with
tau = 0 and an inactive box; the energy inequality from the proof of Prop. 3,
``F(f_{k+1}) + (1/(2 gamma) - L)||f_{k+1} - f_k||^2`` non-increasing on a
linear model with exact ``L``; alpha = 0 giving a momentum-free iteration.
"""

from __future__ import annotations

import numpy as np

from . import cisor, tv


def objective(D_value, x, tau):
    """``F(x) = D(x) + tau TV(x)`` (eq. objective_func; the box indicator is
    zero on iterates, which the prox keeps in the box)."""
    return float(D_value) + tau * tv.tv_value(x)


def gradient_mapping(grad_fn, x, gamma, tau, lo=0.0, hi=2.0, inner=100):
    """``G_gamma(x) = (x - prox_{gamma R}(x - gamma grad D(x))) / gamma``
    (eq. gradient_mapping_def); zero exactly at stationary points of F."""
    z = tv.prox_tv_box(x - gamma * grad_fn(x)[0], gamma * tau, lo, hi, inner)
    return (x - z) / gamma


def rate_bound(L, gamma, F0, Fstar, K):
    """Right-hand side of eq. convergence_rate: a bound on
    ``min_{k <= K} ||G_gamma(f_k)||^2`` for ``gamma <= (1 - alpha^2)/(2L)``."""
    return 2 * L * (3 + gamma * L) ** 2 * (F0 - Fstar) / (K * gamma * L * (1 - gamma * L))


def relaxed_fista(grad_fn, f0, gamma, tau, alpha, K, lo=0.0, hi=2.0, inner=100,
                  callback=None):
    """Run K iterations; ``grad_fn(s) -> (grad D(s), D(s))``.

    Returns ``(f_K, history)`` where history holds per-iteration ``D(s_k)``,
    ``f_k`` and ``t_k``.
    """
    f_prev = np.array(f0, dtype=np.float64)
    f = f_prev.copy()
    s = f.copy()
    t = 1.0
    hist = dict(D=[], f=[], t=[], s=[])
    for k in range(1, K + 1):
        g, D = grad_fn(s)
        hist["D"].append(D)
        hist["s"].append(s.copy())
        f_new = tv.prox_tv_box(s - gamma * g, gamma * tau, lo, hi, inner)
        t_new = (np.sqrt(4.0 * t * t + 1.0) + 1.0) / 2.0
        s = f_new + alpha * ((t - 1.0) / t_new) * (f_new - f)
        f_prev, f, t = f, f_new, t_new
        hist["f"].append(f.copy())
        hist["t"].append(t)
        if callback is not None:
            callback(k, f, s, D)
    return f, hist


def cisor_reconstruct(prob, y_meas, gamma, tau, alpha=0.96, K=20, lo=0.0, hi=2.0,
                      inner=100, tol=1e-10, f0=None):
    """CISOR: relaxed FISTA on ``D + R`` with the Prop. 1 gradient."""
    f0 = np.zeros((prob.n,) * prob.dim) if f0 is None else f0

    def grad_fn(s):
        return cisor.gradient(prob, s, y_meas, tol=tol)

    return relaxed_fista(grad_fn, f0, gamma, tau, alpha, K, lo, hi, inner)
