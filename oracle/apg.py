"""Monotone accelerated proximal gradient (Li and Lin, NIPS 2015), FP64.

Test infrastructure only: the library never imports this package.

The comparison method of the paper's "Proposed Method" section: every
iteration forms an accelerated (FISTA-type) estimate ``z`` from an
extrapolated point ``y`` and a plain proximal-gradient (ISTA) estimate ``v``
from the current iterate ``x``, and keeps whichever has the lower objective
``F = D + R``.  So the gradient of ``D`` is needed at two points (``y`` and
``x``) and ``F`` at two more (``z`` and ``v``), each of which costs forward
solves in the inverse scattering problem; relaxed FISTA needs one gradient.

One iteration, with ``t_0 = 0``, ``t_1 = 1`` and ``x_0 = x_1 = z_1``:

    y_k     = x_k + (t_{k-1}/t_k)(z_k - x_k) + ((t_{k-1} - 1)/t_k)(x_k - x_{k-1})
    z_{k+1} = prox_{a_y R}(y_k - a_y grad D(y_k))
    v_{k+1} = prox_{a_x R}(x_k - a_x grad D(x_k))
    t_{k+1} = (sqrt(4 t_k^2 + 1) + 1) / 2
    x_{k+1} = z_{k+1} if F(z_{k+1}) <= F(v_{k+1}) else v_{k+1}

Pinned by (CPU tests): the convex O(1/k^2) bound
``F(x_{k+1}) - F* <= 2 ||x_0 - x*||^2 / (a_y (k+1)^2)`` on ill-conditioned
least squares (which plain proximal gradient breaks); equality with textbook
FISTA (Beck and Teboulle) when the accelerated estimate is always taken; the
estimate-sequence identity ``u_{k+1} = u_k - a_y t_k grad D(y_k)`` with
``u_k = x_{k-1} + t_{k-1}(z_k - x_{k-1})`` (identity prox), whichever estimate is
taken; monotonicity of ``F`` on a nonconvex problem with ``a_x < 1/L`` (which
the selection guarantees); convergence to ``lstsq``; the first iteration equal
to one ISTA step.
"""

from __future__ import annotations

import numpy as np

from . import cisor, tv


def monotone_apg(grad_fn, obj_fn, prox_fn, x0, gamma_y, gamma_x, K, callback=None):
    """Run K iterations.  ``grad_fn(x) -> (grad D(x), D(x))``;
    ``obj_fn(x) -> F(x)``; ``prox_fn(w, gamma) -> prox_{gamma R}(w)``.

    Returns ``(x_K, history)`` with per-iteration ``F(x_{k+1})``, ``F(z_{k+1})``,
    ``F(v_{k+1})``, ``D(y_k)``, ``D(x_k)``, whether ``z`` was taken, and the points
    ``x_{k+1}``, ``y_k``, ``z_{k+1}``, ``t_{k+1}`` and ``grad D(y_k)``."""
    x_prev = np.array(x0, dtype=np.float64)
    x = x_prev.copy()
    z = x_prev.copy()
    t_prev, t = 0.0, 1.0
    hist = dict(F=[], F_z=[], F_v=[], D_y=[], D_x=[], took_z=[], x=[], y=[], z=[], t=[], g_y=[])
    for k in range(1, K + 1):
        y = x + (t_prev / t) * (z - x) + ((t_prev - 1.0) / t) * (x - x_prev)
        g_y, D_y = grad_fn(y)
        z_new = prox_fn(y - gamma_y * g_y, gamma_y)
        g_x, D_x = grad_fn(x)
        v_new = prox_fn(x - gamma_x * g_x, gamma_x)
        t_prev, t = t, (np.sqrt(4.0 * t * t + 1.0) + 1.0) / 2.0
        F_z, F_v = obj_fn(z_new), obj_fn(v_new)
        took = bool(F_z <= F_v)
        x_prev, x = x, (z_new if took else v_new)
        z = z_new
        hist["F"].append(min(F_z, F_v))
        hist["F_z"].append(F_z)
        hist["F_v"].append(F_v)
        hist["D_y"].append(D_y)
        hist["D_x"].append(D_x)
        hist["took_z"].append(took)
        hist["x"].append(x.copy())
        hist["y"].append(y)
        hist["z"].append(z.copy())
        hist["t"].append(t)
        hist["g_y"].append(g_y)
        if callback is not None:
            callback(k, x, took)
    return x, hist


def cisor_apg(prob, y_meas, gamma_y, gamma_x, tau, K=20, lo=0.0, hi=2.0, inner=100, tol=1e-10, f0=None):
    """Monotone APG on the CISOR objective ``D + tau TV + box`` with the
    Prop. 1 gradient and forward solves for the objective values."""
    f0 = np.zeros((prob.n,) * prob.dim) if f0 is None else f0

    def grad_fn(x):
        return cisor.gradient(prob, x, y_meas, tol=tol)

    def obj_fn(x):
        return cisor.misfit(prob, x, y_meas, tol=tol) + tau * tv.tv_value(x)

    def prox_fn(w, gamma):
        return tv.prox_tv_box(w, gamma * tau, lo, hi, inner)

    return monotone_apg(grad_fn, obj_fn, prox_fn, f0, gamma_y, gamma_x, K)
