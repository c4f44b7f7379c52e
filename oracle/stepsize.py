"""Step-size helper: Lipschitz constant of the linear (first-Born) model.

The paper tunes the relaxed-FISTA step by hand and bounds it through the
Lipschitz constant of ``grad D`` (Prop. 2, Prop. 3).  For a reproducible
choice the tests use the Lipschitz constant of the gradient of the first-Born
misfit (``u = u_in``, the paper's "linear method"):

  ``L_B = lambda_max( v -> sum_t Re{ conj(u_in,t) H^H H (u_in,t v) } )``,

estimated by power iteration from a seeded start.  Pinned by: the dense
eigenvalue of the same (real symmetric) operator on a small grid.
"""

from __future__ import annotations

import numpy as np


def born_operator(prob, v):
    T = prob.T
    uin = prob.u_in.reshape(T, -1)
    y = (prob.H @ (uin * v.reshape(1, -1)).T)          # (M, T)
    back = (np.conj(prob.H).T @ y).T                   # (T, N)
    return np.sum(np.real(np.conj(uin) * back), axis=0).reshape(v.shape)


def born_lipschitz(prob, iters=50, seed=0):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((prob.n,) * prob.dim)
    v /= np.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        w = born_operator(prob, v)
        lam = float(np.sum(v * w))
        v = w / np.linalg.norm(w)
    return lam
