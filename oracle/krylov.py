"""Linear solvers for ``A u = u_in`` and ``A^H v = b`` (eq. u_and_v), FP64.

The paper solves these systems iteratively with ``A`` as an operator ("Proposed
Method", after Prop. 1).  It names conjugate gradients, which presumes a
Hermitian positive definite matrix; ``A = I - G diag(f)`` is complex and
non-Hermitian, so the reading taken here is BiCGSTAB (van der Vorst, 1992),
a short-recurrence Krylov method for general non-Hermitian systems.  The
answer it reaches is the unique solution of the linear system, so the choice
of Krylov method does not change what is computed, only how fast.

Stop test: the *true* relative residual ``||b - A x|| / ||b||`` in FP64.  When
the recurrence residual says converged, the true residual is evaluated; if it
is not yet below ``tol`` the recurrence residual is replaced by the true one
and the iteration restarts from the current ``x``.

Pinned by: ``numpy.linalg.solve`` on the dense matrix (small grids) and the
true-residual check in the tests.
"""

from __future__ import annotations

import numpy as np


def _dot(a, b):
    """Conjugated inner product ``a^H b``."""
    return np.vdot(a.ravel(), b.ravel())


def bicgstab(matvec, b, x0=None, tol=1e-10, maxit=20000):
    """Solve ``matvec(x) = b``.  Returns ``(x, iterations, true_relres)``."""
    b = np.asarray(b, dtype=np.complex128)
    nb = np.linalg.norm(b.ravel())
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    if nb == 0.0:
        return np.zeros_like(b), 0, 0.0
    r = b - matvec(x)
    relres = np.linalg.norm(r.ravel()) / nb
    if relres <= tol:
        return x, 0, relres
    it = 0
    while it < maxit:
        rhat = r.copy()
        rho_old = alpha = omega = 1.0 + 0j
        v = np.zeros_like(b)
        p = np.zeros_like(b)
        while it < maxit:
            it += 1
            rho = _dot(rhat, r)
            if rho == 0:
                break
            beta = (rho / rho_old) * (alpha / omega)
            p = r + beta * (p - omega * v)
            v = matvec(p)
            alpha = rho / _dot(rhat, v)
            s = r - alpha * v
            if np.linalg.norm(s.ravel()) / nb <= tol * 0.5:
                x = x + alpha * p
                r = s
                break
            t = matvec(s)
            tt = _dot(t, t).real
            if tt == 0:
                x = x + alpha * p
                r = s
                break
            omega = _dot(t, s) / tt
            x = x + alpha * p + omega * s
            r = s - omega * t
            rho_old = rho
            if np.linalg.norm(r.ravel()) / nb <= tol * 0.5 or omega == 0:
                break
        # verify against the true residual; restart from x if it is not met
        r = b - matvec(x)
        relres = np.linalg.norm(r.ravel()) / nb
        if relres <= tol:
            return x, it, relres
    return x, it, relres


def dense_solve(Amat, b):
    """Direct solve with the dense matrix (brute force, small systems)."""
    return np.linalg.solve(Amat, b)
