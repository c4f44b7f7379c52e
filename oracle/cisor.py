"""Forward model, misfit and the Prop. 1 gradient (FP64).

Notation follows "Problem Formulation" and Prop. 1:
  * ``u_t = A^{-1} u_in,t`` with ``A = I - G diag(f)``          (eqs. A_def, u_and_v)
  * ``Z_t(f) = H diag(u_t) f``, ``w_t = Z_t(f) - y_t``          (eqs. Z_def, Prop. 1)
  * ``D(f) = 1/2 sum_t ||y_t - Z_t(f)||^2``                      (eq. D_def)
  * ``v_t = A^{-H} diag(f) H^H w_t``                             (eq. u_and_v)
  * ``grad D = sum_t Re{ conj(u_t) (H^H w_t + G^H v_t) }``      (eq. gradient)

Reading: with several transmitters the paper writes ``D`` for one; the misfit
here is the plain sum over transmitters (and so is the gradient).

Pinned by: the dense Jacobian from the proof of Prop. 1 (``gradient_dense``),
central finite differences of ``misfit``, reciprocity, the first-Born limit and
the cylinder Bessel series (all in the CPU tests).
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import geometry, green, operators, krylov


@dataclass
class Problem:
    """A discretised scattering geometry (2D or 3D), all FP64."""
    n: int
    h: float
    dim: int
    u_in: np.ndarray           # (T, n, ..., n)
    H: np.ndarray              # (M, N)
    Ghat: np.ndarray           # (2n, ..., 2n)
    k: float
    eps_b: float = 1.0
    born: bool = False         # linear (first-Born) model: u = u_in, G = 0
    meta: dict = field(default_factory=dict)
    mask: np.ndarray | None = None   # (T, M) 0/1: receivers active for each transmitter

    @property
    def T(self):
        return self.u_in.shape[0]

    @property
    def M(self):
        return self.H.shape[0]

    @property
    def N(self):
        return self.n ** self.dim


def make_problem_2d(n, h, T, M, rx_radius, wavelength=1.0, eps_b=1.0, born=False, tx_pos=None, rx=None,
                    mask=None):
    """Plane waves at angles ``2 pi t/T`` and a ring of ``M`` receivers; or,
    when given, unit point sources at ``tx_pos`` (``(T, 2)``) and receivers at
    ``rx`` (``(M, 2)``), with ``mask`` (``(T, M)``) selecting the receivers
    each transmitter's data use (the paper's experiments switch off the
    receivers near the active transmitter)."""
    k = 2.0 * np.pi / wavelength
    kb = k * np.sqrt(eps_b)
    if tx_pos is not None:
        u_in = geometry.point_sources(n, h, kb, np.asarray(tx_pos, dtype=np.float64))
    else:
        u_in = geometry.plane_waves(n, h, kb, geometry.plane_wave_directions_2d(T))
    rx = geometry.ring_receivers(M, rx_radius) if rx is None else np.asarray(rx, dtype=np.float64)
    H = green.receiver_matrix(rx, n, h, k, eps_b)
    Ghat = green.kernel_spectrum(n, h, k, 2, eps_b)
    return Problem(n=n, h=h, dim=2, u_in=u_in, H=H, Ghat=Ghat, k=k, eps_b=eps_b,
                   born=born, meta=dict(rx=rx), mask=None if mask is None else np.asarray(mask, dtype=np.float64))


def make_problem_3d(n, h, dirs, rx, wavelength=1.0, eps_b=1.0):
    k = 2.0 * np.pi / wavelength
    kb = k * np.sqrt(eps_b)
    u_in = geometry.plane_waves(n, h, kb, dirs)
    H = green.receiver_matrix(rx, n, h, k, eps_b)
    Ghat = green.kernel_spectrum(n, h, k, 3, eps_b)
    return Problem(n=n, h=h, dim=3, u_in=u_in, H=H, Ghat=Ghat, k=k, eps_b=eps_b,
                   meta=dict(rx=rx))


def solve_fields(prob: Problem, f, rhs=None, tol=1e-10, adjoint=False, x0=None):
    """Solve ``A u_t = rhs_t`` (or ``A^H``) for every transmitter t."""
    rhs = prob.u_in if rhs is None else rhs
    if prob.born:
        return (rhs.copy() if not adjoint else rhs.copy()), np.zeros(rhs.shape[0], int)
    op = operators.apply_AH if adjoint else operators.apply_A
    out = np.empty_like(rhs, dtype=np.complex128)
    its = np.zeros(rhs.shape[0], dtype=int)
    for t in range(rhs.shape[0]):
        out[t], its[t], _ = krylov.bicgstab(
            lambda x: op(prob.Ghat, f, x), rhs[t],
            None if x0 is None else x0[t], tol=tol)
    return out, its


def project(prob: Problem, f, u):
    """``y_t = H diag(u_t) f`` for all t, shape ``(T, M)`` (eq. Z_def)."""
    T = u.shape[0]
    return (prob.H @ (f.reshape(-1) * u.reshape(T, -1)).T).T


def forward(prob: Problem, f, tol=1e-10):
    """Total fields and receiver data ``(u, y)``."""
    u, _ = solve_fields(prob, f, tol=tol)
    return u, project(prob, f, u)


def residual(prob: Problem, y, y_meas):
    """``w_t = Z_t(f) - y_t`` on the receivers each transmitter uses (zero on
    the others when the problem has a mask)."""
    w = y - y_meas
    return w if prob.mask is None else w * prob.mask


def misfit(prob: Problem, f, y_meas, tol=1e-10):
    """``D(f) = 1/2 sum_t ||Z_t(f) - y_t||^2`` (eq. D_def), over the active receivers."""
    _, y = forward(prob, f, tol)
    w = residual(prob, y, y_meas)
    return 0.5 * float(np.sum(np.abs(w) ** 2))


def gradient(prob: Problem, f, y_meas, tol=1e-10, return_parts=False):
    """Prop. 1: ``grad D`` by one forward and one adjoint solve per transmitter."""
    T = prob.T
    u, _ = solve_fields(prob, f, tol=tol)
    y = project(prob, f, u)
    w = residual(prob, y, y_meas)
    D = 0.5 * float(np.sum(np.abs(w) ** 2))
    shape = u.shape
    q = (np.conj(prob.H).T @ w.T).T.reshape(shape)           # H^H w_t
    b = f * q                                                # diag(f) H^H w_t
    if prob.born:
        p = np.zeros_like(q)
        v = np.zeros_like(q)
    else:
        v, _ = solve_fields(prob, f, rhs=b, tol=tol, adjoint=True)
        p = operators.apply_GH(prob.Ghat, v)                 # G^H v_t
    g = np.sum(np.real(np.conj(u) * (q + p)), axis=0)
    if return_parts:
        return g, D, dict(u=u, y=y, w=w, q=q, v=v, p=p)
    return g, D


def gradient_dense(prob: Problem, f, y_meas, Gdense):
    """Gradient from the explicit Jacobian in the proof of Prop. 1 (brute force).

    ``dZ_m/df_n = H[m,n] u_n + sum_i H[m,i] f_i du_i/df_n`` with
    ``du/df_n = A^{-1} G e_n u_n`` (from differentiating ``A u = u_in``), so
    ``J_t = H diag(u_t) + H diag(f) A^{-1} G diag(u_t)`` and
    ``grad D = sum_t Re(J_t^H w_t)``.  Dense linear algebra; small grids only.
    """
    N = prob.N
    fv = f.reshape(-1)
    Amat = np.eye(N) - Gdense * fv[None, :]
    Ainv = np.linalg.inv(Amat)
    g = np.zeros(N)
    D = 0.0
    for t in range(prob.T):
        u = Ainv @ prob.u_in[t].reshape(-1)
        y = prob.H @ (fv * u)
        J = prob.H * u[None, :] + (prob.H * fv[None, :]) @ Ainv @ (Gdense * u[None, :])
        m = np.ones(prob.M) if prob.mask is None else prob.mask[t]
        J = J * m[:, None]                       # a switched-off receiver has no data
        r = m * (y - y_meas[t])
        g += np.real(np.conj(J).T @ r)
        D += 0.5 * float(np.sum(np.abs(r) ** 2))
    return g.reshape(f.shape), D


def add_noise(y, snr_db, seed):
    """``y + e`` with complex Gaussian ``e`` scaled so ``20 log10(||y||/||e||) = snr``.

    The noise level is ``sigma = ||y||_F / sqrt(size) * 10^(-snr/20)`` applied to
    standard circular complex normal draws.
    """
    from synth import complex_normal
    e = complex_normal(y.shape, seed)
    sigma = np.linalg.norm(y) / np.sqrt(y.size) * 10 ** (-snr_db / 20.0)
    return y + sigma * e
