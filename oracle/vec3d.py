"""3D vectorial (electromagnetic) model of the paper's appendix on 3D imaging, FP64.

Test infrastructure only: the library never imports this package.

Fields are ``E = (E1, E2, E3)`` on the ``n^3`` grid, shape ``(3, n, n, n)`` per
transmitter (the stacking ``[E^(1); E^(2); E^(3)]`` of eq. u_def).

  * ``B = G0 (f E)`` componentwise: ``G0`` is the scalar Green's convolution
    with the cell integral of ``g`` (``G0 = green`` kernel ``/ k^2``).
  * ``E = E_in + k^2 B + D B`` (eq. discrete0_constrain), so
    ``A E = E - (k^2 I + D)(I_3 x G0 diag f) E`` (eq. 3DA_def).
  * ``D`` is the finite-difference grad-div operator with the printed stencils:
    ``d^2/dx_i^2`` the three-point second difference, ``d^2/dx_i dx_j`` the
    four-corner difference over ``4 delta^2``.
  * ``y_m = delta^3 sum_n sum_j Gd_3j(r_m - r_n) f_n E^(j)_n``
    (eq. discrete0_measurement).  The receivers are polarised along z, so only
    the third row of the dyadic Green's function (eq. dyadicGreen) enters.
  * ``w = mask (y - y_meas)``: a receiver switched off for a transmitter
    (the paper's 3D experiment uses only receivers more than 50 degrees away
    from the transmitter) carries no data.  The adjoint solve is
    ``A^H v = (I_3 x diag f) Ht^H w`` (eq. 3Du_and_v).  Then
    ``g = diag(u)^H (Ht^H w + (I_3 x G0^H)(k^2 I + D^H) v)`` (eq. 3Dg_def) and
    ``grad D = Re sum_i g^(i)`` (eq. 3Dgradient).

Readings where the appendix is silent:
  * the cell quadrature for ``B`` is the equal-volume ball of the scalar model;
    the printed ``delta^3 g`` point quadrature is singular on the diagonal;
  * ``B`` is zero outside the grid in the stencil;
  * the incident fields are plane waves polarised along z projected transverse
    to the propagation direction (x for propagation along z), or unit electric
    dipoles ``Gd(r - s) p / k^2`` with that polarisation for the direction from
    the source to the grid's centre;
  * ``eps_b = 1`` (vacuum background, ``f = eps - 1``).

Pinned by: a dense operator built from Kronecker products of 1D difference
matrices, the dyadic formula against finite differences of ``g``, the scalar
limit without the grad-div term, the first-Born limit, the gradient against
central differences of the misfit (with and without receiver masks), and the
first reconstruction step from ``f = 0`` in closed form (CPU tests).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import geometry, green, krylov


@dataclass
class Problem3V:
    n: int
    h: float
    k: float
    G0hat: np.ndarray          # (2n, 2n, 2n): spectrum of the cell-integrated g
    E_in: np.ndarray           # (T, 3, n, n, n)
    Ht: np.ndarray             # (M, 3N): third dyadic row times delta^3
    rx: np.ndarray             # (M, 3)
    mask: np.ndarray | None = None   # (T, M) 0/1: receivers active for each transmitter

    @property
    def T(self):
        return self.E_in.shape[0]

    @property
    def N(self):
        return self.n ** 3


def polarisations(dirs: np.ndarray) -> np.ndarray:
    """Unit z projected transverse to each direction (x if the direction is z)."""
    out = []
    for d in dirs:
        d = d / np.linalg.norm(d)
        ref = np.array([0.0, 0.0, 1.0]) if abs(d[2]) < 1 - 1e-9 else np.array([1.0, 0.0, 0.0])
        p = ref - np.dot(ref, d) * d
        out.append(p / np.linalg.norm(p))
    return np.array(out)


def dyadic_row3(R: np.ndarray, k: float) -> np.ndarray:
    """Third row ``Gd_3j(R)``, j = 1..3, of eq. dyadicGreen for offsets R (..., 3)."""
    d = np.linalg.norm(R, axis=-1)
    Rh = R / d[..., None]
    g = np.exp(1j * k * d) / (4 * np.pi * d)
    kd = k * d
    a = 3.0 / kd ** 2 - 3j / kd - 1.0
    b = 1.0 + 1j / kd - 1.0 / kd ** 2
    row = a[..., None] * Rh[..., 2:3] * Rh
    row[..., 2] += b
    return k ** 2 * row * g[..., None]


def dyadic(R: np.ndarray, k: float) -> np.ndarray:
    """The dyadic Green's function of eq. dyadicGreen, ``(k^2 I + grad grad) g``,
    at offsets R (..., 3): shape (..., 3, 3)."""
    d = np.linalg.norm(R, axis=-1)
    Rh = R / d[..., None]
    g = np.exp(1j * k * d) / (4 * np.pi * d)
    kd = k * d
    a = 3.0 / kd ** 2 - 3j / kd - 1.0
    b = 1.0 + 1j / kd - 1.0 / kd ** 2
    out = a[..., None, None] * Rh[..., :, None] * Rh[..., None, :] + b[..., None, None] * np.eye(3)
    return k ** 2 * out * g[..., None, None]


def dipole_fields(n, h, k, src, pol):
    """Incident fields of unit electric dipoles at ``src`` (T, 3) with unit
    polarisations ``pol`` (T, 3): ``E_in = Gd(r - s) p / k^2``, shape (T, 3, n, n, n)."""
    pos = geometry.pixel_positions_3d(n, h)
    out = np.empty((src.shape[0], 3, n ** 3), dtype=np.complex128)
    for t in range(src.shape[0]):
        out[t] = (dyadic(pos - src[t], k) @ pol[t]).T / k ** 2
    return out.reshape(src.shape[0], 3, n, n, n)


def make_problem(n, h, dirs, rx, wavelength=1.0, mask=None, src=None):
    """Plane waves travelling along ``dirs`` or, with ``src`` (T, 3), dipoles at
    those positions; either way polarised along z projected transverse to the
    direction towards the grid's centre (eq. dyadicGreen for the dipoles)."""
    k = 2.0 * np.pi / wavelength
    if src is not None:
        src = np.asarray(src, dtype=np.float64)
        dirs = -src
    dirs = np.asarray(dirs, dtype=np.float64)
    dirs = dirs / np.linalg.norm(dirs, axis=1, keepdims=True)
    pol = polarisations(dirs)                                 # (T, 3)
    if src is None:
        pw = geometry.plane_waves(n, h, k, dirs)              # (T, n, n, n)
        E_in = pol[:, :, None, None, None] * pw[:, None]
    else:
        E_in = dipole_fields(n, h, k, src, pol)
    G0hat = green.kernel_spectrum(n, h, k, 3) / k ** 2
    pos = geometry.pixel_positions_3d(n, h)                   # (N, 3)
    rx = np.asarray(rx, dtype=np.float64)
    row = dyadic_row3(rx[:, None, :] - pos[None, :, :], k)    # (M, N, 3)
    Ht = h ** 3 * np.concatenate([row[..., 0], row[..., 1], row[..., 2]], axis=1)
    return Problem3V(n=n, h=h, k=k, G0hat=G0hat, E_in=E_in, Ht=Ht, rx=rx,
                     mask=None if mask is None else np.asarray(mask, dtype=np.float64))


def _conv(Ghat, x, conj=False):
    n = Ghat.shape[0] // 2
    pad = np.zeros(x.shape[:-3] + Ghat.shape, dtype=np.complex128)
    pad[..., :n, :n, :n] = x
    spec = np.fft.fftn(pad, axes=(-3, -2, -1)) * (np.conj(Ghat) if conj else Ghat)
    return np.fft.ifftn(spec, axes=(-3, -2, -1))[..., :n, :n, :n]


def grad_div(B, h):
    """``(D B)^(i) = sum_j d_i d_j B^(j)`` with the printed stencils, B = 0 outside."""
    n = B.shape[-1]
    P = np.zeros((3, n + 2, n + 2, n + 2), dtype=np.complex128)
    P[:, 1:-1, 1:-1, 1:-1] = B
    c = slice(1, n + 1)
    lo, hi = slice(0, n), slice(2, n + 2)

    def at(comp, sx, sy, sz):
        return P[comp][sx, sy, sz]

    def sl(axis, s):
        out = [c, c, c]
        out[axis] = s
        return out

    out = np.zeros_like(B)
    for i in range(3):
        acc = (at(i, *sl(i, hi)) - 2 * at(i, c, c, c) + at(i, *sl(i, lo)))
        for j in range(3):
            if j == i:
                continue
            def corner(si, sj):
                idx = [c, c, c]
                idx[i] = si
                idx[j] = sj
                return at(j, *idx)
            acc = acc + (corner(lo, lo) - corner(lo, hi) - corner(hi, lo) + corner(hi, hi)) / 4.0
        out[i] = acc / h ** 2
    return out


def apply_A(prob: Problem3V, f, E, graddiv=True):
    """``A E = E - (k^2 + D) G0 (f E)`` (componentwise ``G0``)."""
    B = _conv(prob.G0hat, f[None] * E)
    S = prob.k ** 2 * B + (grad_div(B, prob.h) if graddiv else 0.0)
    return E - S


def apply_AH(prob: Problem3V, f, V):
    """``A^H V = V - f G0^H (k^2 V + D V)`` (D is real symmetric)."""
    W = prob.k ** 2 * V + grad_div(V, prob.h)
    return V - f[None] * _conv(prob.G0hat, W, conj=True)


def solve(prob: Problem3V, f, rhs, adjoint=False, tol=1e-10):
    op = apply_AH if adjoint else apply_A
    out = np.empty_like(rhs, dtype=np.complex128)
    its = []
    shape = rhs.shape[1:]
    for t in range(rhs.shape[0]):
        x, it, _ = krylov.bicgstab(lambda v: op(prob, f, v.reshape(shape)).reshape(-1), rhs[t].reshape(-1),
                                   tol=tol)
        out[t] = x.reshape(shape)
        its.append(it)
    return out, np.array(its)


def project(prob: Problem3V, f, E):
    """``y_t = Ht (I_3 x diag f) E_t`` for all t, shape (T, M)."""
    T = E.shape[0]
    return (prob.Ht @ (f[None, None] * E).reshape(T, -1).T).T


def forward(prob: Problem3V, f, tol=1e-10):
    E, _ = solve(prob, f, prob.E_in, tol=tol)
    return E, project(prob, f, E)


def residual(prob: Problem3V, y, y_meas):
    """``w = y - y_meas`` on the active receivers, zero on the others."""
    w = y - y_meas
    return w if prob.mask is None else w * prob.mask


def misfit(prob: Problem3V, f, y_meas, tol=1e-10):
    _, y = forward(prob, f, tol)
    return 0.5 * float(np.sum(np.abs(residual(prob, y, y_meas)) ** 2))


def gradient(prob: Problem3V, f, y_meas, tol=1e-10):
    """eq. 3Dgradient with u, v from eq. 3Du_and_v; returns (grad, D)."""
    E, _ = solve(prob, f, prob.E_in, tol=tol)
    y = project(prob, f, E)
    w = residual(prob, y, y_meas)
    D = 0.5 * float(np.sum(np.abs(w) ** 2))
    T, n = E.shape[0], prob.n
    q = (np.conj(prob.Ht).T @ w.T).T.reshape(T, 3, n, n, n)          # Ht^H w
    V, _ = solve(prob, f, f[None, None] * q, adjoint=True, tol=tol)
    g = np.zeros((n, n, n))
    for t in range(T):
        W = prob.k ** 2 * V[t] + grad_div(V[t], prob.h)
        p = _conv(prob.G0hat, W, conj=True)
        g += np.real(np.sum(np.conj(E[t]) * (q[t] + p), axis=0))
    return g, D


def reconstruct(prob: Problem3V, y_meas, gamma, tau, alpha=0.96, K=10, lo=0.0, hi=2.0, inner=100, tol=1e-10,
                f0=None):
    """CISOR on the vectorial model: relaxed FISTA (eqs. algo1-algo3) with the
    gradient of eq. 3Dgradient and the 3D TV/box prox."""
    from . import fista
    f0 = np.zeros((prob.n,) * 3) if f0 is None else f0

    def grad_fn(s):
        return gradient(prob, s, y_meas, tol=tol)

    return fista.relaxed_fista(grad_fn, f0, gamma, tau, alpha, K, lo, hi, inner)
