"""Discretised Green's function (FP64).

The Lippmann-Schwinger equation ("Problem Formulation") is
``u(r) = u_in(r) + k^2 int g(r - r') f(r') u(r') dr'`` with the outgoing
free-space Green's function (eq. scalarGreens): in 2D ``(i/4) H0^(1)(k_b r)``,
in 3D ``exp(i k_b r) / (4 pi r)``.  Reading of the paper: the 2D sign is taken
as ``+i/4`` -- the outgoing solution that matches the 3D ``exp(+i k r)``
convention; the printed ``-j/4`` does not satisfy the radiation condition with
that time convention, and the cylinder Bessel-series test fails for it.

Discretisation (eqs. discrete2D_measurement / discrete2D_constraint; the
quadrature is not given in 2D, the 3D appendix uses ``delta^3`` point
quadrature): ``f u`` is taken constant on each pixel and the pixel is replaced
by the disk (2D) or ball (3D) of equal area/volume, radius ``a``.  The cell
integrals then have closed forms (Graf addition theorem / mean-value property
of Helmholtz solutions):

2D, ``a = h / sqrt(pi)``, ``c = k^2 / k_b^2 = 1/eps_b``:
  self   ``K(0)   = c [ (i pi/2) k_b a H1^(1)(k_b a) - 1 ]``
  other  ``K(rho) = c (i pi/2) k_b a J1(k_b a) H0^(1)(k_b rho)``   (rho >= a)
3D, ``a = h (3/(4 pi))^(1/3)``:
  self   ``K(0) = c [ (1 - i k_b a) exp(i k_b a) - 1 ]``
  other  ``K(d) = c (4 pi / k_b) (sin k_b a - k_b a cos k_b a) exp(i k_b d)/(4 pi d)``

``G[p, q] = K(|r_p - r_q|)`` and ``H[m, q] = K(|r_m - r_q|)`` (receivers lie
outside the grid), so ``k^2`` and the cell measure are folded into ``G`` and
``H`` and ``y = H diag(u) f`` is the physical scattered field.

Pinned by: quadrature of the cell integrals (tests compare with
``scipy.integrate``), the cylinder Bessel series, brute-force dense solves
(which check the FFT embedding below against ``dense_G``).
"""

from __future__ import annotations

import numpy as np
from scipy import special

from .geometry import pixel_positions_2d, pixel_positions_3d


def cell_radius(h: float, dim: int) -> float:
    if dim == 2:
        return h / np.sqrt(np.pi)
    return h * (3.0 / (4.0 * np.pi)) ** (1.0 / 3.0)


def kernel(rho, k: float, h: float, dim: int, eps_b: float = 1.0) -> np.ndarray:
    """Cell-integrated Green's function ``K(rho)`` (complex128, same shape as rho)."""
    rho = np.asarray(rho, dtype=np.float64)
    kb = k * np.sqrt(eps_b)
    c = 1.0 / eps_b
    a = cell_radius(h, dim)
    ka = kb * a
    out = np.empty(rho.shape, dtype=np.complex128)
    zero = rho == 0.0
    nz = ~zero
    if dim == 2:
        out[zero] = c * (0.5j * np.pi * ka * special.hankel1(1, ka) - 1.0)
        out[nz] = c * 0.5j * np.pi * ka * special.j1(ka) * special.hankel1(0, kb * rho[nz])
    else:
        out[zero] = c * ((1.0 - 1j * ka) * np.exp(1j * ka) - 1.0)
        d = rho[nz]
        out[nz] = (c * (4.0 * np.pi / kb) * (np.sin(ka) - ka * np.cos(ka))
                   * np.exp(1j * kb * d) / (4.0 * np.pi * d))
    return out


def padded_kernel(n: int, h: float, k: float, dim: int, eps_b: float = 1.0) -> np.ndarray:
    """Kernel on the ``(2n)^dim`` circulant grid.

    Offset ``j`` along an axis stands for distance ``j`` (``j < n``) or
    ``2n - j`` (``j > n``) pixels; offset ``n`` is never reached by the cropped
    output and is set to 0.  Circular convolution of this kernel with the
    zero-padded ``f u`` then equals ``G (f u)`` on the first ``n`` samples.
    """
    P = 2 * n
    j = np.arange(P)
    d = np.where(j < n, j, P - j).astype(np.float64)
    valid = j != n
    grids = np.meshgrid(*([d] * dim), indexing="ij")
    rho = h * np.sqrt(sum(g * g for g in grids))
    Kc = kernel(rho, k, h, dim, eps_b)
    mask = np.ones((P,) * dim, dtype=bool)
    for ax in range(dim):
        shape = [1] * dim
        shape[ax] = P
        mask &= valid.reshape(shape)
    return np.where(mask, Kc, 0.0)


def kernel_spectrum(n: int, h: float, k: float, dim: int, eps_b: float = 1.0) -> np.ndarray:
    """``Ghat = FFT(padded kernel)`` on the ``(2n)^dim`` grid."""
    return np.fft.fftn(padded_kernel(n, h, k, dim, eps_b))


def dense_G(n: int, h: float, k: float, dim: int, eps_b: float = 1.0) -> np.ndarray:
    """Dense ``N x N`` matrix ``G[p, q] = K(|r_p - r_q|)`` (brute force; small n only)."""
    pos = pixel_positions_2d(n, h) if dim == 2 else pixel_positions_3d(n, h)
    diff = pos[:, None, :] - pos[None, :, :]
    return kernel(np.sqrt((diff ** 2).sum(-1)), k, h, dim, eps_b)


def receiver_matrix(rx: np.ndarray, n: int, h: float, k: float, eps_b: float = 1.0) -> np.ndarray:
    """``H[m, q] = K(|r_m - r_q|)``, shape ``(M, N)``; receivers must lie off-grid."""
    dim = rx.shape[1]
    pos = pixel_positions_2d(n, h) if dim == 2 else pixel_positions_3d(n, h)
    diff = rx[:, None, :] - pos[None, :, :]
    rho = np.sqrt((diff ** 2).sum(-1))
    if np.any(rho < cell_radius(h, dim)):
        raise ValueError("receiver inside a grid cell")
    return kernel(rho, k, h, dim, eps_b)
