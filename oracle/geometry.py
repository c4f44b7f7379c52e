"""Grids, incident fields and receiver positions (FP64).

Grid: cell-centred samples ``x_i = (i - (n-1)/2) h`` for ``i = 0..n-1`` -- the
0-based form of the appendix's grid ``r_{l,s,t} = ((l - J/2 - 0.5) delta, ...)``
("Discretization" of the 3D appendix; the same convention is used in 2D).
Pixel ``q = i*n + j`` sits at ``(x_i, x_j)`` (row-major, first index = x).

Incident fields are plane waves ``u_in(r) = exp(i k_b dhat . r)`` with
``k_b = k sqrt(eps_b)`` (background wavenumber, "Problem Formulation").
Pinned by: the cylinder Bessel-series test (which fixes grid, wavenumber and
plane-wave phase conventions end to end) and the grid-symmetry tests.
"""

from __future__ import annotations

import numpy as np


def axis(n: int, h: float) -> np.ndarray:
    return (np.arange(n, dtype=np.float64) - (n - 1) / 2.0) * h


def pixel_positions_2d(n: int, h: float) -> np.ndarray:
    """(N, 2) array of pixel centres, row-major."""
    x = axis(n, h)
    X, Y = np.meshgrid(x, x, indexing="ij")
    return np.stack([X.ravel(), Y.ravel()], axis=1)


def pixel_positions_3d(n: int, h: float) -> np.ndarray:
    x = axis(n, h)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


def plane_wave_directions_2d(T: int) -> np.ndarray:
    """Unit propagation directions at uniform angles ``2 pi t / T``."""
    th = 2.0 * np.pi * np.arange(T) / T
    return np.stack([np.cos(th), np.sin(th)], axis=1)


def plane_waves(n: int, h: float, kb: float, dirs: np.ndarray) -> np.ndarray:
    """Incident fields ``exp(i kb dhat.r)`` on the grid, shape ``(T, n, ..., n)``."""
    dim = dirs.shape[1]
    pos = pixel_positions_2d(n, h) if dim == 2 else pixel_positions_3d(n, h)
    phase = kb * (pos @ dirs.T)                      # (N, T)
    return np.exp(1j * phase).T.reshape((dirs.shape[0],) + (n,) * dim)


def point_sources(n: int, h: float, kb: float, src: np.ndarray) -> np.ndarray:
    """Incident fields of unit point sources at ``src`` (``(T, dim)``), the
    background Green's function of the "Problem Formulation" section sampled at
    the pixel centres: ``(i/4) H0^(1)(kb |r - s|)`` in 2D,
    ``exp(i kb |r - s|) / (4 pi |r - s|)`` in 3D.  Shape ``(T, n, ..., n)``."""
    from scipy.special import hankel1
    dim = src.shape[1]
    pos = pixel_positions_2d(n, h) if dim == 2 else pixel_positions_3d(n, h)
    d = np.linalg.norm(pos[None, :, :] - src[:, None, :], axis=2)     # (T, N)
    u = 0.25j * hankel1(0, kb * d) if dim == 2 else np.exp(1j * kb * d) / (4 * np.pi * d)
    return u.reshape((src.shape[0],) + (n,) * dim)


def linear_arrays(count: int, spacing: float, x: float) -> np.ndarray:
    """Two linear detector arrays on the lines ``x = -x`` and ``x = +x``,
    ``count`` sensors each, ``spacing`` apart, centred on ``y = 0``."""
    ys = (np.arange(count) - (count - 1) / 2.0) * spacing
    left = np.stack([np.full(count, -x), ys], axis=1)
    right = np.stack([np.full(count, x), ys], axis=1)
    return np.concatenate([left, right])


def line_sources(x: float, max_deg: float = 60.0, step_deg: float = 5.0) -> np.ndarray:
    """Sources on the line ``x = -x`` at uniform azimuths (seen from the
    origin, measured from the -x axis) in ``[-max_deg, max_deg]``."""
    th = np.deg2rad(np.arange(-max_deg, max_deg + 1e-9, step_deg))
    return np.stack([np.full(th.size, -x), x * np.tan(th)], axis=1)


def ring_receivers(M: int, radius: float) -> np.ndarray:
    """``M`` receivers at ``radius (cos 2 pi m/M, sin 2 pi m/M)``."""
    ph = 2.0 * np.pi * np.arange(M) / M
    return radius * np.stack([np.cos(ph), np.sin(ph)], axis=1)


def cone_directions(T: int, half_angle_deg: float = 45.0) -> np.ndarray:
    """3D plane-wave directions on a downward cone of the given half-angle."""
    a = np.deg2rad(half_angle_deg)
    ph = 2.0 * np.pi * np.arange(T) / T
    return np.stack([np.sin(a) * np.cos(ph), np.sin(a) * np.sin(ph),
                     -np.cos(a) * np.ones(T)], axis=1)


def plane_receivers(side: int, extent: float, z: float) -> np.ndarray:
    """``side x side`` receivers on the plane ``z`` spanning ``[-extent, extent]^2``."""
    c = np.linspace(-extent, extent, side)
    X, Y = np.meshgrid(c, c, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), np.full(side * side, z)], axis=1)
