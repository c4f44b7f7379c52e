"""Seeded phantom and noise generators.

Every generator takes an explicit integer seed and draws from
``numpy.random.default_rng(seed)``; nothing here depends on global state.
Phantoms return the relative permittivity contrast ``f = eps - eps_b`` on a
cell-centred grid (row-major, first index = x), as a float64 array.
"""

from __future__ import annotations

import numpy as np


def _centres(n: int) -> np.ndarray:
    """Pixel-centre coordinates in pixel units, centred on the grid middle."""
    return np.arange(n, dtype=np.float64) - (n - 1) / 2.0


def disks_2d(n: int, seed: int, count: int = 3, radius_px=(2.0, 5.0),
             eps_range=(1.1, 1.5), eps_b: float = 1.0) -> np.ndarray:
    """Disks of uniform permittivity, later disks overwriting earlier ones.

    Radii are uniform in ``radius_px`` (pixels); centres are drawn so each disk
    lies inside the grid; each disk's permittivity is uniform in ``eps_range``.
    """
    rng = np.random.default_rng(seed)
    c = _centres(n)
    X, Y = np.meshgrid(c, c, indexing="ij")
    f = np.zeros((n, n))
    half = (n - 1) / 2.0
    for _ in range(count):
        r = rng.uniform(*radius_px)
        lim = max(half - r, 0.0)
        cx, cy = rng.uniform(-lim, lim, size=2)
        eps = rng.uniform(*eps_range)
        f[(X - cx) ** 2 + (Y - cy) ** 2 <= r * r] = eps - eps_b
    return f


def ellipses_2d(n: int, seed: int, inner: int = 7, outer_axes=(0.6, 0.9),
                inner_axes=(0.08, 0.3), eps_range=(1.0, 2.0),
                eps_b: float = 1.0) -> np.ndarray:
    """A Shepp-Logan-like phantom of random ellipses (not the canonical table).

    One outer ellipse centred on the grid with semi-axes uniform in
    ``outer_axes`` times the half-width, then ``inner`` ellipses with semi-axes
    uniform in ``inner_axes`` times the half-width, random orientation and a
    centre inside the outer ellipse.  Each shape's permittivity is uniform in
    ``eps_range``; later shapes overwrite earlier ones.
    """
    rng = np.random.default_rng(seed)
    hw = n / 2.0
    c = _centres(n)
    X, Y = np.meshgrid(c, c, indexing="ij")
    f = np.zeros((n, n))

    def paint(cx, cy, a, b, th, eps):
        ct, st = np.cos(th), np.sin(th)
        xr = (X - cx) * ct + (Y - cy) * st
        yr = -(X - cx) * st + (Y - cy) * ct
        f[(xr / a) ** 2 + (yr / b) ** 2 <= 1.0] = eps - eps_b

    A, B = rng.uniform(*outer_axes, size=2) * hw
    paint(0.0, 0.0, A, B, rng.uniform(0, np.pi), rng.uniform(*eps_range))
    for _ in range(inner):
        a, b = rng.uniform(*inner_axes, size=2) * hw
        rad = np.sqrt(rng.uniform(0, 1)) * 0.6
        phi = rng.uniform(0, 2 * np.pi)
        cx, cy = rad * A * np.cos(phi), rad * B * np.sin(phi)
        paint(cx, cy, a, b, rng.uniform(0, np.pi), rng.uniform(*eps_range))
    return f


def disk_area_fraction(n: int, h: float, radius: float, sub: int = 32) -> np.ndarray:
    """Fraction of each pixel's area inside a centred disk of ``radius``.

    Pixel centres at ``(i - (n-1)/2) h``.  Interior and exterior pixels are
    exact (1 and 0); pixels cut by the circle are supersampled ``sub x sub``.
    """
    c = _centres(n) * h
    X, Y = np.meshgrid(c, c, indexing="ij")
    half = h / 2.0
    rmin = np.sqrt(np.maximum(np.abs(X) - half, 0) ** 2 + np.maximum(np.abs(Y) - half, 0) ** 2)
    rmax = np.sqrt((np.abs(X) + half) ** 2 + (np.abs(Y) + half) ** 2)
    frac = np.where(rmax <= radius, 1.0, 0.0)
    cut = (rmin < radius) & (rmax > radius)
    o = (np.arange(sub) + 0.5) / sub * h - half
    ox, oy = np.meshgrid(o, o, indexing="ij")
    for i, j in zip(*np.nonzero(cut)):
        inside = (X[i, j] + ox) ** 2 + (Y[i, j] + oy) ** 2 <= radius * radius
        frac[i, j] = inside.mean()
    return frac


def ellipsoids_3d(n: int, seed: int, count_range=(1, 4), axes=(0.1, 0.35),
                  eps_range=(1.0, 1.3), eps_b: float = 1.0) -> np.ndarray:
    """Random axis-aligned ellipsoids inside an ``n^3`` grid (later overwrite)."""
    rng = np.random.default_rng(seed)
    hw = n / 2.0
    c = _centres(n)
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
    f = np.zeros((n, n, n))
    count = int(rng.integers(count_range[0], count_range[1] + 1))
    for _ in range(count):
        ax = rng.uniform(*axes, size=3) * hw
        lim = np.maximum(hw - 1 - ax, 0.0)
        ctr = rng.uniform(-lim, lim)
        eps = rng.uniform(*eps_range)
        m = (((X - ctr[0]) / ax[0]) ** 2 + ((Y - ctr[1]) / ax[1]) ** 2
             + ((Z - ctr[2]) / ax[2]) ** 2) <= 1.0
        f[m] = eps - eps_b
    return f


def complex_normal(shape, seed: int) -> np.ndarray:
    """Standard circular complex normal draws ``(a + i b)/sqrt(2)``, ``a, b ~ N(0,1)``."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(shape)
    b = rng.standard_normal(shape)
    return (a + 1j * b) / np.sqrt(2.0)


def random_field(shape, seed: int) -> np.ndarray:
    """Uniform random complex values in the unit square (generic test vectors)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1, 1, shape) + 1j * rng.uniform(-1, 1, shape)


def mixed_2d(n: int, seed: int, count_range=(1, 6), axes=(0.05, 0.35), eps_range=(1.0, 2.0),
             eps_b: float = 1.0) -> np.ndarray:
    """A random mix of disks and ellipses (later shapes overwrite earlier).

    Semi-axes uniform in ``axes`` times the half-width (equal for disks),
    centres uniform such that the shape's bounding circle stays in the grid,
    random orientation, permittivity uniform in ``eps_range`` per shape.
    """
    rng = np.random.default_rng(seed)
    hw = n / 2.0
    c = _centres(n)
    X, Y = np.meshgrid(c, c, indexing="ij")
    f = np.zeros((n, n))
    count = int(rng.integers(count_range[0], count_range[1] + 1))
    for _ in range(count):
        a = rng.uniform(*axes) * hw
        b = a if rng.uniform() < 0.5 else rng.uniform(*axes) * hw
        lim = max(hw - 1 - max(a, b), 0.0)
        cx, cy = rng.uniform(-lim, lim, size=2)
        th = rng.uniform(0, np.pi)
        ct, st = np.cos(th), np.sin(th)
        xr = (X - cx) * ct + (Y - cy) * st
        yr = -(X - cx) * st + (Y - cy) * ct
        f[(xr / a) ** 2 + (yr / b) ** 2 <= 1.0] = rng.uniform(*eps_range) - eps_b
    return f
