"""Closed-form references used to pin the oracle (independent of it).

Scattering of a plane wave by a homogeneous circular cylinder (textbook
separation of variables).  With background wavenumber ``k0``, cylinder
wavenumber ``k1 = k0 sqrt(eps)`` and radius ``R``, the incident plane wave
``exp(i k0 r cos(phi - theta)) = sum_n i^n J_n(k0 r) exp(i n (phi - theta))``
produces the outgoing scattered field

    u_sc(r, phi) = sum_n i^n a_n H_n^(1)(k0 r) exp(i n (phi - theta)),   r > R,

where continuity of ``u`` and ``du/dr`` at ``r = R`` gives

    a_n = [k1 J_n'(k1 R) J_n(k0 R) - k0 J_n(k1 R) J_n'(k0 R)]
          / [k0 J_n(k1 R) H_n'(k0 R) - k1 J_n'(k1 R) H_n(k0 R)].
"""

from __future__ import annotations

import numpy as np
from scipy import special


def sphere_scattered_field(k0, eps, R, dhat, rx, lmax=None):
    """Scalar plane wave exp(i k0 dhat.r) scattered by a homogeneous sphere of
    radius R (the 3D analogue of the cylinder): with the expansion
    exp(i k r cos g) = sum_l (2l+1) i^l j_l(k r) P_l(cos g),
    u_sc = sum_l (2l+1) i^l a_l h_l^(1)(k0 r) P_l(cos g), and a_l from continuity of
    u and du/dr at r = R (same formula as the cylinder with spherical Bessel
    functions)."""
    k1 = k0 * np.sqrt(eps)
    if lmax is None:
        lmax = int(np.ceil(k1 * R + 4 * (k1 * R) ** (1 / 3) + 12))
    r = np.linalg.norm(rx, axis=1)
    cg = rx @ np.asarray(dhat) / r
    out = np.zeros(rx.shape[0], dtype=np.complex128)
    for l in range(lmax + 1):
        j0, j1 = special.spherical_jn(l, k0 * R), special.spherical_jn(l, k1 * R)
        dj0, dj1 = special.spherical_jn(l, k0 * R, True), special.spherical_jn(l, k1 * R, True)
        h0 = j0 + 1j * special.spherical_yn(l, k0 * R)
        dh0 = dj0 + 1j * special.spherical_yn(l, k0 * R, True)
        a = (k1 * dj1 * j0 - k0 * j1 * dj0) / (k0 * j1 * dh0 - k1 * dj1 * h0)
        hr = special.spherical_jn(l, k0 * r) + 1j * special.spherical_yn(l, k0 * r)
        out += (2 * l + 1) * (1j ** l) * a * hr * special.eval_legendre(l, cg)
    return out


def ball_volume_fraction(n, h, R, sub=8):
    """Fraction of each voxel inside a centred ball (supersampled on cut voxels)."""
    c = (np.arange(n) - (n - 1) / 2) * h
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
    half = h / 2
    rmin = np.sqrt(np.maximum(abs(X) - half, 0) ** 2 + np.maximum(abs(Y) - half, 0) ** 2
                   + np.maximum(abs(Z) - half, 0) ** 2)
    rmax = np.sqrt((abs(X) + half) ** 2 + (abs(Y) + half) ** 2 + (abs(Z) + half) ** 2)
    fr = np.where(rmax <= R, 1.0, 0.0)
    cut = (rmin < R) & (rmax > R)
    o = (np.arange(sub) + 0.5) / sub * h - half
    ox, oy, oz = np.meshgrid(o, o, o, indexing="ij")
    for i, j, l in zip(*np.nonzero(cut)):
        fr[i, j, l] = ((X[i, j, l] + ox) ** 2 + (Y[i, j, l] + oy) ** 2 + (Z[i, j, l] + oz) ** 2 <= R * R).mean()
    return fr


def cylinder_scattered_field(k0, eps, R, theta, rx, nmax=None):
    """Scattered field at receiver positions ``rx`` (M, 2) for plane-wave angle theta."""
    k1 = k0 * np.sqrt(eps)
    if nmax is None:
        nmax = int(np.ceil(k1 * R + 4 * (k1 * R) ** (1 / 3) + 12))
    r = np.hypot(rx[:, 0], rx[:, 1])
    phi = np.arctan2(rx[:, 1], rx[:, 0])
    out = np.zeros(rx.shape[0], dtype=np.complex128)
    for n in range(-nmax, nmax + 1):
        j0, j1 = special.jv(n, k0 * R), special.jv(n, k1 * R)
        dj0, dj1 = special.jvp(n, k0 * R), special.jvp(n, k1 * R)
        h0, dh0 = special.hankel1(n, k0 * R), special.h1vp(n, k0 * R)
        a = (k1 * dj1 * j0 - k0 * j1 * dj0) / (k0 * j1 * dh0 - k1 * dj1 * h0)
        out += (1j ** n) * a * special.hankel1(n, k0 * r) * np.exp(1j * n * (phi - theta))
    return out
