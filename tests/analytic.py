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
