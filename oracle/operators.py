"""Matrix-free forward operator ``A = I - G diag(f)`` and its adjoint (FP64).

eq. A_def defines ``A := I - G diag(f)``; the paper applies ``G`` as a
convolution computed by FFT ("Proposed Method", after Prop. 1).  Fields have
shape ``(..., n, ..., n)`` (leading batch axes allowed); ``f`` has shape
``(n, ..., n)`` and ``Ghat`` is the spectrum of the padded kernel on the
``(2n)^d`` grid (``green.kernel_spectrum``).

Because the padded kernel is even in every axis, ``Ghat`` is even too and
``G`` is complex symmetric (``G^T = G``); hence ``G^H = conj(G)`` is the
convolution with ``conj(Ghat)``.  The adjoint is therefore
``A^H x = x - diag(f) conj(G) x`` -- note that ``f`` multiplies after the
convolution in the adjoint and before it in the forward operator.

Pinned by: brute-force dense ``A`` (``green.dense_G``) on small grids, and the
inner-product (dot) test ``<A x, y> = <x, A^H y>``.
"""

from __future__ import annotations

import numpy as np


def _conv(Ghat: np.ndarray, x: np.ndarray, conj: bool = False) -> np.ndarray:
    d = Ghat.ndim
    n = Ghat.shape[0] // 2
    axes = tuple(range(-d, 0))
    pad = np.zeros(x.shape[:-d] + Ghat.shape, dtype=np.complex128)
    pad[(Ellipsis,) + (slice(0, n),) * d] = x
    spec = np.fft.fftn(pad, axes=axes)
    spec *= np.conj(Ghat) if conj else Ghat
    full = np.fft.ifftn(spec, axes=axes)
    return full[(Ellipsis,) + (slice(0, n),) * d]


def apply_G(Ghat, x):
    """``G x`` (convolution with the Green's kernel, cropped to the grid)."""
    return _conv(Ghat, x, conj=False)


def apply_GH(Ghat, x):
    """``G^H x``."""
    return _conv(Ghat, x, conj=True)


def apply_A(Ghat, f, x):
    """``A x = x - G (f x)``."""
    return x - apply_G(Ghat, f * x)


def apply_AH(Ghat, f, x):
    """``A^H x = x - f (G^H x)``."""
    return x - f * apply_GH(Ghat, x)
