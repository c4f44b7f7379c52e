"""Pins of the oracle's TV proximal map (eq. R_def, step algo1)."""

import numpy as np
import pytest
from scipy.optimize import lsq_linear

from oracle import tv


def test_grad_div_adjoint():
    rng = np.random.default_rng(0)
    for shape in [(7, 9), (4, 5, 6)]:
        x = rng.standard_normal(shape)
        p = rng.standard_normal((len(shape),) + shape)
        assert abs(np.sum(tv.grad(x) * p) + np.sum(x * tv.div(p))) < 1e-12


def test_tv_value_closed_form():
    """Isotropic TV of a ramp and of a single step."""
    n = 6
    ramp = np.outer(np.arange(n), np.ones(n)) * 0.5      # varies along axis 0
    assert abs(tv.tv_value(ramp) - 0.5 * (n - 1) * n) < 1e-12
    x = np.zeros((4, 4))
    x[1, 2] = 1.0   # neighbours: diffs at (0,2) down, (1,1) right, (1,2) both
    expected = 1.0 + 1.0 + np.sqrt(2.0)
    assert abs(tv.tv_value(x) - expected) < 1e-12


def test_prox_special_cases():
    rng = np.random.default_rng(1)
    z = rng.uniform(-0.5, 2.5, (12, 12))
    # lam = 0: plain projection on the box
    assert np.array_equal(tv.prox_tv_box(z, 0.0, 0.0, 2.0), np.clip(z, 0.0, 2.0))
    # constant image: stays constant (clipped)
    c = np.full((9, 9), 2.7)
    assert np.allclose(tv.prox_tv_box(c, 0.3, 0.0, 2.0, iters=50), 2.0)
    c = np.full((9, 9), 0.7)
    assert np.allclose(tv.prox_tv_box(c, 0.3, 0.0, 2.0, iters=50), 0.7)
    # very large lam: the constant clip(mean)
    x = tv.prox_tv_box(z, 1e4, -np.inf, np.inf, iters=3000)
    assert np.allclose(x, z.mean(), atol=1e-5)
    x = tv.prox_tv_box(z - 1.5, 1e4, 0.0, 2.0, iters=3000)
    assert np.allclose(x, np.clip((z - 1.5).mean(), 0, 2), atol=1e-5)


def test_prox_one_dimensional_image_matches_1d_tv():
    """An image varying along one axis has a prox that varies along that axis only,
    equal to the 1-D TV prox of the profile with the same lam.  The 1-D prox is
    g - lam D^T p* with p* = argmin_{|p|<=1} 1/2||g - lam D^T p||^2 (bounded LS)."""
    rng = np.random.default_rng(2)
    m = 20
    g = np.cumsum(rng.standard_normal(m)) * 0.3
    lam = 0.4
    z = np.repeat(g[:, None], 7, axis=1)
    x = tv.prox_tv_box(z, lam, iters=4000)
    D = np.zeros((m - 1, m))
    D[np.arange(m - 1), np.arange(m - 1)] = -1
    D[np.arange(m - 1), np.arange(1, m)] = 1
    res = lsq_linear(lam * D.T, g, bounds=(-1, 1), tol=1e-14, lsmr_tol="auto", max_iter=10000)
    x1 = g - lam * D.T @ res.x
    assert np.allclose(x, x1[:, None], atol=1e-6)


def test_prox_duality_gap_closes():
    """Primal-dual gap of the box-constrained problem goes to zero (weak duality
    bounds the primal from below by the dual for every feasible p)."""
    rng = np.random.default_rng(3)
    z = rng.uniform(-0.2, 1.5, (16, 16))
    lam = 0.15
    x, p = tv.prox_tv_box(z, lam, 0.0, 1.0, iters=3000, return_dual=True)
    P = tv.primal_value(x, z, lam)
    Dv = tv.dual_value(p, z, lam, 0.0, 1.0)
    assert Dv <= P + 1e-12
    assert P - Dv < 1e-7 * P
    # after few iterations the gap is still open, and positive
    x5, p5 = tv.prox_tv_box(z, lam, 0.0, 1.0, iters=5, return_dual=True)
    assert tv.primal_value(x5, z, lam) - tv.dual_value(p5, z, lam, 0.0, 1.0) > 1e-4


def test_prox_3d_duality_gap():
    rng = np.random.default_rng(4)
    z = rng.uniform(0, 1, (6, 7, 5))
    lam = 0.1
    x, p = tv.prox_tv_box(z, lam, 0.0, 0.8, iters=3000, return_dual=True)
    P = tv.primal_value(x, z, lam)
    assert P - tv.dual_value(p, z, lam, 0.0, 0.8) < 1e-7 * P
