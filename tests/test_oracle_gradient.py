"""Pins of the oracle's Prop. 1 gradient and the Born step-size helper."""

import numpy as np
import pytest

from oracle import cisor, green, stepsize
from synth import complex_normal, disks_2d

K = 2 * np.pi


def _setup(n=10, T=3, M=12, seed=0, born=False):
    h = 1 / 8
    prob = cisor.make_problem_2d(n, h, T=T, M=M, rx_radius=n * h, born=born)
    f = disks_2d(n, seed, count=2, radius_px=(1.5, 3.0), eps_range=(1.2, 1.6))
    y_meas = 0.3 * complex_normal((T, M), seed + 100)
    return prob, f, y_meas


def test_prop1_gradient_equals_dense_jacobian():
    """eq. gradient (Prop. 1) equals Re(J^H w) with the explicit Jacobian from its proof."""
    prob, f, y = _setup()
    g, D = cisor.gradient(prob, f, y, tol=1e-13)
    gd, Dd = cisor.gradient_dense(prob, f, y, green.dense_G(prob.n, prob.h, K, 2))
    assert abs(D - Dd) < 1e-11 * abs(Dd)
    assert np.linalg.norm(g - gd) < 1e-9 * np.linalg.norm(gd)


def test_prop1_gradient_matches_central_differences():
    """Directional derivative of D (eq. D_def) by central differences."""
    prob, f, y = _setup(n=8, seed=3)
    g, _ = cisor.gradient(prob, f, y, tol=1e-13)
    rng = np.random.default_rng(1)
    for _ in range(3):
        d = rng.standard_normal(f.shape)
        eps = 1e-4
        fd = (cisor.misfit(prob, f + eps * d, y, tol=1e-14)
              - cisor.misfit(prob, f - eps * d, y, tol=1e-14)) / (2 * eps)
        assert abs(fd - np.sum(g * d)) < 1e-7 * max(1.0, abs(fd))


def test_gradient_pixelwise_fd():
    prob, f, y = _setup(n=6, T=2, M=8, seed=5)
    g, _ = cisor.gradient(prob, f, y, tol=1e-14)
    for (i, j) in [(0, 0), (2, 3), (5, 5)]:
        e = np.zeros_like(f)
        e[i, j] = 1.0
        eps = 1e-5
        fd = (cisor.misfit(prob, f + eps * e, y, tol=1e-14)
              - cisor.misfit(prob, f - eps * e, y, tol=1e-14)) / (2 * eps)
        assert abs(fd - g[i, j]) < 1e-7 * max(1.0, np.abs(g).max())


def test_born_model_gradient_is_linear_least_squares():
    """With u = u_in (linear method) D is the quadratic 1/2||B f - y||^2 with
    B = stacked [Re; Im] of H diag(u_in,t); its gradient is B^T (B f - y)."""
    prob, f, y = _setup(born=True)
    g, _ = cisor.gradient(prob, f, y)
    rows = []
    for t in range(prob.T):
        rows.append(prob.H * prob.u_in[t].reshape(1, -1))
    Bc = np.concatenate(rows, axis=0)
    B = np.concatenate([Bc.real, Bc.imag], axis=0)
    yv = np.concatenate([y.reshape(-1).real, y.reshape(-1).imag])
    gref = B.T @ (B @ f.reshape(-1) - yv)
    assert np.allclose(g.reshape(-1), gref, rtol=1e-11, atol=1e-12 * np.abs(gref).max())


def test_born_lipschitz_matches_dense_eigenvalue():
    prob, f, y = _setup(n=8, born=True)
    rows = [prob.H * prob.u_in[t].reshape(1, -1) for t in range(prob.T)]
    Bc = np.concatenate(rows, axis=0)
    B = np.concatenate([Bc.real, Bc.imag], axis=0)
    lam = np.linalg.eigvalsh(B.T @ B)[-1]
    est = stepsize.born_lipschitz(prob, iters=300)
    assert abs(est - lam) < 1e-6 * lam


def test_noise_snr():
    y = complex_normal((8, 32), 1)
    yn = cisor.add_noise(y, 40.0, seed=2)
    snr = 20 * np.log10(np.linalg.norm(y) / np.linalg.norm(yn - y))
    assert abs(snr - 40.0) < 1.0
