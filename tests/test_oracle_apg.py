"""Pins of the oracle's monotone APG (the Li-Lin comparison method of the
paper's "Proposed Method" section)."""

import numpy as np

from oracle import apg


def _least_squares(m=240, n=200, spread=1e-4, seed=0):
    """Ill-conditioned least squares: singular values log-spaced down to sqrt(spread)."""
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((m, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = np.sqrt(np.logspace(0, np.log10(spread), n))
    A = (U * s) @ V.T
    b = rng.standard_normal(m)
    x_star = np.linalg.lstsq(A, b, rcond=None)[0]
    F = lambda x: 0.5 * float(np.sum((A @ x - b) ** 2))
    grad = lambda x: (A.T @ (A @ x - b), F(x))
    return A, b, x_star, F, grad, float(s[0] ** 2)


def test_convex_rate_bound():
    """Li and Lin's convex bound F(x_{k+1}) - F* <= 2 ||x_0 - x*||^2 / (a_y (k+1)^2)
    at every k, on a problem where plain proximal gradient (ISTA) violates it."""
    A, b, x_star, F, grad, L = _least_squares()
    a = 1.0 / L
    x0 = np.zeros(A.shape[1])
    K = 400
    _, hist = apg.monotone_apg(grad, F, lambda w, g: w, x0, a, a, K)
    Fs = F(x_star)
    r2 = float(np.sum((x0 - x_star) ** 2))
    gaps = np.array(hist["F"]) - Fs
    bound = 2 * r2 / (a * (np.arange(1, K + 1) + 1) ** 2)
    assert np.all(gaps <= bound)
    # ISTA (gradient descent) from the same start breaks the bound on this problem
    x = x0.copy()
    ista_violates = False
    for k in range(1, K + 1):
        x = x - a * grad(x)[0]
        ista_violates |= F(x) - Fs > 2 * r2 / (a * (k + 1) ** 2)
    assert ista_violates


def test_monotone_on_a_nonconvex_problem():
    """With a_x < 1/L the ISTA estimate cannot increase F, so neither can the
    selected iterate: F(x_{k+1}) <= F(x_k) for a nonconvex smooth D plus a box."""
    rng = np.random.default_rng(3)
    n = 50
    A = rng.standard_normal((40, n)) / np.sqrt(40)
    b = rng.standard_normal(40)
    beta = 2.0
    D = lambda x: 0.5 * float(np.sum((A @ x - b) ** 2)) + beta * float(np.sum(np.cos(3 * x)))
    grad = lambda x: (A.T @ (A @ x - b) - 3 * beta * np.sin(3 * x), D(x))
    L = np.linalg.norm(A, 2) ** 2 + 9 * beta
    lo, hi = -1.0, 1.5
    prox = lambda w, g: np.clip(w, lo, hi)
    x0 = rng.uniform(lo, hi, n)
    _, hist = apg.monotone_apg(grad, D, prox, x0, 0.9 / L, 0.9 / L, 300)
    F = [D(x0)] + hist["F"]
    assert np.all(np.diff(F) <= 1e-12 * np.abs(F[1:]))
    assert any(hist["took_z"]) and not all(hist["took_z"])
    # and the accelerated estimate alone (always taking z) is not monotone here
    assert np.any(np.diff([D(x0)] + hist["F_z"]) > 0)


def test_converges_to_least_squares_and_first_step_is_ista():
    A, b, x_star, F, grad, L = _least_squares(m=80, n=30, spread=1e-2, seed=5)
    a = 1.0 / L
    x, hist = apg.monotone_apg(grad, F, lambda w, g: w, np.zeros(30), a, a, 3000)
    assert np.linalg.norm(x - x_star) < 1e-8 * np.linalg.norm(x_star)
    x1 = hist["x"][0]
    assert np.array_equal(x1, 0 - a * grad(np.zeros(30))[0])


def _fista_textbook(grad, prox, x0, a, K):
    """Beck and Teboulle's FISTA: x_k = prox(y_k - a grad(y_k)),
    t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2, y_{k+1} = x_k + ((t_k - 1)/t_{k+1})(x_k - x_{k-1})."""
    x_prev = x0.copy()
    y = x0.copy()
    t = 1.0
    out = []
    for _ in range(K):
        x = prox(y - a * grad(y)[0], a)
        t_next = (1.0 + np.sqrt(1.0 + 4.0 * t * t)) / 2.0
        y = x + ((t - 1.0) / t_next) * (x - x_prev)
        x_prev, t = x, t_next
        out.append(x)
    return out


def test_reduces_to_fista_when_the_accelerated_estimate_always_wins():
    A, b, x_star, F, grad, L = _least_squares(m=120, n=100, spread=1e-3, seed=2)
    a = 1.0 / L
    x0 = np.zeros(100)
    K = 150
    _, hist = apg.monotone_apg(grad, F, lambda w, g: w, x0, a, a, K)
    took = hist["took_z"]
    first_v = took.index(False) if not all(took) else K      # FISTA's first ripple
    assert first_v >= 50
    ref = _fista_textbook(grad, lambda w, g: w, x0, a, K)
    for k in range(first_v):
        assert np.allclose(hist["x"][k], ref[k], rtol=0, atol=1e-12 * (1 + np.abs(ref[k]).max()))
    # where FISTA's objective goes up, the monotone method takes the ISTA estimate instead
    if first_v < K:
        assert F(ref[first_v]) > F(ref[first_v - 1]) or F(ref[first_v]) > hist["F_v"][first_v]


def test_estimate_sequence_identity_whichever_estimate_is_taken():
    """u_k = x_{k-1} + t_{k-1}(z_k - x_{k-1}) moves by -a t_k grad D(y_k) at every
    iteration when the prox is the identity (an algebraic consequence of the
    extrapolation and the z update), also after iterations that took v."""
    rng = np.random.default_rng(11)
    n = 40
    A = rng.standard_normal((30, n)) / np.sqrt(30)
    b = rng.standard_normal(30)
    beta = 1.5
    D = lambda x: 0.5 * float(np.sum((A @ x - b) ** 2)) + beta * float(np.sum(np.cos(3 * x)))
    grad = lambda x: (A.T @ (A @ x - b) - 3 * beta * np.sin(3 * x), D(x))
    L = np.linalg.norm(A, 2) ** 2 + 9 * beta
    a = 0.9 / L
    x0 = rng.uniform(-1, 1, n)
    K = 200
    _, hist = apg.monotone_apg(grad, D, lambda w, g: w, x0, a, a, K)
    took = hist["took_z"]
    assert any(took) and not all(took)
    xs = [x0] + hist["x"]            # x_1 = x_0, then x_2, x_3, ...: xs[j] = x_{j+1}
    zs = [x0] + hist["z"]            # z_1 = x_0, then z_2, ...
    ts = [1.0] + hist["t"]           # t_1 = 1, then t_2, ...
    x_of = lambda k: x0 if k <= 1 else xs[k - 1]      # x_k, k >= 0 (x_0 = x_1)
    u = lambda k: x_of(k - 1) + (0.0 if k == 1 else ts[k - 2]) * (zs[k - 1] - x_of(k - 1))
    for k in range(1, K):
        step = u(k + 1) - u(k)
        want = -a * ts[k - 1] * hist["g_y"][k - 1]
        assert np.allclose(step, want, rtol=0, atol=1e-9 * (1 + np.abs(want).max())), k


def test_cisor_objective_is_monotone_and_consistent():
    """The CISOR wrapper on a small 2D problem: the selected objective never
    goes up, and F(x_{k+1}) is D + tau TV at the selected iterate."""
    from oracle import cisor, stepsize, tv
    from synth import disks_2d
    n, h, T, M = 12, 1 / 8, 4, 16
    prob = cisor.make_problem_2d(n, h, T, M, n * h)
    ftrue = disks_2d(n, 1, count=2, radius_px=(2, 3), eps_range=(1.1, 1.4))
    _, y = cisor.forward(prob, ftrue, tol=1e-12)
    gamma = 0.5 / stepsize.born_lipschitz(prob)
    tau = 1e-3
    x, hist = apg.cisor_apg(prob, y, gamma, gamma, tau, K=6, tol=1e-12)
    F = hist["F"]
    assert np.all(np.diff(F) <= 1e-12 * np.abs(F[1:]))
    assert np.isclose(F[-1], cisor.misfit(prob, x, y, tol=1e-12) + tau * tv.tv_value(x), rtol=1e-10)
