"""Pins of the oracle's relaxed FISTA (eqs. algo1-algo3) and of one full CISOR run."""

import numpy as np
import pytest

from oracle import cisor, fista, stepsize, tv
from synth import complex_normal, disks_2d


def _linear_problem(n=4, T=4, M=16, h=0.5):
    prob = cisor.make_problem_2d(n, h, T=T, M=M, rx_radius=n * h, born=True)
    rows = [prob.H * prob.u_in[t].reshape(1, -1) for t in range(T)]
    Bc = np.concatenate(rows, axis=0)
    B = np.concatenate([Bc.real, Bc.imag], axis=0)
    L = np.linalg.eigvalsh(B.T @ B)[-1]
    return prob, B, L


def _quad(B, y):
    def grad_fn(s):
        r = B @ s.reshape(-1) - y
        return (B.T @ r).reshape(s.shape), 0.5 * float(r @ r)
    return grad_fn


def _data(prob, f):
    yc = cisor.project(prob, f, prob.u_in)
    return yc, np.concatenate([yc.reshape(-1).real, yc.reshape(-1).imag])


def test_linear_model_converges_to_least_squares():
    """tau = 0, inactive box: relaxed FISTA minimises the quadratic Born misfit,
    whose minimiser is the least-squares solution."""
    prob, B, L = _linear_problem()
    ftrue = np.random.default_rng(0).uniform(0, 1, (4, 4))
    yc, yv = _data(prob, ftrue)
    yv = yv + 0.01 * np.random.default_rng(1).standard_normal(yv.shape)
    fstar = np.linalg.lstsq(B, yv, rcond=None)[0]
    grad_fn = _quad(B, yv)
    f, _ = fista.relaxed_fista(grad_fn, np.zeros((4, 4)), 1.0 / L, 0.0, 0.96, 4000,
                               lo=-np.inf, hi=np.inf)
    assert np.allclose(f.reshape(-1), fstar, atol=1e-8 * np.abs(fstar).max())
    # the same through the oracle's Prop. 1 gradient of the Born model
    yc_noisy = (yv[:yv.size // 2] + 1j * yv[yv.size // 2:]).reshape(yc.shape)
    f2, _ = fista.relaxed_fista(lambda s: cisor.gradient(prob, s, yc_noisy), np.zeros((4, 4)),
                                1.0 / L, 0.0, 0.96, 4000, lo=-np.inf, hi=np.inf)
    assert np.allclose(f2.reshape(-1), fstar, atol=1e-8 * np.abs(fstar).max())


def test_energy_inequality_prop3():
    """Proof of Prop. 3: for gamma <= (1 - alpha^2)/(2L),
    F(f_k) + (1/(2 gamma) - L)||f_k - f_{k-1}||^2 is non-increasing (tau = 0 with an
    active box makes the prox exact)."""
    prob, B, L = _linear_problem(h=1 / 8)
    ftrue = np.random.default_rng(3).uniform(0, 1, (4, 4))
    _, yv = _data(prob, ftrue)
    alpha = 0.96
    gamma = (1 - alpha ** 2) / (2 * L)
    grad_fn = _quad(B, yv)
    f, hist = fista.relaxed_fista(grad_fn, np.zeros((4, 4)), gamma, 0.0, alpha, 300,
                                  lo=0.0, hi=0.6)
    fs = [np.zeros((4, 4))] + hist["f"]
    Fv = [grad_fn(x)[1] for x in fs]
    phi = [Fv[k] + (1 / (2 * gamma) - L) * np.sum((fs[k] - fs[k - 1]) ** 2) for k in range(1, len(fs))]
    assert np.all(np.diff(phi) <= 1e-12 * max(phi))


def test_alpha_one_has_fista_rate_and_alpha_zero_is_ista():
    """alpha = 1 is FISTA: F(f_k) - F* <= 2 L ||f_0 - f*||^2 / (k+1)^2 (Beck-Teboulle
    rate) on an ill-conditioned quadratic, which ISTA (alpha = 0) violates; and
    alpha = 0 iterates equal plain proximal-gradient (ISTA) iterates."""
    rng = np.random.default_rng(5)
    m = 25
    Q, _ = np.linalg.qr(rng.standard_normal((m, m)))
    eig = np.logspace(-4, 0, m)
    B = (Q * np.sqrt(eig)) @ Q.T
    fstar = Q @ np.ones(m)
    yv = B @ fstar
    L = eig.max()
    grad_fn = _quad(B, yv)
    bound = lambda k: 2 * L * np.sum(fstar ** 2) / (k + 1) ** 2
    K = 400
    _, h1 = fista.relaxed_fista(grad_fn, np.zeros((5, 5)), 1 / L, 0.0, 1.0, K, -np.inf, np.inf)
    gap1 = np.array([grad_fn(x)[1] for x in h1["f"]])
    assert np.all(gap1 <= np.array([bound(k) for k in range(1, K + 1)]) * (1 + 1e-9))
    _, h0 = fista.relaxed_fista(grad_fn, np.zeros((5, 5)), 1 / L, 0.0, 0.0, K, -np.inf, np.inf)
    gap0 = np.array([grad_fn(x)[1] for x in h0["f"]])
    assert np.any(gap0 > np.array([bound(k) for k in range(1, K + 1)]))
    x = np.zeros((5, 5))
    for k in range(K):
        x = x - (1 / L) * grad_fn(x)[0]
        if k in (0, 10, K - 1):
            assert np.allclose(x, h0["f"][k], rtol=0, atol=1e-13)


def test_gradient_mapping_rate_prop3():
    """eq. convergence_rate: min_k ||G_gamma(f_k)||^2 <= 2L(3+gamma L)^2 (F(f0)-F*) /
    (K gamma L (1 - gamma L)) on a linear model with TV and box."""
    prob, B, L = _linear_problem(h=1 / 8)
    ftrue = np.random.default_rng(6).uniform(0, 1, (4, 4))
    _, yv = _data(prob, ftrue)
    alpha, tau = 0.96, 1e-3
    gamma = (1 - alpha ** 2) / (2 * L)
    grad_fn = _quad(B, yv)
    K = 60
    _, hist = fista.relaxed_fista(grad_fn, np.zeros((4, 4)), gamma, tau, alpha, K, 0.0, 2.0, inner=400)
    Gm = [np.sum(fista.gradient_mapping(grad_fn, x, gamma, tau, 0.0, 2.0, 400) ** 2) for x in hist["f"]]
    F0 = fista.objective(grad_fn(np.zeros((4, 4)))[1], np.zeros((4, 4)), tau)
    assert min(Gm) <= fista.rate_bound(L, gamma, F0, 0.0, K)
    # without the regulariser the prox is the box projection, so the mapping
    # is grad D itself (no box) or (x - clip(x - gamma grad D)) / gamma
    x = hist["f"][5]
    gD = grad_fn(x)[0]
    assert np.allclose(fista.gradient_mapping(grad_fn, x, gamma, 0.0, -np.inf, np.inf), gD, rtol=1e-12, atol=0)
    ref = (x - np.clip(x - gamma * gD, 0.3, 0.6)) / gamma
    assert np.allclose(fista.gradient_mapping(grad_fn, x, gamma, 0.0, 0.3, 0.6), ref, rtol=1e-12, atol=1e-12)
    # the bound is the printed expression: doubling K halves it, F0 - F* scales it
    assert np.isclose(fista.rate_bound(L, gamma, F0, 0.0, 2 * K), 0.5 * fista.rate_bound(L, gamma, F0, 0.0, K))
    assert np.isclose(fista.rate_bound(L, gamma, 2 * F0, F0, K), fista.rate_bound(L, gamma, F0, 0.0, K))


def _proof_of_prop3_pieces(L, gamma):
    """The constants of the individual steps of the proof of Prop. 3, each
    collected from its own step (not from the printed final bound):

    * step (a)/(b) of the energy inequality: the ||s_{k+1} - f_{k+1}||^2
      terms are +L/2 (Young on the Lipschitz cross term) and -1/(2 gamma)
      (three-point identity), the ||f_{k+1} - f_k||^2 terms combine to
      -(1/(2 gamma) - L) once gamma <= (1 - alpha^2)/(2L) absorbs the
      momentum term;
    * eq. Gfs: ||G(f_k) - G(s_k)|| <= (1/gamma + 1/gamma + L) ||s_k - f_k||
      (triangle inequality, non-expansive prox, Lipschitz gradient);
    * G(s_k) = (s_k - f_k)/gamma, so ||G(f_k)|| <= (1 + gamma lip_G) ||G(s_k)||.
    """
    c_s = 1.0 / (2 * gamma) - L / 2.0          # coefficient of ||s_{k+1} - f_{k+1}||^2
    c_f = 1.0 / (2 * gamma) - L                # coefficient of the telescoping ||f_{k+1} - f_k||^2
    lip_G = 1.0 / gamma + 1.0 / gamma + L      # eq. Gfs
    ratio = 1.0 + gamma * lip_G                # ||G(f_k)|| / ||G(s_k)|| at most
    return c_s, c_f, lip_G, ratio


def _nonconvex_quad(B, y, mu):
    """D(x) = 1/2 ||B x - y||^2 - mu/2 ||x||^2: a smooth nonconvex term whose
    exact gradient Lipschitz constant is the largest |eigenvalue| of B^T B - mu I."""
    def grad_fn(s):
        x = s.reshape(-1)
        r = B @ x - y
        return (B.T @ r - mu * x).reshape(s.shape), 0.5 * float(r @ r) - 0.5 * mu * float(x @ x)
    ev = np.linalg.eigvalsh(B.T @ B - mu * np.eye(B.shape[1]))
    return grad_fn, float(np.abs(ev).max())


def _prop3_cases():
    prob, B, L = _linear_problem(h=1 / 8)
    _, yv = _data(prob, np.random.default_rng(6).uniform(0, 1, (4, 4)))
    yield "convex, box", _quad(B, yv), L, 0.0, (0.0, 0.6)
    yield "convex, TV + box", _quad(B, yv), L, 1e-3, (0.0, 2.0)
    mu = 0.5 * np.linalg.eigvalsh(B.T @ B)[-1]
    g, Lnc = _nonconvex_quad(B, yv, mu)
    yield "nonconvex, box", g, Lnc, 0.0, (0.0, 0.6)
    rng = np.random.default_rng(21)
    B2 = rng.standard_normal((30, 16))
    g2, L2 = _nonconvex_quad(B2, rng.standard_normal(30), 0.8 * np.linalg.eigvalsh(B2.T @ B2)[-1])
    yield "nonconvex random, TV + box", g2, L2, 5e-2, (-1.0, 1.0)


@pytest.mark.parametrize("alpha", [0.0, 0.5, 0.96])
def test_prop3_proof_steps_hold_on_iterates(alpha):
    """Each step of the proof of Prop. 3 holds on relaxed-FISTA iterates of
    convex and nonconvex linear models with exact L and gamma = (1-alpha^2)/(2L):
    the per-iteration energy inequality (b), its telescoped sum with F(f_K) in
    place of F*, the identity G(s_k) = (s_k - f_k)/gamma, and eq. Gfs."""
    for name, grad_fn, L, tau, (lo, hi) in _prop3_cases():
        gamma = (1 - alpha ** 2) / (2 * L)
        c_s, c_f, lip_G, ratio = _proof_of_prop3_pieces(L, gamma)
        inner = 3000 if tau > 0 else 1
        K = 40
        f0 = np.zeros((4, 4))
        _, hist = fista.relaxed_fista(grad_fn, f0, gamma, tau, alpha, K, lo, hi, inner=inner)
        fs = [f0, f0] + hist["f"]                          # f_{-1} = f_0, f_0, f_1 ... f_K
        ss = hist["s"]                                     # s_1 ... s_K
        Fv = [fista.objective(grad_fn(x)[1], x, tau) for x in fs]
        sq = lambda a: float(np.sum(a * a))
        slack = 1e-9 * (abs(Fv[1]) + 1.0)
        # (b): F(f_{k+1}) - F(f_k) <= c_f ||f_k - f_{k-1}||^2 - c_f ||f_{k+1} - f_k||^2 - c_s ||s_{k+1} - f_{k+1}||^2
        for k in range(0, K):
            lhs = Fv[k + 2] - Fv[k + 1]
            rhs = c_f * sq(fs[k + 1] - fs[k]) - c_f * sq(fs[k + 2] - fs[k + 1]) - c_s * sq(ss[k] - fs[k + 2])
            assert lhs <= rhs + slack, (name, alpha, k, lhs, rhs)
        # summed: c_s sum_k ||s_k - f_k||^2 <= F(f_0) - F(f_K) - c_f ||f_K - f_{K-1}||^2
        total = c_s * sum(sq(ss[k] - fs[k + 2]) for k in range(K))
        assert total <= Fv[1] - Fv[-1] - c_f * sq(fs[-1] - fs[-2]) + slack, name
        # G(s_k) = (s_k - f_k)/gamma and eq. Gfs on every iterate
        for k in (0, 1, 5, K - 1):
            s, f = ss[k], fs[k + 2]
            Gs = fista.gradient_mapping(grad_fn, s, gamma, tau, lo, hi, inner)
            Gf = fista.gradient_mapping(grad_fn, f, gamma, tau, lo, hi, inner)
            assert np.allclose(Gs, (s - f) / gamma, rtol=0, atol=1e-6 * (1 + np.abs(Gs).max())), (name, k)
            assert np.sqrt(sq(Gf - Gs)) <= lip_G * np.sqrt(sq(s - f)) * (1 + 1e-9) + 1e-9, (name, k)
            assert np.sqrt(sq(Gf)) <= ratio * np.sqrt(sq(Gs)) * (1 + 1e-9) + 1e-9, (name, k)


def test_rate_bound_assembled_from_the_proof_steps():
    """eq. convergence_rate is the chain of the proof: summing the energy
    inequality gives sum_k ||s_k - f_k||^2 <= (F_0 - F*)/c_s, i.e. eq.
    partial_sum for G(s_k) = (s_k - f_k)/gamma; eq. Gfs scales each term by
    ratio^2; the minimum is at most the mean over K.  The oracle's bound must
    equal that assembly for every (L, gamma, F_0 - F*, K) with gamma L < 1
    (so a changed constant or exponent anywhere in it fails)."""
    rng = np.random.default_rng(33)
    for _ in range(200):
        L = float(10 ** rng.uniform(-3, 3))
        gamma = float(rng.uniform(0.01, 0.99)) / L
        F0 = float(rng.uniform(0.1, 1e3))
        Fs = float(rng.uniform(-1e2, 0.09))
        K = int(rng.integers(1, 10000))
        c_s, _, _, ratio = _proof_of_prop3_pieces(L, gamma)
        partial_sum = (F0 - Fs) / c_s / gamma ** 2       # bound on sum_k ||G(s_k)||^2
        assembled = ratio ** 2 * partial_sum / K
        assert np.isclose(fista.rate_bound(L, gamma, F0, Fs, K), assembled, rtol=1e-11, atol=0), (L, gamma, K)


@pytest.mark.slow
def test_cisor_small_reconstruction_decreases_misfit():
    """CISOR on a small nonlinear problem: D decreases and SNR improves over f0 = 0."""
    n, T, M = 16, 4, 16
    prob = cisor.make_problem_2d(n, 1 / 8, T=T, M=M, rx_radius=n / 8)
    ftrue = disks_2d(n, 0, count=2, radius_px=(2, 4), eps_range=(1.1, 1.3))
    _, y = cisor.forward(prob, ftrue, tol=1e-12)
    gamma = 0.5 / stepsize.born_lipschitz(prob)
    f, hist = fista.cisor_reconstruct(prob, y, gamma, 1e-4, K=30, tol=1e-10)
    assert hist["D"][-1] < 0.2 * hist["D"][0]
    assert np.linalg.norm(f - ftrue) < 0.8 * np.linalg.norm(ftrue)


def test_momentum_sequence_properties():
    """t_1 = 1 makes the first momentum weight zero (s_2 = f_1); the sequence of
    eq. algo2 satisfies t_{k+1}^2 - t_{k+1} = t_k^2 and t_k >= (k+1)/2
    (Beck-Teboulle, Lemma 4.3), so the weights alpha (t_k-1)/t_{k+1} lie in [0, 1)."""
    rng = np.random.default_rng(9)
    B = rng.standard_normal((12, 9))
    yv = rng.standard_normal(12)
    grad_fn = _quad(B, yv)
    L = np.linalg.eigvalsh(B.T @ B)[-1]
    _, hist = fista.relaxed_fista(grad_fn, np.zeros((3, 3)), 1 / L, 0.0, 0.96, 30, -np.inf, np.inf)
    assert np.array_equal(hist["s"][1], hist["f"][0])
    t = [1.0] + hist["t"]
    for k in range(1, len(t)):
        assert abs(t[k] ** 2 - t[k] - t[k - 1] ** 2) < 1e-10 * t[k] ** 2
        assert t[k - 1] >= k / 2.0
    # realised weights (s_{k+1} - f_k) / (f_k - f_{k-1}) match alpha (t_k - 1)/t_{k+1}
    fs = [np.zeros((3, 3))] + hist["f"]
    for k in range(2, 12):
        d = fs[k] - fs[k - 1]
        w = np.sum((hist["s"][k] - fs[k]) * d) / np.sum(d * d)
        assert 0.0 <= w < 0.96


def test_fgp_dual_rate():
    """FGP is FISTA on the dual: after k iterations the dual suboptimality is at most
    2 (4 d lam^2) ||p*||^2 / (k+1)^2 (Beck-Teboulle rate with p_0 = 0)."""
    rng = np.random.default_rng(11)
    z = rng.uniform(0, 1, (24, 24))
    z[6:18, 6:18] += 1.0
    lam = 0.6
    _, pstar = tv.prox_tv_box(z, lam, 0.0, 1.5, iters=20000, return_dual=True)
    dstar = tv.dual_value(pstar, z, lam, 0.0, 1.5)
    Ld = 8.0 * lam ** 2
    for k in (5, 10, 20, 40, 80):
        _, p = tv.prox_tv_box(z, lam, 0.0, 1.5, iters=k, return_dual=True)
        gap = dstar - tv.dual_value(p, z, lam, 0.0, 1.5)
        assert gap <= 2 * Ld * np.sum(pstar ** 2) / (k + 1) ** 2 * (1 + 1e-9)


def test_rate_bound_is_the_oracle_expression():
    """The diagnostics module evaluates eq. convergence_rate as the oracle does."""
    from paper_1708_01663_amd.diagnostics import rate_bound
    for L, g, F0, Fs, K in ((3.0, 0.01, 5.0, 0.0, 40), (327.0, 1e-4, 2204.4, 100.0, 100)):
        assert np.isclose(rate_bound(L, g, F0, Fs, K), fista.rate_bound(L, g, F0, Fs, K), rtol=1e-14)
