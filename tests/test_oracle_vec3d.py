"""Pins of the oracle's 3D vectorial model (the paper's appendix on 3D imaging)."""

import numpy as np

from oracle import green, operators, vec3d
from oracle.geometry import cone_directions, plane_receivers
from synth import ellipsoids_3d


def _dense_operator(prob, f):
    """A = I - (k^2 I + D)(I_3 x G0 diag f) with D assembled from Kronecker
    products of 1D matrices: the three-point second difference and the central
    first difference (whose product along two axes is the four-corner stencil)."""
    n, h, k = prob.n, prob.h, prob.k
    N = n ** 3
    I1 = np.eye(n)
    D2 = (np.diag(-2 * np.ones(n)) + np.diag(np.ones(n - 1), 1) + np.diag(np.ones(n - 1), -1)) / h ** 2
    C = (np.diag(np.ones(n - 1), 1) - np.diag(np.ones(n - 1), -1)) / (2 * h)
    ops1 = [[None] * 3 for _ in range(3)]
    for i in range(3):
        for j in range(3):
            mats = [I1, I1, I1]
            if i == j:
                mats[i] = D2
            else:
                mats[i] = C
                mats[j] = C
            ops1[i][j] = np.kron(np.kron(mats[0], mats[1]), mats[2])
    Dm = np.block(ops1)
    G0 = green.dense_G(n, h, k, 3) / k ** 2
    GF = np.kron(np.eye(3), G0 * f.reshape(-1)[None, :])
    return np.eye(3 * N) - (k ** 2 * np.eye(3 * N) + Dm) @ GF


def _small(n=4, T=2, M=4):
    h = 0.15
    prob = vec3d.make_problem(n, h, cone_directions(T), plane_receivers(2, 0.6, -1.0)[:M])
    f = np.random.default_rng(1).uniform(0.1, 0.4, (n, n, n))
    return prob, f


def test_operator_matches_the_dense_kronecker_construction():
    prob, f = _small()
    A = _dense_operator(prob, f)
    E = np.random.default_rng(2).standard_normal((3,) + f.shape) + 1j * np.random.default_rng(3).standard_normal(
        (3,) + f.shape)
    assert np.allclose(vec3d.apply_A(prob, f, E).reshape(-1), A @ E.reshape(-1), rtol=0, atol=1e-10)
    assert np.allclose(vec3d.apply_AH(prob, f, E).reshape(-1), np.conj(A).T @ E.reshape(-1), rtol=0, atol=1e-10)
    # and the solve inverts it
    u, _ = vec3d.solve(prob, f, prob.E_in, tol=1e-13)
    assert np.allclose(A @ u[0].reshape(-1), prob.E_in[0].reshape(-1), rtol=0, atol=1e-9)


def test_dyadic_green_row_matches_finite_differences_of_g():
    """eq. dyadicGreen: (k^2 I + grad grad) g, third row, against a numerical Hessian."""
    k = 2 * np.pi
    R = np.array([0.7, -0.4, 1.1])
    g = lambda r: np.exp(1j * k * np.linalg.norm(r)) / (4 * np.pi * np.linalg.norm(r))
    e = 1e-4
    row = np.zeros(3, dtype=complex)
    for j in range(3):
        ej, e3 = np.eye(3)[j] * e, np.eye(3)[2] * e
        row[j] = (g(R + e3 + ej) - g(R + e3 - ej) - g(R - e3 + ej) + g(R - e3 - ej)) / (4 * e * e)
    row[2] += k ** 2 * g(R)
    assert np.allclose(vec3d.dyadic_row3(R[None], k)[0], row, rtol=1e-6)


def test_scalar_limit_without_grad_div():
    """Without D, each component obeys the scalar equation (k^2 G0 is the
    scalar model's cell-integrated kernel)."""
    prob, f = _small()
    e = np.random.default_rng(4).standard_normal(f.shape) + 0j
    E = np.stack([e, np.zeros_like(e), np.zeros_like(e)])
    out = vec3d.apply_A(prob, f, E, graddiv=False)
    Ghat = green.kernel_spectrum(prob.n, prob.h, prob.k, 3)
    assert np.allclose(out[0], operators.apply_A(Ghat, f, e), rtol=0, atol=1e-12)
    assert np.all(out[1:] == 0)


def test_incident_polarisation_is_transverse_and_unit():
    dirs = np.vstack([cone_directions(5), [[0.0, 0.0, -1.0]]])
    p = vec3d.polarisations(dirs)
    assert np.allclose(np.sum(p * dirs, axis=1), 0, atol=1e-14)
    assert np.allclose(np.linalg.norm(p, axis=1), 1)


def test_first_born_limit():
    prob, f = _small(n=5)
    f = ellipsoids_3d(5, 2, eps_range=(1.1, 1.3))
    yB = lambda s: vec3d.project(prob, s * f, prob.E_in)
    dev = []
    for s in (0.02, 0.01):
        _, y = vec3d.forward(prob, s * f, tol=1e-13)
        dev.append(np.linalg.norm(y - yB(s)) / np.linalg.norm(yB(s)))
    assert 1.8 < dev[0] / dev[1] < 2.2


def test_gradient_matches_central_differences():
    prob, f = _small()
    y_meas = 0.01 * (np.random.default_rng(5).standard_normal((prob.T, prob.Ht.shape[0])) * (1 + 1j))
    g, D = vec3d.gradient(prob, f, y_meas, tol=1e-13)
    d = np.random.default_rng(6).standard_normal(f.shape)
    eps = 1e-5
    fd = (vec3d.misfit(prob, f + eps * d, y_meas, 1e-13) - vec3d.misfit(prob, f - eps * d, y_meas, 1e-13)) / (2 * eps)
    assert abs(np.sum(g * d) - fd) < 1e-6 * abs(fd)


def test_masked_gradient_matches_central_differences_and_ignores_inactive_receivers():
    prob, f = _small(M=6)
    T, M = prob.T, prob.Ht.shape[0]
    mask = np.ones((T, M))
    mask[0, :2] = 0
    mask[1, 3:] = 0
    prob.mask = mask
    y_meas = 0.01 * (np.random.default_rng(7).standard_normal((T, M)) * (1 - 1j))
    g, D = vec3d.gradient(prob, f, y_meas, tol=1e-13)
    d = np.random.default_rng(8).standard_normal(f.shape)
    eps = 1e-5
    fd = (vec3d.misfit(prob, f + eps * d, y_meas, 1e-13) - vec3d.misfit(prob, f - eps * d, y_meas, 1e-13)) / (2 * eps)
    assert abs(np.sum(g * d) - fd) < 1e-6 * abs(fd)
    # D is the sum over the active receivers only
    _, y = vec3d.forward(prob, f, tol=1e-13)
    assert np.isclose(D, 0.5 * sum(abs(y[t, m] - y_meas[t, m]) ** 2 for t in range(T) for m in range(M) if mask[t, m]),
                      rtol=1e-12)
    g2, D2 = vec3d.gradient(prob, f, y_meas + (1 - mask) * 3.0, tol=1e-13)
    assert D2 == D and np.array_equal(g2, g)


def test_first_reconstruction_step_in_closed_form():
    """From f = 0: E = E_in, y = 0, w = -y_meas, V = 0, so grad D(0) =
    Re sum_t sum_j conj(E_in) Ht^H(-y_meas) and f_1 = prox(-gamma grad D(0))."""
    from oracle import tv
    prob, _ = _small(n=6, T=3, M=4)
    y_meas = 0.05 * (np.random.default_rng(12).standard_normal((3, 4)) + 1j)
    gamma, tau = 2.0, 1e-2
    f1, hist = vec3d.reconstruct(prob, y_meas, gamma, tau, K=1, tol=1e-13)
    q = (np.conj(prob.Ht).T @ (-y_meas).T).T.reshape(3, 3, 6, 6, 6)
    g0 = np.real(np.sum(np.conj(prob.E_in) * q, axis=(0, 1)))
    assert np.isclose(hist["D"][0], 0.5 * np.sum(np.abs(y_meas) ** 2), rtol=1e-14)
    ref = tv.prox_tv_box(-gamma * g0, gamma * tau, 0.0, 2.0, 100)
    assert np.allclose(f1, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    assert np.abs(ref).max() > 0 and tv.tv_value(ref) > 0
    # later steps lower the misfit on data made by the model itself
    ftrue = np.zeros((6, 6, 6))
    ftrue[2:4, 2:5, 1:4] = 0.3
    _, y = vec3d.forward(prob, ftrue, tol=1e-13)
    _, hist = vec3d.reconstruct(prob, y, 0.5, 1e-4, K=6, tol=1e-12)
    assert hist["D"][-1] < 0.95 * hist["D"][0]


def test_dyadic_matches_finite_differences_and_its_third_row():
    k = 2 * np.pi
    R = np.array([-0.5, 0.9, 0.6])
    g = lambda r: np.exp(1j * k * np.linalg.norm(r)) / (4 * np.pi * np.linalg.norm(r))
    e = 1e-4
    Gfd = np.zeros((3, 3), dtype=complex)
    for i in range(3):
        for j in range(3):
            ei, ej = np.eye(3)[i] * e, np.eye(3)[j] * e
            Gfd[i, j] = (g(R + ei + ej) - g(R + ei - ej) - g(R - ei + ej) + g(R - ei - ej)) / (4 * e * e)
    Gfd += k ** 2 * g(R) * np.eye(3)
    G = vec3d.dyadic(R[None], k)[0]
    assert np.allclose(G, Gfd, rtol=1e-6)
    assert np.allclose(G, G.T)
    assert np.allclose(vec3d.dyadic_row3(R[None], k)[0], G[2], rtol=1e-14)


def test_far_dipole_is_a_transverse_plane_wave():
    """A dipole far away illuminates the grid with the plane wave travelling from
    it, polarised along the transverse part of its moment, times g(|s|)."""
    from oracle import geometry
    n, h, k = 6, 0.2, 2 * np.pi
    src = np.array([[0.3e6, -0.4e6, 1.2e6]])
    d = -src[0] / np.linalg.norm(src[0])
    p = vec3d.polarisations(d[None])[0]
    E = vec3d.dipole_fields(n, h, k, src, p[None])[0]
    pw = geometry.plane_waves(n, h, k, d[None])[0]
    R = np.linalg.norm(src[0])
    g = np.exp(1j * k * R) / (4 * np.pi * R)
    ratio = E / (g * pw)[None]
    assert np.allclose(ratio, p[:, None, None, None], rtol=0, atol=1e-5)


def test_dipole_field_is_divergence_free():
    """div E_in = 0 away from the source (the field solves the source-free
    vector Helmholtz equation there): central differences on a fine grid."""
    k = 2 * np.pi
    s = np.array([[1.3, -0.7, 0.9]])
    p = np.array([[0.0, 0.6, 0.8]])
    n, h = 9, 0.01
    E = vec3d.dipole_fields(n, h, k, s, p)[0]
    c = n // 2
    div = ((E[0, c + 1, c, c] - E[0, c - 1, c, c]) + (E[1, c, c + 1, c] - E[1, c, c - 1, c])
           + (E[2, c, c, c + 1] - E[2, c, c, c - 1])) / (2 * h)
    grad_mag = np.abs(E[0, c + 1, c, c] - E[0, c - 1, c, c]) / (2 * h)
    assert abs(div) < 1e-3 * grad_mag


def test_dipole_problem_solves_and_reduces_to_plane_waves_far_away():
    prob_far = vec3d.make_problem(4, 0.15, None, plane_receivers(2, 0.6, -1.0), src=np.array([[0.0, 0.0, 3e5]]))
    prob_pw = vec3d.make_problem(4, 0.15, np.array([[0.0, 0.0, -1.0]]), plane_receivers(2, 0.6, -1.0))
    R = 3e5
    g = np.exp(1j * 2 * np.pi * R) / (4 * np.pi * R)
    assert np.allclose(prob_far.E_in / g, prob_pw.E_in, rtol=0, atol=1e-4)
