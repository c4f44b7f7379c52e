"""Pins of the oracle's physics: Green's-function cells, operators, solves.

Each test checks the oracle against something other than itself: numerical
quadrature, brute-force dense linear algebra, a closed-form scattering
solution, or an exact invariant.
"""

import numpy as np
import pytest
from scipy import integrate, special

from analytic import cylinder_scattered_field
from oracle import cisor, green, krylov, operators
from synth import disk_area_fraction, disks_2d, ellipsoids_3d, random_field

K = 2 * np.pi


def _cquad2(fn, a0, a1, b0, b1):
    re = integrate.dblquad(lambda y, x: fn(x, y).real, a0, a1, b0, b1, epsabs=1e-13, epsrel=1e-11)[0]
    im = integrate.dblquad(lambda y, x: fn(x, y).imag, a0, a1, b0, b1, epsabs=1e-13, epsrel=1e-11)[0]
    return re + 1j * im


@pytest.mark.parametrize("h", [1 / 8, 1 / 10])
def test_kernel_2d_matches_quadrature(h):
    """eq. scalarGreens (2D, outgoing +i/4 reading): cell integral of k^2 g over the
    equal-area disk, self and off-diagonal, equals the closed form."""
    a = green.cell_radius(h, 2)
    # self term: k^2 (i/4) 2 pi int_0^a H0(k r) r dr
    re = integrate.quad(lambda r: (special.hankel1(0, K * r) * r).real, 0, a, limit=200, epsabs=1e-15)[0]
    im = integrate.quad(lambda r: (special.hankel1(0, K * r) * r).imag, 0, a, limit=200, epsabs=1e-15)[0]
    self_q = K ** 2 * 0.25j * 2 * np.pi * (re + 1j * im)
    assert abs(green.kernel(np.array([0.0]), K, h, 2)[0] - self_q) < 1e-8 * abs(self_q)
    # off-diagonal at distance rho: polar integral over the source disk
    for rho in (h, 3.7 * h):
        fn = lambda r, ph: special.hankel1(0, K * np.sqrt(rho ** 2 + r ** 2 - 2 * rho * r * np.cos(ph))) * r
        val = K ** 2 * 0.25j * _cquad2(fn, 0, a, 0, 2 * np.pi)
        ker = green.kernel(np.array([rho]), K, h, 2)[0]
        assert abs(ker - val) < 1e-8 * abs(val)


def test_kernel_3d_matches_quadrature():
    """eq. scalarGreens (3D): k^2 int_ball exp(ikr)/(4 pi r) over the equal-volume ball."""
    h = 1 / 6
    a = green.cell_radius(h, 3)
    re = integrate.quad(lambda r: (r * np.exp(1j * K * r)).real, 0, a)[0]
    im = integrate.quad(lambda r: (r * np.exp(1j * K * r)).imag, 0, a)[0]
    self_q = K ** 2 * (re + 1j * im)           # 4 pi r^2 / (4 pi r) = r
    assert abs(green.kernel(np.array([0.0]), K, h, 3)[0] - self_q) < 1e-10 * abs(self_q)
    d = 2.3 * h

    def fn(r, th):
        dist = np.sqrt(d * d + r * r - 2 * d * r * np.cos(th))
        return np.exp(1j * K * dist) / (4 * np.pi * dist) * r * r * np.sin(th) * 2 * np.pi

    val = K ** 2 * _cquad2(fn, 0, a, 0, np.pi)
    ker = green.kernel(np.array([d]), K, h, 3)[0]
    assert abs(ker - val) < 1e-8 * abs(val)


def test_padded_kernel_even_and_spectrum_even():
    """FFT embedding of G: the padded kernel and its spectrum are even per axis,
    so G is complex symmetric and G^H is the convolution with conj(Ghat)."""
    n, h = 8, 1 / 8
    Kc = green.padded_kernel(n, h, K, 2)
    P = 2 * n
    idx = (-np.arange(P)) % P
    assert np.allclose(Kc, Kc[idx][:, idx], atol=0)
    Gh = green.kernel_spectrum(n, h, K, 2)
    assert np.allclose(Gh, Gh[idx][:, idx], rtol=1e-12, atol=1e-12)
    Gd = green.dense_G(n, h, K, 2)
    assert np.allclose(Gd, Gd.T, rtol=0, atol=0)


@pytest.mark.parametrize("n", [7, 12, 20])
def test_fft_operator_matches_dense(n):
    """eq. A_def: FFT matvec A x = x - G(f x) and A^H equal the brute-force dense
    matrices I - G diag(f) and its conjugate transpose."""
    h = 1 / 8
    prob = cisor.make_problem_2d(n, h, T=1, M=4, rx_radius=n * h)
    f = disks_2d(n, 1, count=2, radius_px=(1.5, 3.0), eps_range=(1.2, 1.6))
    A = np.eye(n * n) - green.dense_G(n, h, K, 2) * f.reshape(1, -1)
    x = random_field((n, n), 5)
    assert np.allclose(operators.apply_A(prob.Ghat, f, x).ravel(), A @ x.ravel(), rtol=0, atol=1e-12)
    assert np.allclose(operators.apply_AH(prob.Ghat, f, x).ravel(), A.conj().T @ x.ravel(),
                       rtol=0, atol=1e-12)


def _square_symmetry(x, g):
    """g-th symmetry of the square grid (g % 4 quarter turns, then a transpose
    when g >= 4) on the last two axes."""
    y = np.rot90(x, g % 4, axes=(-2, -1))
    return np.swapaxes(y, -2, -1) if g >= 4 else y


@pytest.mark.parametrize("n", [9, 16])
def test_operator_commutes_with_the_symmetries_of_the_grid(n):
    """eq. A_def on the centred square grid: the cell-integrated kernel depends on
    the distance only, so A(g f) (g x) = g (A(f) x) for the eight symmetries g of
    the grid (the invariant behind the warm-start training's augmentation: a
    solution pair maps to a solution pair of the mapped problem)."""
    h = 1 / 8
    prob = cisor.make_problem_2d(n, h, T=1, M=4, rx_radius=n * h)
    f = disks_2d(n, 7, count=3, radius_px=(1.0, 3.0), eps_range=(1.1, 1.8))
    x = random_field((n, n), 9)
    ax = operators.apply_A(prob.Ghat, f, x)
    for g in range(8):
        lhs = operators.apply_A(prob.Ghat, _square_symmetry(f, g), _square_symmetry(x, g))
        assert np.allclose(lhs, _square_symmetry(ax, g), rtol=0, atol=1e-12), g
    # and it is not a trivial statement: a shift of the contrast breaks it
    lhs = operators.apply_A(prob.Ghat, np.roll(f, 1, axis=0), x)
    assert not np.allclose(lhs, ax, atol=1e-6)


def test_training_symmetry_matches_the_grid_symmetry():
    """The training code's map of flattened fields equals the grid symmetry above."""
    torch = pytest.importorskip("torch")
    from paper_1708_01663_amd.warmstart import dihedral
    n = 6
    x = random_field((3, n, n), 4)
    for g in range(8):
        got = dihedral(torch.tensor(x.reshape(3, n * n)), n, g).numpy().reshape(3, n, n)
        assert np.array_equal(got, _square_symmetry(x, g)), g


def test_fft_operator_matches_dense_3d():
    n, h = 5, 1 / 6
    Gh = green.kernel_spectrum(n, h, K, 3)
    f = ellipsoids_3d(n, 2, axes=(0.4, 0.8))
    A = np.eye(n ** 3) - green.dense_G(n, h, K, 3) * f.reshape(1, -1)
    x = random_field((n, n, n), 3)
    assert np.allclose(operators.apply_A(Gh, f, x).ravel(), A @ x.ravel(), atol=1e-12)
    assert np.allclose(operators.apply_AH(Gh, f, x).ravel(), A.conj().T @ x.ravel(), atol=1e-12)


def test_dot_test_adjoint():
    """<A x, y> = <x, A^H y> in FP64."""
    n, h = 16, 1 / 10
    Gh = green.kernel_spectrum(n, h, K, 2)
    f = disks_2d(n, 4, count=3, radius_px=(2, 4), eps_range=(1.0, 2.0))
    x, y = random_field((n, n), 1), random_field((n, n), 2)
    lhs = np.vdot(y, operators.apply_A(Gh, f, x))
    rhs = np.vdot(operators.apply_AH(Gh, f, y), x)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


@pytest.mark.parametrize("n", [8, 16, 24])
def test_bicgstab_matches_dense_solve(n):
    """eq. u_and_v: the FFT-BiCGSTAB forward and adjoint solves equal the dense
    direct solves of A u = u_in and A^H v = b (brute force)."""
    h = 1 / 8
    prob = cisor.make_problem_2d(n, h, T=3, M=8, rx_radius=n * h)
    f = disks_2d(n, n, count=3, radius_px=(2, 4), eps_range=(1.1, 1.5))
    A = np.eye(n * n) - green.dense_G(n, h, K, 2) * f.reshape(1, -1)
    u, _ = cisor.solve_fields(prob, f, tol=1e-12)
    ud = np.linalg.solve(A, prob.u_in.reshape(3, -1).T).T
    assert np.linalg.norm(u.reshape(3, -1) - ud) < 1e-10 * np.linalg.norm(ud)
    b = random_field((3, n, n), 9)
    v, _ = cisor.solve_fields(prob, f, rhs=b, tol=1e-12, adjoint=True)
    vd = np.linalg.solve(A.conj().T, b.reshape(3, -1).T).T
    assert np.linalg.norm(v.reshape(3, -1) - vd) < 1e-10 * np.linalg.norm(vd)


def test_bicgstab_true_residual_meets_tol():
    n, h = 32, 1 / 10
    prob = cisor.make_problem_2d(n, h, T=2, M=8, rx_radius=n * h)
    f = disks_2d(n, 3, count=4, radius_px=(3, 7), eps_range=(1.5, 2.0))
    for t in range(2):
        x, it, rel = krylov.bicgstab(lambda z: operators.apply_A(prob.Ghat, f, z), prob.u_in[t], tol=1e-9)
        r = prob.u_in[t] - operators.apply_A(prob.Ghat, f, x)
        assert np.linalg.norm(r) / np.linalg.norm(prob.u_in[t]) <= 1e-9
        assert it > 0


def test_cylinder_bessel_series_convergence():
    """LS solve + kernel + sign + H, end to end: receiver data for a homogeneous
    cylinder (area-fraction contrast) converge to the Bessel-series solution at
    second order.  The printed -i/4 sign fails this by O(1)."""
    R, eps = 0.9, 1.5
    errs = []
    for h in (1 / 16, 1 / 32):
        n = int(np.ceil(2 * R / h)) + 2
        prob = cisor.make_problem_2d(n, h, T=2, M=24, rx_radius=2.7)
        f = (eps - 1) * disk_area_fraction(n, h, R)
        _, y = cisor.forward(prob, f, tol=1e-10)
        e = 0.0
        for t in range(2):
            ref = cylinder_scattered_field(K, eps, R, np.pi * t, prob.meta["rx"])
            e = max(e, np.linalg.norm(y[t] - ref) / np.linalg.norm(ref))
        errs.append(e)
    assert errs[0] < 2e-2
    assert errs[0] / errs[1] > 3.0
    # wrong (incoming) sign: conjugating the kernel gives an O(1) error
    h = 1 / 16
    n = int(np.ceil(2 * R / h)) + 2
    prob = cisor.make_problem_2d(n, h, T=1, M=24, rx_radius=2.7)
    prob.Ghat = np.fft.fftn(np.conj(green.padded_kernel(n, h, K, 2)))
    prob.H = np.conj(prob.H)
    f = (eps - 1) * disk_area_fraction(n, h, R)
    _, y = cisor.forward(prob, f, tol=1e-10)
    ref = cylinder_scattered_field(K, eps, R, 0.0, prob.meta["rx"])
    assert np.linalg.norm(y[0] - ref) / np.linalg.norm(ref) > 0.3


def test_sphere_mie_series_convergence_3d():
    """3D forward model end to end (ball cell integrals, 3D FFT embedding, solve,
    receiver matrix): receiver data for a homogeneous sphere (volume-fraction
    contrast) converge to the scalar Mie series at second order."""
    from analytic import ball_volume_fraction, sphere_scattered_field
    R, eps = 0.6, 1.3
    dirs = np.array([[0, 0, 1.0], [np.sin(1.0), 0, np.cos(1.0)]])
    ph = np.linspace(0, 2 * np.pi, 12, endpoint=False)
    rx = np.stack([2.0 * np.cos(ph), 2.0 * np.sin(ph), 0.3 * np.ones(12)], 1)
    errs = []
    for h in (1 / 10, 1 / 20):
        n = int(np.ceil(2 * R / h)) + 2
        prob = cisor.make_problem_3d(n, h, dirs, rx)
        f = (eps - 1) * ball_volume_fraction(n, h, R)
        _, y = cisor.forward(prob, f, tol=1e-10)
        errs.append(max(np.linalg.norm(y[t] - sphere_scattered_field(K, eps, R, dirs[t], rx))
                        / np.linalg.norm(sphere_scattered_field(K, eps, R, dirs[t], rx)) for t in range(2)))
    assert errs[1] < 2e-2
    assert errs[0] / errs[1] > 3.0


def test_first_born_limit():
    """Linear method (u = u_in) is the small-contrast limit: the deviation of the
    nonlinear data from the Born data scales as O(c) relative, ratio -> 2."""
    n, h = 24, 1 / 10
    prob = cisor.make_problem_2d(n, h, T=3, M=16, rx_radius=n * h)
    f = disks_2d(n, 7, count=3, radius_px=(2, 5), eps_range=(1.5, 2.0))
    dev = []
    for c in (1e-3, 5e-4):
        _, y = cisor.forward(prob, c * f, tol=1e-13)
        yb = cisor.project(prob, c * f, prob.u_in)
        dev.append(np.linalg.norm(y - yb) / np.linalg.norm(yb))
    assert dev[0] < 1e-2
    assert 1.8 <= dev[0] / dev[1] <= 2.2


def test_reciprocity():
    """G = G^T makes F A^{-1} symmetric: the field at receiver m due to plane wave t
    equals u_in,t^T F A^{-1} h_m with the receiver row as incident field."""
    n, h = 20, 1 / 10
    prob = cisor.make_problem_2d(n, h, T=4, M=6, rx_radius=n * h)
    f = disks_2d(n, 11, count=3, radius_px=(2, 5), eps_range=(1.2, 1.8))
    tol = 1e-12
    u, y = cisor.forward(prob, f, tol=tol)
    hm = prob.H.reshape(prob.M, n, n)
    uh, _ = cisor.solve_fields(prob, f, rhs=hm, tol=tol)
    for t in range(prob.T):
        for m in range(prob.M):
            rhs = np.sum(prob.u_in[t] * f * uh[m])
            assert abs(y[t, m] - rhs) <= 1e-9 * np.abs(y).max()
