"""Pins of the oracle's point-source transmitters, free receiver positions and
per-transmitter receiver masks (the geometry of the paper's experiments)."""

import numpy as np

from oracle import cisor as ocisor
from oracle import geometry, green, operators
from synth import disks_2d


def test_far_point_source_is_a_plane_wave():
    """A unit line source far away illuminates the grid with the plane wave
    travelling from it towards the origin (large-argument form of H0), up to a
    constant factor."""
    n, h, k = 16, 0.125, 2 * np.pi
    R = 1e6
    th = 0.7
    src = np.array([[-R * np.cos(th), -R * np.sin(th)]])
    u = geometry.point_sources(n, h, k, src)[0]
    pw = geometry.plane_waves(n, h, k, np.array([[np.cos(th), np.sin(th)]]))[0]
    ratio = u / pw
    assert np.std(ratio) / np.abs(np.mean(ratio)) < 1e-4
    # the constant is the Hankel asymptote (i/4) sqrt(2/(pi k R)) exp(i(k R - pi/4))
    const = 0.25j * np.sqrt(2 / (np.pi * k * R)) * np.exp(1j * (k * R - np.pi / 4))
    assert abs(np.mean(ratio) / const - 1) < 1e-4


def test_point_source_3d_is_the_free_space_green_function():
    n, h, k = 6, 0.2, 2 * np.pi
    src = np.array([[2.0, -1.0, 0.5]])
    u = geometry.point_sources(n, h, k, src)[0].reshape(-1)
    r = geometry.pixel_positions_3d(n, h)
    d = np.linalg.norm(r - src[0], axis=1)
    assert np.allclose(u, np.exp(1j * k * d) / (4 * np.pi * d), rtol=1e-14, atol=0)


def test_source_receiver_reciprocity():
    """diag(f)(I - G diag f)^{-1} is symmetric, so the scattered field at B
    from a source at A equals the field at A from a source at B (with the
    receiver kernel proportional to the source field)."""
    n, h = 14, 1 / 8
    A, B = np.array([1.7, -0.4]), np.array([-0.9, 1.6])
    pts = np.stack([A, B])
    prob = ocisor.make_problem_2d(n, h, 2, 2, 0.0, tx_pos=pts, rx=pts)
    f = disks_2d(n, 5, count=2, radius_px=(2, 4), eps_range=(1.2, 1.8))
    u, y = ocisor.forward(prob, f, tol=1e-13)
    assert abs(y[0, 1] - y[1, 0]) < 1e-10 * abs(y[0, 1])
    # and the fields solve the discrete equation with the point-source right-hand side
    for t in range(2):
        r = prob.u_in[t] - operators.apply_A(prob.Ghat, f, u[t])
        assert np.linalg.norm(r) < 1e-12 * np.linalg.norm(prob.u_in[t])


def test_masked_gradient_matches_the_dense_jacobian():
    """With receivers switched off per transmitter, D and its Prop. 1 gradient
    equal the brute-force Jacobian result over the active receivers only."""
    n, h, T, M = 10, 1 / 8, 3, 12
    rx = geometry.ring_receivers(M, 2.0)
    tx = geometry.ring_receivers(T, 2.5) + 0.01
    mask = np.ones((T, M))
    mask[0, :4] = 0
    mask[1, 5:9] = 0
    mask[2, ::2] = 0
    prob = ocisor.make_problem_2d(n, h, T, M, 0.0, tx_pos=tx, rx=rx, mask=mask)
    f = disks_2d(n, 1, count=2, radius_px=(2, 3), eps_range=(1.1, 1.4))
    y_meas = np.random.default_rng(3).standard_normal((T, M)) * (1 + 1j) * 0.05
    g, D = ocisor.gradient(prob, f, y_meas, tol=1e-13)
    Gd = green.dense_G(n, h, prob.k, 2)
    g_ref, D_ref = ocisor.gradient_dense(prob, f, y_meas, Gd)
    assert abs(D - D_ref) < 1e-10 * D_ref
    assert np.linalg.norm(g - g_ref) < 1e-8 * np.linalg.norm(g_ref)
    # switched-off receivers carry no data: changing their measurements changes nothing
    y2 = y_meas + (1 - mask) * 7.0
    g2, D2 = ocisor.gradient(prob, f, y2, tol=1e-13)
    assert D2 == D and np.array_equal(g2, g)
    # an all-ones mask is the unmasked problem
    prob1 = ocisor.make_problem_2d(n, h, T, M, 0.0, tx_pos=tx, rx=rx, mask=np.ones((T, M)))
    prob0 = ocisor.make_problem_2d(n, h, T, M, 0.0, tx_pos=tx, rx=rx)
    assert np.allclose(ocisor.gradient(prob1, f, y_meas, tol=1e-13)[0], ocisor.gradient(prob0, f, y_meas, tol=1e-13)[0],
                       rtol=1e-12, atol=0)


def test_paper_style_linear_arrays_and_line_sources():
    """Two detector arrays of 169 sensors 3.84 apart at x = +-95.9 and sources on
    the line 48 further left at azimuths -60..60 every 5 degrees (lengths in cm)."""
    rx = geometry.linear_arrays(169, 3.84, 95.9)
    assert rx.shape == (338, 2)
    assert np.allclose(np.diff(rx[:169, 1]), 3.84) and np.allclose(rx[:169, 0], -95.9)
    assert np.allclose(rx[169:, 0], 95.9) and abs(rx[:169, 1].mean()) < 1e-12
    tx = geometry.line_sources(95.9 + 48.0)
    assert tx.shape == (25, 2) and np.allclose(tx[:, 0], -143.9)
    az = np.degrees(np.arctan2(tx[:, 1], -tx[:, 0]))
    assert np.allclose(az, np.arange(-60, 61, 5))


def test_synthetic_paper_geometries():
    """The benchmark's paper geometries (positions only, in wavelengths) are the
    ones the oracle's helpers build from the published lengths."""
    from synth import fresnel_like_geometry, paper_sim_geometry
    lam = 7.49
    n, h, tx, rx = paper_sim_geometry()
    assert n == 128 and np.isclose(n * h, 120.0 / lam)
    assert np.allclose(rx, geometry.linear_arrays(169, 3.84 / lam, 95.9 / lam))
    assert np.allclose(tx, geometry.line_sources((95.9 + 48.0) / lam))
    n, h, tx, rx, mask = fresnel_like_geometry()
    assert np.allclose(rx, geometry.ring_receivers(360, 1670.0 / 99.9))
    assert np.allclose(tx, geometry.ring_receivers(8, 1670.0 / 99.9))
    assert np.all(mask.sum(1) == 241)
    for t in range(8):     # the switched-off receivers are the 119 nearest to the source
        d = np.linalg.norm(rx - tx[t], axis=1)
        assert d[mask[t] == 0].max() <= d[mask[t] == 1].min() + 1e-12


def test_synthetic_3d_experimental_layout():
    """81 transmitters (9 azimuths x 9 polar angles on a sphere), 36 receivers
    on the azimuthal circle of the same radius, a receiver active when more
    than 50 degrees from the transmitter; two touching spheres."""
    from synth import fresnel3d_like_geometry, two_spheres_3d
    n, h, dirs, rx, mask = fresnel3d_like_geometry()
    assert n == 32 and np.isclose(h, 4.7 / 74.9)
    assert dirs.shape == (81, 3) and np.allclose(np.linalg.norm(dirs, axis=1), 1)
    assert rx.shape == (36, 3) and np.allclose(rx[:, 2], 0) and np.allclose(np.linalg.norm(rx, axis=1), 1769 / 74.9)
    # a transmitter on the equator at azimuth 20 degrees: receivers at -30..70 degrees are within 50
    pol = np.degrees(np.arccos(-dirs[:, 2]))
    az = np.degrees(np.arctan2(-dirs[:, 1], -dirs[:, 0])) % 360
    t = int(np.flatnonzero(np.isclose(pol, 90) & np.isclose(az, 20))[0])
    off = np.flatnonzero(mask[t] == 0)
    assert sorted((10 * off).tolist()) == [0, 10, 20, 30, 40, 50, 60, 70, 330, 340, 350]
    # a transmitter at polar angle 30 is at least 60 degrees from every receiver
    t30 = np.flatnonzero(np.isclose(pol, 30))
    assert np.all(mask[t30] == 1)
    f = two_spheres_3d(32, h)
    assert set(np.unique(f)) == {0.0, 1.6}
    assert np.array_equal(f, f[::-1])        # symmetric about x = 0
    r_px = 25.0 / 4.7
    vol = f.astype(bool).sum()
    assert abs(vol - 2 * 4 / 3 * np.pi * r_px ** 3) < 0.1 * vol
