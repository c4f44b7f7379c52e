"""The synthetic workloads reproduce the experimental layouts the paper prints
(tests/golden/experimental_layouts.json, each value with its passage): the
simulated-data line of sources and two linear arrays, the 2D ring with the
nearest receivers off, and the 3D sphere of transmitters with the azimuthal
ring of receivers.  Lengths of the workloads are in wavelengths."""

import json
import os

import numpy as np

from synth import fresnel3d_like_geometry, fresnel3d_like_sources, fresnel_like_geometry, paper_sim_geometry

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "experimental_layouts.json")))


def _v(section, key):
    return GOLD[section][key]["value"]


def test_simulated_data_layout():
    lam = _v("simulated", "wavelength_cm")
    n, h, tx, rx = paper_sim_geometry()
    assert n == _v("simulated", "image_pixels")
    assert np.isclose(n * h * lam, _v("simulated", "image_side_cm"))
    m = _v("simulated", "sensors_per_detector")
    assert rx.shape[0] == 2 * m
    d = _v("simulated", "detector_distance_cm") / lam
    assert np.allclose(np.abs(rx[:, 0]), d)
    assert np.allclose(np.diff(rx[:m, 1]) * lam, _v("simulated", "sensor_spacing_cm"))
    assert np.allclose(tx[:, 0] * lam, -(_v("simulated", "detector_distance_cm") + _v("simulated", "source_line_offset_cm")))
    lo, hi, step = _v("simulated", "source_azimuth_deg")
    az = np.degrees(np.arctan2(tx[:, 1], -tx[:, 0]))
    assert np.allclose(az, np.arange(lo, hi + step / 2, step))


def test_experimental_2d_layout():
    lam = _v("experimental_2d", "wavelength_mm")
    n, h, tx, rx, mask = fresnel_like_geometry()
    assert tx.shape[0] == _v("experimental_2d", "transmitters") and rx.shape[0] == _v("experimental_2d", "receivers")
    R = _v("experimental_2d", "circle_radius_m") * 1000 / lam
    assert np.allclose(np.linalg.norm(tx, axis=1), R) and np.allclose(np.linalg.norm(rx, axis=1), R)
    assert np.all(mask.sum(1) == _v("experimental_2d", "active_receivers_per_transmitter"))
    assert np.isclose(h * lam, _v("experimental_2d", "pixel_mm"))
    # the reconstruction grid covers the object region
    assert n * h * lam >= _v("experimental_2d", "region_side_mm")


def test_experimental_3d_layout():
    lam = _v("experimental_3d", "wavelength_mm_two_spheres")
    n, h, dirs, rx, mask = fresnel3d_like_geometry()
    assert n == _v("experimental_3d", "grid") and np.isclose(h * lam, _v("experimental_3d", "pixel_mm_two_spheres"))
    a0, a1, da = _v("experimental_3d", "tx_azimuth_deg")
    p0, p1, dp = _v("experimental_3d", "tx_polar_deg")
    src = -dirs                                            # transmitter directions seen from the origin
    az = np.degrees(np.arctan2(src[:, 1], src[:, 0])) % 360
    pol = np.degrees(np.arccos(src[:, 2]))
    assert sorted(set(np.round(az).astype(int))) == list(range(a0, a1 + 1, da))
    assert sorted(set(np.round(pol).astype(int))) == list(range(p0, p1 + 1, dp))
    assert dirs.shape[0] == len(range(a0, a1 + 1, da)) * len(range(p0, p1 + 1, dp))
    r0, r1, dr = _v("experimental_3d", "rx_azimuth_deg")
    R = _v("experimental_3d", "sphere_radius_m") * 1000 / lam
    assert np.allclose(np.linalg.norm(rx, axis=1), R) and np.allclose(rx[:, 2], 0)
    assert np.allclose(np.degrees(np.arctan2(rx[:, 1], rx[:, 0])) % 360, np.arange(r0, r1 + 1, dr))
    ang = np.degrees(np.arccos(np.clip(src @ (rx / R).T, -1, 1)))
    assert np.array_equal(mask == 1, ang > _v("experimental_3d", "min_tx_rx_angle_deg") + 1e-9)


def test_experimental_3d_sources_on_the_sphere():
    lam = _v("experimental_3d", "wavelength_mm_two_spheres")
    src = fresnel3d_like_sources()
    _, _, dirs, _, _ = fresnel3d_like_geometry()
    R = _v("experimental_3d", "sphere_radius_m") * 1000 / lam
    assert np.allclose(np.linalg.norm(src, axis=1), R)
    assert np.allclose(-src / R, dirs)
