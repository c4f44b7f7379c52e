"""Named workload recipes (sizes, wavelengths, noise levels, seeds).

Lengths are in wavelengths (lambda = 1, so the vacuum wavenumber is 2*pi).
Transmitters are plane waves at uniform angles over 2*pi; receivers sit on a
ring of radius ``rx_radius_halfwidths`` times the grid half-width.
"""

from __future__ import annotations

from dataclasses import dataclass, field


@dataclass(frozen=True)
class Workload:
    name: str
    n: int                 # grid side (pixels)
    h: float               # pixel size in wavelengths
    T: int                 # transmitters
    M: int                 # receivers
    phantom: str           # "disks" | "ellipses"
    phantom_kw: dict = field(default_factory=dict)
    snr_db: float = 30.0
    tau: float = 5e-4
    iters: int = 100       # relaxed-FISTA iterations
    ls_tol: float = 1e-6
    precision: str = "c64"
    rx_radius_halfwidths: float = 2.0
    eps_b: float = 1.0
    seed: int = 0
    alpha: float = 0.96
    lo: float = 0.0
    hi: float = 2.0

    @property
    def N(self) -> int:
        return self.n * self.n

    @property
    def rx_radius(self) -> float:
        return self.rx_radius_halfwidths * (self.n * self.h / 2.0)


WORKLOADS = {
    # 32x32, lambda/8 pixels, three weak disks, 8 Tx, 32 Rx, complex128, LS 1e-8.
    "small_c128": Workload(
        name="small_c128", n=32, h=1.0 / 8, T=8, M=32, phantom="disks",
        phantom_kw=dict(count=3, radius_px=(2.0, 5.0), eps_range=(1.1, 1.5)),
        snr_db=40.0, tau=1e-3, iters=20, ls_tol=1e-8, precision="c128"),
    # 256x256, lambda/10 pixels, random ellipses eps in [1, 2], 60 Tx, 360 Rx.
    "strong_256": Workload(
        name="strong_256", n=256, h=1.0 / 10, T=60, M=360, phantom="ellipses",
        phantom_kw=dict(inner=7, eps_range=(1.0, 2.0)),
        snr_db=30.0, tau=5e-4, iters=100, ls_tol=1e-6, precision="c64"),
}


def make_phantom(w: Workload):
    """Contrast image of a workload (float64, shape (n, n))."""
    from .phantoms import disks_2d, ellipses_2d
    if w.phantom == "disks":
        return disks_2d(w.n, w.seed, eps_b=w.eps_b, **w.phantom_kw)
    if w.phantom == "ellipses":
        return ellipses_2d(w.n, w.seed, eps_b=w.eps_b, **w.phantom_kw)
    raise ValueError(w.phantom)


# Batched uneven reconstructions: 32 independent problems, grids drawn from
# {64, 96, 128, 192, 256, 384, 512}^2, 8..64 plane-wave transmitters each,
# receivers = 4 x transmitters on a ring of twice the half-width, seeded random
# disks eps in [1.05, 1.8], lambda/10 pixels, 30 dB noise, 50 iterations.
BATCH_GRIDS = (64, 96, 128, 192, 256, 384, 512)


def batched_uneven(count=32, seed=0, grids=BATCH_GRIDS, t_range=(8, 64), h=0.1, tau=5e-4, snr_db=30.0, iters=50):
    """Per-problem recipes of the batched workload: a list of Workload records
    (name batch_<i>) with their own grid, transmitter count and phantom seed."""
    import numpy as np
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.choice(grids))
        T = int(rng.integers(t_range[0], t_range[1] + 1))
        out.append(Workload(
            name=f"batch_{i}", n=n, h=h, T=T, M=4 * T, phantom="disks",
            phantom_kw=dict(count=int(rng.integers(2, 7)), radius_px=(n / 32, n / 12), eps_range=(1.05, 1.8)),
            snr_db=snr_db, tau=tau, iters=iters, ls_tol=1e-6, precision="c64", seed=1000 + i))
    return out


# The paper's geometries, as positions only (lengths in wavelengths).
#
# Simulated-data setup: lambda = 7.49 cm; a 120 cm square image on 128^2 pixels
# (lambda/8); two linear detectors of 169 sensors 3.84 cm apart at x = -+95.9
# cm; 25 line sources on the line 48.0 cm left of the left detector, at
# azimuths (seen from the origin) -60..60 degrees every 5 degrees.
#
# 2D experimental setup (stand-in for the measured data, which are not used):
# 8 sources and 360 receivers on a circle of 1.67 m at lambda = 99.9 mm
# (16.7 lambda), uniformly spaced; for each source the 119 receivers nearest
# to it are switched off (241 active).  The 128^2 grid at lambda/16 used here is
# coarser than the paper's 1.2 mm pixels (so the object region is 8 lambda
# wide, not 1.5 lambda).
def paper_sim_geometry():
    """(n, h, tx_pos [25, 2], rx_pos [338, 2]) of the simulated-data setup."""
    import numpy as np
    lam = 7.49
    det, spacing, src = 95.9 / lam, 3.84 / lam, (95.9 + 48.0) / lam
    ys = (np.arange(169) - 84) * spacing
    rx = np.concatenate([np.stack([np.full(169, -det), ys], 1), np.stack([np.full(169, det), ys], 1)])
    th = np.deg2rad(np.arange(-60, 61, 5))
    tx = np.stack([np.full(th.size, -src), src * np.tan(th)], 1)
    return 128, 120.0 / lam / 128, tx, rx


def fresnel_like_geometry(n=128, h=1.2 / 99.9):
    """(n, h, tx_pos [8, 2], rx_pos [360, 2], mask [8, 360]) of the 2D
    experimental setup's layout in wavelengths (3 GHz, lambda 99.9 mm, pixel
    1.2 mm, so 128 pixels cover the 150 mm object region): sources and
    receivers on one circle, the 119 receivers nearest to each source off."""
    import numpy as np
    R = 1670.0 / 99.9
    ph_t = 2 * np.pi * np.arange(8) / 8
    ph_r = 2 * np.pi * np.arange(360) / 360
    tx = R * np.stack([np.cos(ph_t), np.sin(ph_t)], 1)
    rx = R * np.stack([np.cos(ph_r), np.sin(ph_r)], 1)
    mask = np.ones((8, 360), dtype=np.uint8)
    for t in range(8):
        d = np.abs(np.angle(np.exp(1j * (ph_r - ph_t[t]))))
        mask[t, np.argsort(d, kind="stable")[:119]] = 0
    return n, h, tx, rx, mask


def fresnel3d_like_geometry(n=32):
    """(n, h, tx_dir [81, 3], rx_pos [36, 3], mask [81, 36]) of the 3D
    experimental setup's layout in wavelengths (4 GHz, lambda 74.9 mm, voxel
    4.7 mm): transmitters on the sphere of radius 1.769 m at azimuths 20..340
    every 40 degrees and polar angles 30..150 every 15 degrees, each seen on the
    grid as the plane wave travelling from it towards the origin; receivers on
    the azimuthal circle of the same radius every 10 degrees, active for a
    transmitter when more than 50 degrees away from it."""
    import numpy as np
    lam = 74.9
    R = 1769.0 / lam
    az = np.deg2rad(np.arange(20, 341, 40))
    pol = np.deg2rad(np.arange(30, 151, 15))
    A, P = np.meshgrid(az, pol, indexing="ij")
    src = np.stack([np.sin(P) * np.cos(A), np.sin(P) * np.sin(A), np.cos(P)], -1).reshape(-1, 3)
    ph = np.deg2rad(np.arange(0, 351, 10))
    rx_unit = np.stack([np.cos(ph), np.sin(ph), np.zeros_like(ph)], 1)
    ang = np.degrees(np.arccos(np.clip(src @ rx_unit.T, -1.0, 1.0)))
    mask = (ang > 50.0 + 1e-9).astype(np.uint8)     # exactly 50 degrees counts as within
    return n, 4.7 / lam, -src, R * rx_unit, mask


def fresnel3d_like_sources():
    """Positions [81, 3] (in wavelengths at 4 GHz) of the 3D experiment's
    transmitters on the sphere of radius 1.769 m, in the order of the
    directions of fresnel3d_like_geometry (which point from them to the origin)."""
    _, _, dirs, _, _ = fresnel3d_like_geometry()
    return -dirs * (1769.0 / 74.9)


def two_spheres_3d(n, h, radius=25.0 / 74.9, contrast=1.6):
    """Contrast f = eps - 1 of two touching spheres (diameter 50 mm at lambda
    74.9 mm, eps 2.6) side by side along x, centred in the grid; voxels whose
    centre lies inside a sphere take the full contrast."""
    import numpy as np
    x = (np.arange(n) - (n - 1) / 2.0) * h
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    f = np.zeros((n, n, n))
    for cx in (-radius, radius):
        f[(X - cx) ** 2 + Y ** 2 + Z ** 2 <= radius ** 2] = contrast
    return f
