"""Point-source transmitters, free receiver positions and per-transmitter
receiver masks on the GPU against the oracle (the geometry of the paper's
experiments: sources on a line, two linear detector arrays, receivers switched
off near the active transmitter)."""

import numpy as np
import pytest
import torch

from gpu_common import rel, say, to_dev, to_np
from oracle import cisor as ocisor
from oracle import fista as ofista
from oracle import geometry, stepsize
from synth import disks_2d

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _paper_like(n, h, prec, masked=True):
    """Sources on the line x = -(1.5 + 0.75) L at azimuths -60..60 every 20
    degrees, two 24-sensor arrays at x = +-1.5 L (L the half-width), and the
    three sensors of the far array nearest to each source's line of sight off."""
    from paper_1708_01663_amd.cisor import Cisor
    half = n * h / 2
    tx = geometry.line_sources(2.25 * half, 60.0, 20.0)
    rx = geometry.linear_arrays(24, 2 * half / 12, 1.5 * half)
    T, M = tx.shape[0], rx.shape[0]
    mask = None
    if masked:
        mask = np.ones((T, M), dtype=np.uint8)
        for t in range(T):
            y_sight = tx[t, 1] * rx[24, 0] / tx[t, 0]      # the source-origin line at the far array
            far = 24 + np.argsort(np.abs(rx[24:, 1] - y_sight))[:3]
            mask[t, far] = 0
    prob = ocisor.make_problem_2d(n, h, T, M, 0.0, tx_pos=tx, rx=rx, mask=mask)
    op = Cisor(n, h, None, rx, precision=prec, tx_pos=tx)
    if masked:
        op.set_rx_mask(mask)
    return prob, op, mask


@pytest.mark.parametrize("prec,bar", [("c128", 1e-12), ("c64", 1e-6)])
def test_point_source_incident_fields(prec, bar):
    say(f"point-source incident fields {prec}")
    prob, op, _ = _paper_like(40, 1 / 8, prec, masked=False)
    assert rel(to_np(op.uin()).reshape(prob.u_in.shape), prob.u_in) < bar


def test_point_source_incident_fields_3d():
    from paper_1708_01663_amd.cisor import Cisor, plane_rx
    n, h = 8, 1 / 6
    src = np.array([[1.0, 0.3, -0.2], [-0.1, 0.2, 1.4]])
    rx = plane_rx(4, 1.0, -1.5)
    op = Cisor(n, h, None, rx, precision="c128", tx_pos=src)
    ref = geometry.point_sources(n, h, 2 * np.pi, src)
    assert rel(to_np(op.uin()).reshape(ref.shape), ref) < 1e-12


@pytest.mark.parametrize("prec,tol,bar", [("c128", 1e-11, 1e-8), ("c64", 1e-6, 1e-4)])
def test_forward_and_masked_gradient_match_oracle(prec, tol, bar):
    from paper_1708_01663_amd.cisor import SolveOpts
    say(f"point sources, arrays, mask: forward and gradient {prec}")
    n, h = 32, 1 / 8
    prob, op, mask = _paper_like(n, h, prec)
    f = disks_2d(n, 3, count=3, radius_px=(2, 5), eps_range=(1.1, 1.5))
    fd = to_dev(f.ravel(), op, real=True)
    u, y, its, code = op.forward(fd, SolveOpts(tol=tol, start=1))
    u_ref, y_ref = ocisor.forward(prob, f, tol=1e-13)
    assert code == 0
    assert rel(to_np(u).reshape(u_ref.shape), u_ref) < bar
    assert rel(to_np(y), y_ref) < bar                     # predicted data on every receiver
    y_meas = y_ref * 0.9 + 0.01 * (1 + 1j)
    g, D, *_ = op.grad(fd, to_dev(y_meas, op), SolveOpts(tol=tol, start=1))
    g_ref, D_ref = ocisor.gradient(prob, f, y_meas, tol=1e-13)
    assert abs(D - D_ref) <= bar * D_ref
    assert rel(to_np(g).reshape(n, n), g_ref) < 2 * bar
    # data on switched-off receivers are ignored
    y_junk = y_meas + (1 - mask) * 5.0
    g2, D2, *_ = op.grad(fd, to_dev(y_junk, op), SolveOpts(tol=tol, start=1))
    assert D2 == D and torch.equal(g2, g)
    # clearing the mask gives the unmasked problem
    op.set_rx_mask(None)
    g3, D3, *_ = op.grad(fd, to_dev(y_meas, op), SolveOpts(tol=tol, start=1))
    prob.mask = None
    g3_ref, D3_ref = ocisor.gradient(prob, f, y_meas, tol=1e-13)
    assert abs(D3 - D3_ref) <= bar * D3_ref and D3 > D


def test_masked_reconstruction_matches_oracle():
    """Five relaxed-FISTA iterations on the paper-like geometry with the mask."""
    from paper_1708_01663_amd.cisor import Fista, SolveOpts
    say("masked FISTA")
    n, h = 32, 1 / 8
    prob, op, _ = _paper_like(n, h, "c64")
    ftrue = disks_2d(n, 8, count=3, radius_px=(2, 5), eps_range=(1.1, 1.4))
    _, y = ocisor.forward(prob, ftrue, tol=1e-12)
    gamma = 0.5 / stepsize.born_lipschitz(prob)
    K, tau = 5, 1e-3
    f_ref, hist = ofista.cisor_reconstruct(prob, y, gamma, tau, alpha=0.96, K=K, tol=1e-12)
    fi = Fista(op, to_dev(y, op), gamma, tau, alpha=0.96, opts=SolveOpts(tol=1e-6, start=4))
    for k in range(K):
        rec = fi.step()
        assert abs(rec["D"] - hist["D"][k]) <= 1e-3 * hist["D"][k]
    assert rel(to_np(fi.f).reshape(n, n), f_ref) < 1e-3


def test_batch_with_point_sources_equals_single_contexts():
    from paper_1708_01663_amd.cisor import Batch, Cisor, SolveOpts
    n, h = 32, 1 / 8
    half = n * h / 2
    specs = [dict(n=n, h=h, tx_pos=geometry.line_sources(2.25 * half, 60.0, 30.0),
                  rx_pos=geometry.linear_arrays(16, 0.25, 1.5 * half)),
             dict(n=48, h=h, tx_pos=geometry.line_sources(2.25 * 3.0, 45.0, 45.0),
                  rx_pos=geometry.ring_receivers(20, 5.0))]
    b = Batch(specs, precision="c64", autotune=False)
    fs = [torch.tensor(disks_2d(s["n"], i, count=2, radius_px=(2, 5), eps_range=(1.1, 1.4)).ravel(),
                       dtype=torch.float32, device="cuda") for i, s in enumerate(specs)]
    us, ys, its, code = b.forward(fs, SolveOpts(tol=1e-6, start=1))
    assert code == 0
    for i, s in enumerate(specs):
        op = Cisor(s["n"], s["h"], None, s["rx_pos"], tx_pos=s["tx_pos"])
        u1, y1, its1, _ = op.forward(fs[i], SolveOpts(tol=1e-6, start=1))
        assert np.array_equal(its[i], its1)
        assert rel(to_np(ys[i]), to_np(y1)) < 1e-6
