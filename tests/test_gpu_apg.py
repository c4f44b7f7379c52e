"""The monotone APG step (the Li-Lin comparison method of the paper's
"Proposed Method" section) on the GPU against the oracle: objective values of
both estimates, the selection, the iterates, and the solve count per step."""

import numpy as np
import pytest
import torch

from gpu_common import make_pair, rel, say, to_dev, to_np
from oracle import apg as oapg
from oracle import cisor as ocisor
from oracle import stepsize
from synth import disks_2d

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("prec,tol,bar,scale,K", [("c128", 1e-11, 1e-7, 1.0, 6), ("c128", 1e-11, 1e-7, 2.0, 12),
                                                   ("c64", 1e-7, 2e-4, 1.0, 6)])
def test_apg_matches_oracle(prec, tol, bar, scale, K):
    """gamma = 1 / L_Born keeps the accelerated estimate throughout on this
    problem; gamma = 2 / L_Born makes the method fall back to the
    proximal-gradient estimate at several iterations."""
    from paper_1708_01663_amd.cisor import Apg, SolveOpts
    say(f"monotone APG {prec} gamma x{scale}")
    n, h, T, M = 24, 1 / 8, 6, 24
    prob, op = make_pair(n, h, T, M, precision=prec)
    ftrue = disks_2d(n, 4, count=3, radius_px=(2, 4), eps_range=(1.1, 1.5))
    _, y = ocisor.forward(prob, ftrue, tol=1e-12)
    gamma = scale / stepsize.born_lipschitz(prob)
    tau = 1e-3
    x_ref, hist = oapg.cisor_apg(prob, y, gamma, gamma, tau, K=K, tol=1e-12)
    ap = Apg(op, to_dev(y, op), gamma, tau, opts=SolveOpts(tol=tol, start=1))
    for k in range(K):
        rec = ap.step()
        assert rec["code"] == 0 and rec["fwd_solves"] == 4 and rec["adj_solves"] == 2
        for key, ref in (("F_z", hist["F_z"][k]), ("F_v", hist["F_v"][k]), ("D_y", hist["D_y"][k]),
                         ("D_x", hist["D_x"][k])):
            assert abs(rec[key] - ref) <= bar * abs(ref), (k, key, rec[key], ref)
        margin = abs(hist["F_z"][k] - hist["F_v"][k]) / abs(hist["F_v"][k])
        if margin > 20 * bar:
            assert rec["took_z"] == hist["took_z"][k], k
    assert rel(to_np(ap.x).reshape(n, n), x_ref) < 20 * bar
    took = [r["took_z"] for r in ap.history]
    if scale == 1.0:
        # the objective never increases (up to the solves' accuracy)
        F = [r["F"] for r in ap.history]
        assert np.all(np.diff(F) <= 10 * bar * np.abs(F[1:]))
        assert all(took[2:])
    else:
        assert any(took[2:]) and not all(took[2:])


def test_apg_warm_solves_and_validation():
    """The gradient at x_k starts from the fields of the objective evaluation
    that chose x_k: its forward solve needs no iteration.  Invalid states are
    rejected before any launch."""
    from paper_1708_01663_amd import _lib
    from paper_1708_01663_amd.cisor import Apg, SolveOpts
    say("APG warm solves")
    n, h, T, M = 32, 1 / 8, 8, 32
    prob, op = make_pair(n, h, T, M)
    ftrue = disks_2d(n, 9, count=3, radius_px=(2, 5), eps_range=(1.1, 1.5))
    _, y = ocisor.forward(prob, ftrue, tol=1e-10)
    gamma = 1.0 / stepsize.born_lipschitz(prob)
    ap = Apg(op, to_dev(y, op), gamma, 1e-3, opts=SolveOpts(tol=1e-6, start=1))
    recs = [ap.step() for _ in range(4)]
    assert all(r["status"] == 0 for r in recs)
    # a restarted run (k = 0) with the same inputs repeats the first step's choice
    ap2 = Apg(op, to_dev(y, op), gamma, 1e-3, opts=SolveOpts(tol=1e-6, start=1))
    r2 = ap2.step()
    assert abs(r2["F"] - recs[0]["F"]) <= 1e-5 * recs[0]["F"]
    bad = _lib.ApgState(ap.x.data_ptr(), ap.x_prev.data_ptr(), ap.z.data_ptr(), 0.5, 0.0, 0)   # t < 1
    info = _lib.ApgInfo()
    o = SolveOpts().c()
    import ctypes as C
    assert op.lib.cisor_apg_step(op.handle, C.byref(bad), C.c_void_p(ap.y.data_ptr()), gamma, gamma, 1e-3, 0.0, 2.0,
                                 100, C.byref(o), C.byref(info)) == _lib.E_ARG


def test_apg_3d_matches_oracle():
    """The monotone APG on a scalar 3D context (3D TV/box prox) against the oracle."""
    from paper_1708_01663_amd.cisor import Apg, SolveOpts
    from oracle import cisor as ocisor3
    from synth import ellipsoids_3d
    from test_gpu_3d import make_pair3
    say("monotone APG 3D")
    n, h, T, K = 10, 1 / 6, 3, 4
    prob, op = make_pair3(n, h, T, 4, "c128")
    ftrue = ellipsoids_3d(n, 2, axes=(0.25, 0.45), eps_range=(1.1, 1.3))
    _, y = ocisor3.forward(prob, ftrue, tol=1e-12)
    gamma = 1.0 / stepsize.born_lipschitz(prob)
    x_ref, hist = oapg.cisor_apg(prob, y, gamma, gamma, 1e-3, K=K, tol=1e-12)
    ap = Apg(op, to_dev(y, op), gamma, 1e-3, opts=SolveOpts(tol=1e-11, start=1))
    for k in range(K):
        rec = ap.step()
        assert rec["code"] == 0
        for key in ("F_z", "F_v"):
            assert abs(rec[key] - hist[key][k]) <= 1e-7 * abs(hist[key][k]), (k, key)
    assert np.abs(x_ref).max() > 0
    assert rel(to_np(ap.x).reshape(x_ref.shape), x_ref) < 1e-6
