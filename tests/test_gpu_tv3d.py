"""3D CISOR on the GPU against the oracle: the TV/box prox and the TV value on
n^3 volumes (the 3D form of eq. R_def), relaxed-FISTA steps of the scalar 3D
model, and relaxed-FISTA steps of the vectorial model (the paper's appendix on
3D imaging) with that prox."""

import numpy as np
import pytest
import torch

from gpu_common import rel, say, to_dev, to_np
from oracle import fista as ofista
from oracle import tv as otv
from oracle import vec3d as ovec
from synth import ellipsoids_3d

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("n,prec,bar", [(9, "c128", 1e-12), (16, "c128", 1e-12), (16, "c64", 2e-5),
                                        (2, "c128", 1e-12)])
def test_tv_prox_and_value_3d_match_oracle(n, prec, bar):
    from test_gpu_3d import make_pair3
    say(f"3D TV prox n={n} {prec}")
    _, op = make_pair3(n, 1 / 6, 2, 4, prec, with_oracle=False)
    z = np.random.default_rng(n).uniform(-0.3, 1.8, (n, n, n))
    zd = to_dev(z.ravel(), op, real=True)
    zc = to_np(zd).reshape(n, n, n)          # the values the device holds
    for lam, lo, hi, iters in ((0.05, 0.0, 1.5, 100), (0.4, -1.0, 3.0, 37), (0.0, 0.0, 1.0, 10)):
        x = to_np(op.tv_prox(zd, lam, lo, hi, iters)).reshape(n, n, n)
        ref = otv.prox_tv_box(zc, lam, lo, hi, iters)
        assert rel(x, ref) < bar, (lam, iters)
    assert abs(op.tv_value(zd) - otv.tv_value(zc)) <= 1e-12 * otv.tv_value(zc)


def test_scalar_3d_fista_matches_oracle():
    from paper_1708_01663_amd.cisor import Fista, SolveOpts
    from oracle import cisor as ocisor
    from test_gpu_3d import make_pair3
    say("scalar 3D FISTA")
    n, h, T, K = 12, 1 / 6, 3, 3
    prob, op = make_pair3(n, h, T, 4, "c128")
    ftrue = ellipsoids_3d(n, 1, axes=(0.25, 0.45), eps_range=(1.1, 1.3))
    _, y = ocisor.forward(prob, ftrue, tol=1e-12)
    from oracle import stepsize
    gamma, tau = 1.0 / stepsize.born_lipschitz(prob), 1e-3
    f_ref, hist = ofista.cisor_reconstruct(prob, y, gamma, tau, alpha=0.96, K=K, tol=1e-12)
    fi = Fista(op, to_dev(y, op), gamma, tau, alpha=0.96, opts=SolveOpts(tol=1e-11, start=2))
    for k in range(K):
        rec = fi.step()
        assert rec["code"] == 0
        assert abs(rec["D"] - hist["D"][k]) <= 1e-8 * hist["D"][k], k
    assert np.abs(f_ref).max() > 0 and hist["D"][-1] < hist["D"][0]
    assert rel(to_np(fi.f).reshape(f_ref.shape), f_ref) < 1e-8


def test_vectorial_fista_matches_oracle():
    from paper_1708_01663_amd.cisor import SolveOpts
    from paper_1708_01663_amd.vec3d import VecCisor, VecFista
    from test_gpu_vec3d import make_vec
    say("vectorial FISTA")
    n, T, M, K = 8, 3, 8, 3
    prob, op = make_vec(n, 0.125, T, M)
    ftrue = ellipsoids_3d(n, 4, axes=(0.25, 0.45), eps_range=(1.1, 1.4))
    _, y = ovec.forward(prob, ftrue, tol=1e-13)
    gamma, tau = 10.0, 1e-4
    f_ref, hist = ovec.reconstruct(prob, y, gamma, tau, alpha=0.96, K=K, tol=1e-13)
    yd = torch.from_numpy(np.ascontiguousarray(y)).to(torch.complex128).cuda()
    fi = VecFista(op, yd, gamma, tau, alpha=0.96, opts=SolveOpts(tol=1e-12, start=2))
    for k in range(K):
        rec = fi.step()
        assert rec["code"] == 0
        assert abs(rec["D"] - hist["D"][k]) <= 1e-9 * hist["D"][k], k
    assert np.abs(f_ref).max() > 0 and hist["D"][-1] < hist["D"][0]
    assert rel(fi.f.cpu().numpy().reshape(f_ref.shape), f_ref) < 1e-8
