"""GPU checks of the differentiable forward model (autograd over the C ABI).

The backward pass is the proof of Prop. 1 with the data-space cotangent w in
place of the residual; the oracle's VJP is therefore its Prop. 1 gradient with
y_meas := y(f) - w.  Checked against that, against cisor_grad, and against
central finite differences (step 1e-3) on 16 random pixels.
"""

import numpy as np
import pytest
import torch

from gpu_common import make_pair, rel, say, to_dev, to_np
from oracle import cisor as ocisor
from synth import complex_normal, disks_2d

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("prec,tol,bar", [("c64", 1e-7, 2e-4), ("c128", 1e-11, 1e-8)])
def test_vjp_matches_oracle_and_grad(prec, tol, bar):
    from paper_1708_01663_amd.autograd import scatter
    from paper_1708_01663_amd.cisor import SolveOpts
    n, h, T, M = 32, 1 / 8, 6, 24
    say(f"vjp {prec}")
    prob, op = make_pair(n, h, T, M, precision=prec)
    f = disks_2d(n, 3, count=3, radius_px=(3, 6), eps_range=(1.1, 1.6))
    _, y = ocisor.forward(prob, f, tol=1e-12)
    w = 0.2 * complex_normal((T, M), 5)
    g_ref, _ = ocisor.gradient(prob, f, y - w, tol=1e-12)
    ft = to_dev(f.ravel(), op, real=True).requires_grad_(True)
    yt = scatter(ft, op, SolveOpts(tol=tol))
    loss = (torch.conj(to_dev(w, op)) * yt).real.sum()   # dL/dRe y + i dL/dIm y = w
    loss.backward()
    assert rel(to_np(ft.grad).reshape(n, n), g_ref) < bar
    # with w = y - y_meas the VJP is the gradient of D
    y_meas = ocisor.add_noise(y, 30.0, seed=2)
    ft.grad = None
    yt = scatter(ft, op, SolveOpts(tol=tol))
    D = 0.5 * (yt - to_dev(y_meas, op)).abs().pow(2).sum()
    D.backward()
    g, Dv, *_ = op.grad(to_dev(f.ravel(), op, real=True), to_dev(y_meas, op), SolveOpts(tol=tol))
    assert rel(to_np(ft.grad), to_np(g)) < bar
    assert abs(float(D.detach()) - Dv) < 1e-5 * Dv


@pytest.mark.parametrize("mode", ["host", "recompute"])
def test_checkpoint_modes_agree(mode):
    from paper_1708_01663_amd.autograd import scatter
    from paper_1708_01663_amd.cisor import SolveOpts
    n, h, T, M = 48, 1 / 10, 5, 20
    prob, op = make_pair(n, h, T, M)
    f = disks_2d(n, 4, count=3, radius_px=(4, 9), eps_range=(1.2, 1.8))
    w = to_dev(complex_normal((T, M), 6), op)
    grads = []
    for m in ("device", mode):
        ft = to_dev(f.ravel(), op, real=True).requires_grad_(True)
        (torch.conj(w) * scatter(ft, op, SolveOpts(tol=1e-7), checkpoint=m)).real.sum().backward()
        grads.append(to_np(ft.grad))
    assert rel(grads[1], grads[0]) < 1e-4


def _fd_setup(prec, tol):
    from paper_1708_01663_amd.autograd import scatter
    from paper_1708_01663_amd.cisor import SolveOpts
    n, h, T, M = 64, 1 / 10, 8, 32
    prob, op = make_pair(n, h, T, M, precision=prec)
    f = disks_2d(n, 9, count=4, radius_px=(5, 12), eps_range=(1.1, 1.5))
    cnp = complex_normal((T, M), 7)
    c = to_dev(cnp, op)
    opts = SolveOpts(tol=tol)
    ft = to_dev(f.ravel(), op, real=True).requires_grad_(True)
    (torch.conj(c) * scatter(ft, op, opts)).real.sum().backward()
    g = to_np(ft.grad)

    def L(fv):
        _, y, _, _ = op.forward(to_dev(fv, op, real=True), opts)
        return float(np.sum((np.conj(cnp) * to_np(y)).real))   # summed in FP64

    return n, f, g, L


def test_finite_differences_on_random_pixels_c128():
    """Central differences of a random linear functional of y, step 1e-3, on 16
    random pixels inside the object (FP64 path: solve noise is negligible, so the
    O(step^2) truncation dominates)."""
    say("autograd FD pixels c128")
    n, f, g, L = _fd_setup("c128", 1e-12)
    rng = np.random.default_rng(0)
    pix = rng.choice(np.flatnonzero(f.ravel() > 0), 16, replace=False)
    step = 1e-3
    for q in pix:
        fp, fm = f.ravel().copy(), f.ravel().copy()
        fp[q] += step
        fm[q] -= step
        fd = (L(fp) - L(fm)) / (2 * step)
        assert abs(fd - g[q]) <= 1e-4 * max(abs(fd), 1e-2 * np.abs(g).max()), (q, fd, g[q])


def test_finite_differences_directional_c64():
    """complex64 path: central difference (step 1e-3) along random directions
    supported on the object, within 1e-2 relative."""
    say("autograd FD directional c64")
    n, f, g, L = _fd_setup("c64", 1e-7)
    rng = np.random.default_rng(1)
    for _ in range(3):
        d = rng.standard_normal(n * n) * (f.ravel() > 0)
        step = 1e-3
        fd = (L(f.ravel() + step * d) - L(f.ravel() - step * d)) / (2 * step)
        an = float(np.dot(g, d))
        assert abs(fd - an) <= 1e-2 * abs(an), (fd, an)
