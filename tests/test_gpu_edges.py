"""GPU edge cases: the largest grids (checked by properties that hold at any
size: the FP64 true residual of the returned field, evaluated by the oracle's
operator, and the receiver projection of that field), degenerate shapes,
single-problem batches, and bitwise reproducibility."""

import numpy as np
import pytest
import torch

from gpu_common import make_pair, rel, say, to_dev, to_np
from oracle import cisor as ocisor
from oracle import operators
from synth import disks_2d, ellipses_2d

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("n,T", [(512, 2), (384, 2), (150, 3)])   # P = 1024, 768, 384
def test_large_and_non_power_of_two_grids_meet_the_true_residual(n, T):
    """eq. u_and_v at the largest compiled FFT length and at lengths with a
    factor 3: the returned complex64 field has an FP64 true residual (oracle
    operator) within the tolerance, and its projection equals the oracle's
    projection of the same field (eq. Z_def)."""
    from paper_1708_01663_amd.cisor import SolveOpts
    say(f"large grid n={n}")
    h = 1 / 10
    prob, op = make_pair(n, h, T, 16)
    f = ellipses_2d(n, 3, inner=4, eps_range=(1.0, 1.3))
    u, y, its, code = op.forward(to_dev(f.ravel(), op, real=True), SolveOpts(tol=1e-6, maxit=20000))
    assert code == 0
    un = to_np(u).reshape(T, n, n)
    for t in range(T):
        r = prob.u_in[t] - operators.apply_A(prob.Ghat, f, un[t])
        assert np.linalg.norm(r) / np.linalg.norm(prob.u_in[t]) <= 1.05e-6, (t, its)
    assert rel(to_np(y), ocisor.project(prob, f, un)) < 2e-5


def test_single_transmitter_single_receiver_and_minimal_grid():
    """T = 1, M = 1 on the smallest grid (n = 2, P = 64) and a 16^2 grid."""
    from paper_1708_01663_amd.cisor import SolveOpts
    for n in (2, 16):
        h = 1 / 8
        prob, op = make_pair(n, h, 1, 1, rx_radius=3.0, precision="c128")
        f = np.full((n, n), 0.4)
        u_ref, y_ref = ocisor.forward(prob, f, tol=1e-13)
        u, y, its, code = op.forward(to_dev(f.ravel(), op, real=True), SolveOpts(tol=1e-12))
        assert code == 0
        assert rel(to_np(u).reshape(1, n, n), u_ref) < 1e-9
        assert rel(to_np(y), y_ref) < 1e-9
        w = np.array([[0.3 - 0.2j]])
        g, _, _ = op.vjp(to_dev(f.ravel(), op, real=True), u, to_dev(w, op), SolveOpts(tol=1e-12))
        g_ref, _ = ocisor.gradient(prob, f, y_ref - w, tol=1e-13)
        assert rel(to_np(g).reshape(n, n), g_ref) < 1e-8


def test_single_problem_batch_equals_context():
    from paper_1708_01663_amd.cisor import Batch, SolveOpts, plane_wave_dirs, ring
    n, h, T, M = 48, 1 / 10, 5, 20
    f = disks_2d(n, 4, count=3, radius_px=(3, 9), eps_range=(1.1, 1.6))
    b = Batch([dict(n=n, h=h, tx_dir=plane_wave_dirs(T), rx_pos=ring(M, n * h))], autotune=False)
    assert b.groups == 1
    fd = torch.tensor(f.ravel(), dtype=torch.float32, device="cuda")
    us, ys, its, code = b.forward([fd], SolveOpts(tol=1e-6, start=1))
    _, op = make_pair(n, h, T, M)
    u1, y1, its1, _ = op.forward(fd, SolveOpts(tol=1e-6, start=1))
    assert code == 0 and np.array_equal(its[0], its1)
    assert np.array_equal(to_np(us[0]), to_np(u1))
    assert np.array_equal(to_np(ys[0]), to_np(y1))


def test_solves_and_fista_steps_are_bitwise_reproducible():
    """Every reduction has a fixed order (no atomics): repeated runs agree bit
    for bit."""
    from paper_1708_01663_amd.cisor import Fista, SolveOpts
    n, h, T, M = 64, 1 / 10, 6, 24
    prob, op = make_pair(n, h, T, M)
    f = disks_2d(n, 7, count=3, radius_px=(4, 10), eps_range=(1.2, 1.8))
    fd = to_dev(f.ravel(), op, real=True)
    runs = [op.forward(fd, SolveOpts(tol=1e-6)) for _ in range(2)]
    assert np.array_equal(to_np(runs[0][0]), to_np(runs[1][0]))
    assert np.array_equal(runs[0][2], runs[1][2])
    y = runs[0][1]
    out = []
    for _ in range(2):
        fi = Fista(op, y, 1e-3, 1e-3, opts=SolveOpts(tol=1e-6, start=2))
        for _ in range(3):
            fi.step()
        out.append(to_np(fi.f))
    assert np.array_equal(out[0], out[1])


def test_column_variant_range_is_checked():
    """cisor_set_col_variant accepts exactly the compiled variants 0..COL_VARIANTS-1
    and refuses the indices next to them with CISOR_E_ARG, leaving the context usable."""
    from paper_1708_01663_amd import _lib
    from paper_1708_01663_amd.cisor import COL_VARIANTS
    say("column variant range")
    prob, op = make_pair(24, 1 / 8, 2, 4)
    for v in range(COL_VARIANTS):
        op.set_col_variant(v)
    for bad in (-1, COL_VARIANTS):
        with pytest.raises(_lib.CisorError) as e:
            op.set_col_variant(bad)
        assert e.value.code == _lib.E_ARG
    f = disks_2d(24, 1, count=2, radius_px=(2, 5), eps_range=(1.1, 1.5))
    x = np.random.default_rng(3).standard_normal((2, 24 * 24)) + 0j
    y = op.apply_A(to_dev(f.ravel(), op, real=True), to_dev(x, op))
    ref = operators.apply_A(prob.Ghat, f, x.reshape(2, 24, 24))
    assert rel(to_np(y).reshape(ref.shape), ref) < 2e-6


def test_solve_after_a_failed_solve_does_not_read_stale_workspaces():
    """A solve's first BiCGSTAB iteration (beta = 0) forms p = r without reading
    the p and v workspaces, which are not cleared between solves.  A solve with
    an absurd contrast (1e38) overflows its operator output v to non-finite
    values and ends unconverged or failed (a status, not a fault); the next solve
    on the same context must still match the oracle's solve (eq. u_and_v)."""
    from paper_1708_01663_amd import _lib
    from paper_1708_01663_amd.cisor import SolveOpts
    n, h, T, M = 32, 1 / 8, 4, 16
    say("solve after a failed solve")
    prob, op = make_pair(n, h, T, M, rx_radius=n * h)
    bad = torch.full((n * n,), 1e38, dtype=torch.float32, device="cuda")
    try:
        op.forward(bad, SolveOpts(tol=1e-6, start=0, maxit=20), project=False)
    except _lib.CisorError:
        pass
    f = disks_2d(n, 3, count=3, radius_px=(2, 5), eps_range=(1.1, 1.5))
    u, _, its, code = op.forward(to_dev(f.ravel(), op, real=True), SolveOpts(tol=1e-7, start=0), project=False)
    assert code == 0 and its.max() > 0
    u_ref, _ = ocisor.forward(prob, f, tol=1e-12)
    assert rel(to_np(u).reshape(T, n, n), u_ref) < 1e-4
