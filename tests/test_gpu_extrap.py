"""Extrapolated starting guesses of the FISTA solves (start mode 4): the
iterates equal those of the previous-fields start up to the solve tolerance,
the solves take fewer BiCGSTAB iterations, and the mode is refused outside a
FISTA step.  (Parity of the mode with the oracle's reconstruction is in
test_gpu_parity.)"""

import numpy as np
import pytest
import torch

from gpu_common import rel, say, to_dev, to_np
from synth import ellipses_2d

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _reconstruct(start, n, T, M, K, seed=0):
    from paper_1708_01663_amd.cisor import Cisor, Fista, SolveOpts, plane_wave_dirs, ring
    op = Cisor(n, 0.1, plane_wave_dirs(T), ring(M, n * 0.1))
    f = ellipses_2d(n, seed, inner=7, eps_range=(1.0, 2.0))
    _, y, _, code = op.forward(to_dev(f.ravel(), op, real=True), SolveOpts(tol=1e-7, maxit=20000, start=1))
    assert code == 0
    gamma = 1.0 / op.born_lipschitz(30)
    fi = Fista(op, y, gamma, 5e-4, alpha=0.96, opts=SolveOpts(tol=1e-6, start=start))
    its, D = 0, []
    for _ in range(K):
        rec = fi.step()
        assert rec["code"] == 0 and rec["status"] == 0, rec
        assert rec["relres"] <= 1e-6
        its += rec["fwd_sum"] + rec["adj_sum"]
        D.append(rec["D"])
    return to_np(fi.f), np.array(D), its


def test_extrapolated_start_same_iterates_fewer_iterations():
    """25 iterations on a 128^2 grid (eps in [1, 2], 16 Tx): start 4 against
    start 2 from the same data."""
    n, T, M, K = 128, 16, 64, 25
    say("extrapolated start vs previous fields, 128^2")
    f2, D2, it2 = _reconstruct(2, n, T, M, K)
    f4, D4, it4 = _reconstruct(4, n, T, M, K)
    say(f"BiCGSTAB iterations: previous fields {it2}, extrapolated {it4}")
    assert np.all(np.abs(D4 - D2) <= 1e-4 * D2)
    assert rel(f4, f2) < 1e-3
    assert it4 < it2


def test_extrapolated_start_is_refused_outside_fista():
    from paper_1708_01663_amd import _lib
    from paper_1708_01663_amd.cisor import Cisor, SolveOpts, plane_wave_dirs, ring
    op = Cisor(32, 0.125, plane_wave_dirs(2), ring(4, 4.0))
    f = torch.zeros(op.N, dtype=op.rdtype, device=op.device)
    with pytest.raises(_lib.CisorError):
        op.forward(f, SolveOpts(start=4))
    with pytest.raises(_lib.CisorError):   # start 5 (guess with zero fallback) is valid; 6 is not a mode
        op.forward(f, SolveOpts(start=6))
