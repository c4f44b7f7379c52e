"""The non-allocating proximal map (cisor_tv_prox_noalloc) against the
context's cisor_tv_prox: the same kernels on a static work area, so the
results must be bit-identical.  Two calls in a row on one GPU share that area;
the second call is smaller than the first, so it also shows that nothing of
the first call's contents leaks into the second."""

import ctypes as C

import numpy as np
import pytest
import torch

from gpu_common import say

pytestmark = pytest.mark.gpu


def _ctx(dim, n, precision):
    from paper_1708_01663_amd.cisor import Cisor, cone_dirs, plane_rx, plane_wave_dirs, ring
    h = 1 / 10
    if dim == 2:
        return Cisor(n, h, plane_wave_dirs(1), ring(4, n * h), precision=precision)
    hw = n * h / 2
    return Cisor(n, h, cone_dirs(1), plane_rx(2, 2 * hw, -2 * hw), precision=precision)


def _noalloc(dim, n, precision, z, lam, lo, hi, inner):
    from paper_1708_01663_amd import _lib
    lib = _lib.load()
    x = torch.empty_like(z)
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    code = lib.cisor_tv_prox_noalloc(dim, n, 0 if precision == "c64" else 1, C.c_void_p(z.data_ptr()),
                                     C.c_void_p(x.data_ptr()), lam, lo, hi, inner, stream)
    _lib.check(code, "cisor_tv_prox_noalloc", allow_not_converged=False)
    return x


def _z(dim, n, seed, dtype):
    rng = np.random.default_rng(seed)
    z = rng.uniform(-0.3, 2.3, (n,) * dim)
    z[(slice(n // 4, 3 * n // 4),) * dim] += 0.7
    return torch.tensor(z.ravel(), dtype=dtype, device="cuda")


CASES = [
    # (dim, precision, first n, second n): the second call is smaller than the first
    (2, "c64", 96, 37),
    (2, "c128", 512, 50),        # 512^2 in double fills the whole static work area
    (3, "c64", 24, 9),
    (3, "c128", 64, 13),         # 64^3 in double fills it too
]


@pytest.mark.parametrize("dim,prec,n1,n2", CASES)
def test_noalloc_prox_equals_context_prox(dim, prec, n1, n2):
    for call, n in enumerate((n1, n2)):
        say(f"noalloc prox dim={dim} {prec} n={n} call {call}")
        op = _ctx(dim, n, prec)
        z = _z(dim, n, 100 * dim + n, op.rdtype)
        for lam, lo, hi, inner in ((0.05, 0.0, 2.0, 100), (0.3, 0.2, 1.0, 13), (0.0, 0.0, 2.0, 100),
                                   (0.1, -1.0, 3.0, 0)):
            ref = op.tv_prox(z, lam, lo, hi, inner)
            got = _noalloc(dim, n, prec, z, lam, lo, hi, inner)
            torch.cuda.synchronize()
            assert torch.equal(got, ref), (dim, prec, n, lam, inner)
        # in place (x aliases z), as the context call allows
        zz = z.clone()
        from paper_1708_01663_amd import _lib
        code = _lib.load().cisor_tv_prox_noalloc(dim, n, 0 if prec == "c64" else 1, C.c_void_p(zz.data_ptr()),
                                                 C.c_void_p(zz.data_ptr()), 0.05, 0.0, 2.0, 100,
                                                 C.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert code == 0
        torch.cuda.synchronize()
        assert torch.equal(zz, op.tv_prox(z, 0.05, 0.0, 2.0, 100))
        op.close()


def test_noalloc_prox_rejects_oversize_without_launching():
    from paper_1708_01663_amd import _lib
    lib = _lib.load()
    z = torch.zeros(8, device="cuda")
    p = C.c_void_p(z.data_ptr())
    assert lib.cisor_tv_prox_noalloc(2, 513, 0, p, p, 0.1, 0.0, 1.0, 10, None) == _lib.E_SIZE
    assert lib.cisor_tv_prox_noalloc(3, 65, 1, p, p, 0.1, 0.0, 1.0, 10, None) == _lib.E_SIZE
    torch.cuda.synchronize()
    assert torch.count_nonzero(z).item() == 0
