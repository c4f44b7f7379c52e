"""Host-side checks of the C ABI boundary (no GPU needed)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cisor.h")
LIB = os.path.join(ROOT, "paper_1708_01663_amd", "libcisor.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cisor_[A-Za-z0-9_]+)\s*\(", src)))


def test_header_declares_the_core_calls():
    names = declared_functions()
    for core in ("cisor_forward", "cisor_grad", "cisor_tv_prox", "cisor_fista_step"):
        assert core in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcisor.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcisor.so not built")
def test_binding_covers_header():
    from paper_1708_01663_amd import _lib
    assert sorted(_lib.exported_symbols()) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcisor.so not built")
def test_create_rejects_bad_geometry_before_touching_the_device():
    from paper_1708_01663_amd import _lib
    lib = _lib.load()
    handle = ctypes.c_void_p()
    assert lib.cisor_create(None, None, ctypes.byref(handle)) == _lib.E_ARG
    tx = (ctypes.c_double * 2)(1.0, 0.0)
    rx = (ctypes.c_double * 2)(10.0, 0.0)
    g = _lib.Geometry(2, 0, 0.1, 1.0, 1.0, 1, 1, tx, rx, 0)        # n = 0
    assert lib.cisor_create(ctypes.byref(g), None, ctypes.byref(handle)) == _lib.E_ARG
    g = _lib.Geometry(2, 600, 0.1, 1.0, 1.0, 1, 1, tx, rx, 0)      # 2n > 1024
    assert lib.cisor_create(ctypes.byref(g), None, ctypes.byref(handle)) == _lib.E_UNSUPPORTED
    g = _lib.Geometry(2, 32, 0.1, 1.0, 1.0, 1, 1, tx, rx, 7)       # bad precision
    assert lib.cisor_create(ctypes.byref(g), None, ctypes.byref(handle)) == _lib.E_ARG
    g = _lib.Geometry(4, 32, 0.1, 1.0, 1.0, 1, 1, tx, rx, 0)       # only 2D and 3D grids
    assert lib.cisor_create(ctypes.byref(g), None, ctypes.byref(handle)) == _lib.E_ARG
    # point sources: a kind other than 0/1, no positions, a source inside the grid's square
    src_in = (ctypes.c_double * 2)(0.5, -1.0)          # |x| < n h / 2 = 1.6 and |y| < 1.6
    src_out = (ctypes.c_double * 2)(0.5, -1.7)
    for kind, pos in ((2, src_out), (1, None), (1, src_in)):
        g = _lib.Geometry(2, 32, 0.1, 1.0, 1.0, 1, 1, None, rx, 0, kind, pos)
        assert lib.cisor_create(ctypes.byref(g), None, ctypes.byref(handle)) == _lib.E_ARG
    g = _lib.Geometry(2, 32, 0.1, 1.0, 1.0, 1, 1, None, rx, 0)    # plane waves need directions
    assert lib.cisor_create(ctypes.byref(g), None, ctypes.byref(handle)) == _lib.E_ARG
    assert lib.cisor_set_rx_mask(None, None) == _lib.E_ARG
    assert lib.cisor_tv_value(None, None, None) == _lib.E_ARG
    assert lib.cisor_destroy(None) == _lib.E_ARG
    assert lib.cisor_status_string(_lib.E_ARG) == b"invalid argument"


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcisor.so not built")
def test_batch_create_rejects_bad_geometries_before_touching_the_device():
    from paper_1708_01663_amd import _lib
    lib = _lib.load()
    handle = ctypes.c_void_p()
    tx = (ctypes.c_double * 2)(1.0, 0.0)
    rx = (ctypes.c_double * 2)(10.0, 0.0)
    ok = _lib.Geometry(2, 32, 0.1, 1.0, 1.0, 1, 1, tx, rx, 0)
    assert lib.cisor_batch_create(None, 1, None, ctypes.byref(handle)) == _lib.E_ARG
    geoms = (_lib.Geometry * 2)(ok, ok)
    assert lib.cisor_batch_create(geoms, 0, None, ctypes.byref(handle)) == _lib.E_ARG
    geoms[1] = _lib.Geometry(2, 32, 0.1, 1.0, 1.0, 1, 1, tx, rx, 1)     # mixed precision
    assert lib.cisor_batch_create(geoms, 2, None, ctypes.byref(handle)) == _lib.E_ARG
    geoms[1] = _lib.Geometry(3, 16, 0.1, 1.0, 1.0, 1, 1, tx, rx, 0)     # 3D is not batched
    assert lib.cisor_batch_create(geoms, 2, None, ctypes.byref(handle)) == _lib.E_ARG
    geoms[1] = _lib.Geometry(2, 32, 0.1, 1.0, 1.0, 1, 1, None, rx, 0, 1,
                             (ctypes.c_double * 2)(0.0, 0.0))          # a source at the grid centre
    assert lib.cisor_batch_create(geoms, 2, None, ctypes.byref(handle)) == _lib.E_ARG
    geoms[1] = _lib.Geometry(2, 600, 0.1, 1.0, 1.0, 1, 1, tx, rx, 0)    # 2n > 1024
    assert lib.cisor_batch_create(geoms, 2, None, ctypes.byref(handle)) == _lib.E_UNSUPPORTED
    assert lib.cisor_batch_destroy(None) == _lib.E_ARG
    assert lib.cisor_set_col_variant(None, 0) == _lib.E_ARG


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_1708_01663_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".cpp", ".hip", ".hpp", ".h")):
                src = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in src and "from oracle" not in src, fn


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcisor.so not built")
def test_vectorial_create_rejects_bad_geometry_before_touching_the_device():
    from paper_1708_01663_amd import _lib
    lib = _lib.load()
    handle = ctypes.c_void_p()
    D = ctypes.c_double
    tx = (D * 3)(0.0, 0.6, -0.8)
    rx_out = (D * 3)(0.0, 0.0, -2.0)       # outside the cube of half-width 8 * 0.125 / 2 = 0.5
    rx_in = (D * 3)(0.1, 0.2, -0.4)        # inside it: the dyadic kernel is singular there
    good = dict(dim=3, n=8, h=0.125, wl=1.0, eps=1.0, T=1, M=1, tx=tx, rx=rx_out, prec=1, kind=0, pos=None)

    def make(**kw):
        a = dict(good, **kw)
        return _lib.Geometry(a["dim"], a["n"], a["h"], a["wl"], a["eps"], a["T"], a["M"], a["tx"], a["rx"],
                             a["prec"], a["kind"], a["pos"])

    cases = [(dict(dim=2), _lib.E_ARG), (dict(n=1), _lib.E_ARG), (dict(h=-1.0), _lib.E_ARG),
             (dict(rx=rx_in), _lib.E_ARG), (dict(tx=(D * 3)(0.0, 0.0, 0.0)), _lib.E_ARG),
             (dict(rx=None), _lib.E_ARG), (dict(prec=0), _lib.E_UNSUPPORTED),
             (dict(eps=2.0), _lib.E_UNSUPPORTED), (dict(kind=1, pos=(D * 3)(0.0, 0.0, 0.3)), _lib.E_ARG),   # dipole inside the cube
             (dict(kind=1, pos=None), _lib.E_ARG),
             (dict(n=600, h=0.001), _lib.E_UNSUPPORTED)]
    for kw, want in cases:
        g = make(**kw)
        assert lib.cisor_vec_create(ctypes.byref(g), None, ctypes.byref(handle)) == want, kw
        assert not handle.value
    assert lib.cisor_vec_create(None, None, ctypes.byref(handle)) == _lib.E_ARG
    # calls on a null context
    assert lib.cisor_vec_apply_A(None, None, None, None, 0) == _lib.E_ARG
    assert lib.cisor_vec_destroy(None) == _lib.E_ARG


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcisor.so not built")
def test_new_entry_points_reject_null_handles_before_touching_the_device():
    """The monotone APG step, the vectorial model's calls and the 3D-capable
    TV calls validate their arguments on the host first."""
    from paper_1708_01663_amd import _lib
    lib = _lib.load()
    o = _lib.LsOpts(1e-6, 100, 1, 50, 10)
    st = _lib.ApgState(None, None, None, 1.0, 0.0, 0)
    info = _lib.ApgInfo()
    assert lib.cisor_apg_step(None, ctypes.byref(st), None, 1.0, 1.0, 0.0, 0.0, 1.0, 10, ctypes.byref(o),
                              ctypes.byref(info)) == _lib.E_ARG
    fs = _lib.FistaState(None, None, None, 1.0, 0)
    si = _lib.StepInfo()
    assert lib.cisor_vec_fista_step(None, ctypes.byref(fs), None, 1.0, 0.0, 0.9, 0.0, 1.0, 10, ctypes.byref(o),
                                    ctypes.byref(si)) == _lib.E_ARG
    D = ctypes.c_double()
    mr = ctypes.c_double()
    assert lib.cisor_vec_grad(None, None, None, None, ctypes.byref(D), ctypes.byref(o), None,
                              ctypes.byref(mr)) == _lib.E_ARG
    assert lib.cisor_vec_forward(None, None, ctypes.byref(o), None, None, None, None) == _lib.E_ARG
    assert lib.cisor_vec_project(None, None, None, None) == _lib.E_ARG
    assert lib.cisor_vec_set_rx_mask(None, None) == _lib.E_ARG
    assert lib.cisor_vec_set_stream(None, None) == _lib.E_ARG
    assert lib.cisor_vec_get_uin(None, None) == _lib.E_ARG
    assert lib.cisor_tv_prox(None, None, None, 0.1, 0.0, 1.0, 10) == _lib.E_ARG
    assert lib.cisor_tv_value(None, None, ctypes.byref(D)) == _lib.E_ARG


def test_binding_fails_loudly_without_the_library(tmp_path):
    """There is no CPU fallback: loading a missing library raises at once (the
    binding's cache is cleared for the call and restored afterwards)."""
    from paper_1708_01663_amd import _lib
    saved = _lib._lib
    _lib._lib = None
    try:
        with pytest.raises(RuntimeError, match="no CPU fallback"):
            _lib.load(str(tmp_path / "libcisor.so"))
    finally:
        _lib._lib = saved


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcisor.so not built")
def test_noalloc_prox_rejects_bad_arguments_before_touching_the_device():
    """cisor_tv_prox_noalloc checks its arguments and the size limit of its
    static work area on the host, before it looks up any device."""
    from paper_1708_01663_amd import _lib
    lib = _lib.load()
    dummy = ctypes.c_void_p(256)          # never dereferenced: every call below is rejected first
    assert lib.cisor_tv_prox_noalloc(4, 8, 0, dummy, dummy, 0.1, 0.0, 1.0, 10, None) == _lib.E_ARG
    assert lib.cisor_tv_prox_noalloc(2, 0, 0, dummy, dummy, 0.1, 0.0, 1.0, 10, None) == _lib.E_ARG
    assert lib.cisor_tv_prox_noalloc(2, 8, 2, dummy, dummy, 0.1, 0.0, 1.0, 10, None) == _lib.E_ARG
    assert lib.cisor_tv_prox_noalloc(2, 8, 0, None, dummy, 0.1, 0.0, 1.0, 10, None) == _lib.E_ARG
    assert lib.cisor_tv_prox_noalloc(2, 8, 0, dummy, None, 0.1, 0.0, 1.0, 10, None) == _lib.E_ARG
    assert lib.cisor_tv_prox_noalloc(2, 8, 0, dummy, dummy, -0.1, 0.0, 1.0, 10, None) == _lib.E_ARG
    assert lib.cisor_tv_prox_noalloc(2, 8, 0, dummy, dummy, 0.1, 1.0, 0.0, 10, None) == _lib.E_ARG
    assert lib.cisor_tv_prox_noalloc(2, 8, 0, dummy, dummy, 0.1, 0.0, 1.0, -1, None) == _lib.E_ARG
    assert lib.cisor_tv_prox_noalloc(2, 513, 0, dummy, dummy, 0.1, 0.0, 1.0, 10, None) == _lib.E_SIZE
    assert lib.cisor_tv_prox_noalloc(3, 65, 1, dummy, dummy, 0.1, 0.0, 1.0, 10, None) == _lib.E_SIZE
    assert lib.cisor_status_string(_lib.E_SIZE).startswith(b"problem larger than the static work area")
