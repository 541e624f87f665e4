"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/lmspdhg.h declares, and its argument checks run
before any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lmspdhg.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lm_\w+|tv_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2201_05497_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        from paper_2201_05497_amd import build
        build.build()
    return L


def test_exports_every_declared_symbol(lib):
    L = lib.load()
    names = declared_functions()
    assert len(names) >= 18
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # and the binding declares a signature for each of them
    assert sorted(lib.SIGNATURES) == names


def _geom(lib, n=(16, 16, 1), n_tof=5):
    return lib.LMGeom(0x1000, 8, 1, (ctypes.c_int32 * 3)(*n), (ctypes.c_double * 3)(2.0, 2.0, 2.0),
                      n_tof, 10.0, 20.0, 3.0, 1)


def test_plan_bytes_host_only(lib):
    L = lib.load()
    b = ctypes.c_size_t(0)
    g = _geom(lib)
    assert L.lm_plan_bytes(ctypes.byref(g), 1000, 4, ctypes.byref(b)) == 0
    small = b.value
    assert L.lm_plan_bytes(ctypes.byref(g), 100000, 4, ctypes.byref(b)) == 0
    assert b.value > small > 0


def test_plan_bytes_optional_parts(lib):
    """lm_plan_bytes_ex adds the memory of each optional part to the base
    plan (lm_plan_bytes) and rejects unknown part flags."""
    L = lib.load()
    g = _geom(lib, n=(20, 20, 8))
    b = ctypes.c_size_t(0)
    assert L.lm_plan_bytes(ctypes.byref(g), 5000, 4, ctypes.byref(b)) == 0
    base = b.value
    assert L.lm_plan_bytes_ex(ctypes.byref(g), 5000, 4, 0, ctypes.byref(b)) == 0
    assert b.value == base
    ne = 20 * 20 * 8  # whole 4x4x4 bricks: no padding at this size
    sizes = {}
    for part, want in ((1, 2 * 3 * ne * 4), (2, 5000 * 4), (4, 5 * ne * 4)):
        assert L.lm_plan_bytes_ex(ctypes.byref(g), 5000, 4, part, ctypes.byref(b)) == 0
        sizes[part] = b.value - base
        assert sizes[part] == want, (part, sizes[part], want)
    assert L.lm_plan_bytes_ex(ctypes.byref(g), 5000, 4, 7, ctypes.byref(b)) == 0
    assert b.value == base + sum(sizes.values())
    assert L.lm_plan_bytes_ex(ctypes.byref(g), 5000, 4, 8, ctypes.byref(b)) == lib.LM_EINVAL


@pytest.mark.parametrize("field,value", [("n_tof", 4), ("n_tof", 0), ("n_cry", 0)])
def test_invalid_geometry_rejected(lib, field, value):
    L = lib.load()
    g = _geom(lib)
    setattr(g, field, value)
    b = ctypes.c_size_t(0)
    assert L.lm_plan_bytes(ctypes.byref(g), 10, 1, ctypes.byref(b)) == lib.LM_EINVAL
    assert len(L.lm_last_error()) > 0


def test_invalid_image_size_rejected(lib):
    L = lib.load()
    b = ctypes.c_size_t(0)
    for n in ((0, 4, 4), (513, 4, 4)):
        g = _geom(lib, n=n)
        assert L.lm_plan_bytes(ctypes.byref(g), 10, 1, ctypes.byref(b)) == lib.LM_EINVAL
    assert L.lm_fwd(None, None, None, 0, None, None) == lib.LM_EINVAL
    assert L.lm_spdhg_epoch(None, None, None, 0, None) == lib.LM_EINVAL
    assert L.lm_plan_destroy(None) == 0
    n3 = (ctypes.c_int32 * 3)(0, 1, 1)
    assert L.tv_grad(n3, 0x1000, 0x1000, None) == lib.LM_EINVAL


def test_new_entry_points_check_arguments_first(lib):
    """lm_emtv and the plan's model setters reject bad arguments before any
    device work (the pointers below are never dereferenced)."""
    L = lib.load()
    g = _geom(lib)
    P_ = 0x1000
    # lm_emtv(G, ev, s, n, n_subsets, n_iter, g, beta, denoise_iter, x, stream)
    for args in ((P_, P_, 10, 0, 1, P_, 0.03, 20, P_),      # no subsets
                 (P_, P_, -1, 4, 1, P_, 0.03, 20, P_),      # negative count
                 (P_, P_, 10, 4, -1, P_, 0.03, 20, P_),     # negative iterations
                 (P_, P_, 10, 4, 1, P_, 0.03, -5, P_),      # negative denoising steps
                 (P_, P_, 10, 4, 1, P_, -0.1, 20, P_),      # negative beta
                 (P_, P_, 10, 4, 1, P_, float("nan"), 20, P_),
                 (P_, P_, 10, 4, 1, None, 0.03, 20, P_),    # no sensitivity image
                 (None, P_, 10, 4, 1, P_, 0.03, 20, P_)):   # no events
        assert L.lm_emtv(ctypes.byref(g), *args, None) == lib.LM_EINVAL, args
        assert len(L.lm_last_error()) > 0
    bad = _geom(lib, n=(0, 4, 4))
    assert L.lm_emtv(ctypes.byref(bad), P_, P_, 10, 4, 1, P_, 0.03, 20, P_, None) == lib.LM_EINVAL
    # no iterations: nothing to do
    assert L.lm_emtv(ctypes.byref(g), P_, P_, 10, 4, 0, P_, 0.03, 20, P_, None) == 0
    f3 = (ctypes.c_double * 3)(1.0, 1.0, 1.0)
    assert L.lm_plan_set_prior_image(None, P_, 0.1, None) == lib.LM_EINVAL
    assert L.lm_plan_set_event_factors(None, P_, None) == lib.LM_EINVAL
    assert L.lm_plan_set_resolution(None, f3, None) == lib.LM_EINVAL
    assert L.lm_plan_set_tracing(None, 1) == lib.LM_EINVAL


def test_noalloc_size_limit_host_only(lib):
    """lm_fwd_noalloc refuses an image beyond its scratch array before any
    device work (the pointers are never dereferenced)."""
    L = lib.load()
    g = _geom(lib, n=(512, 512, 72))
    assert L.lm_fwd_noalloc(ctypes.byref(g), 0x1000, 0x1000, 10, 0x1000, None) == lib.LM_EINVAL
    assert b"scratch" in L.lm_last_error()
