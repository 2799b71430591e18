"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function declared in include/srf.h, and rejects invalid parameters
before touching the device."""
import ctypes as C
import os
import re

import pytest

import paper_1211_4406_amd as srf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "srf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(srf_\w+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert "srf_tree_build" in names and "srf_short_range_adjoint" in names
    L = srf.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_strerror_and_status_codes():
    L = srf.lib()
    for s in (0, -1, -2, -3, -4, -5, 7):
        assert L.srf_strerror(s)


def _build_status(**kw):
    L = srf.lib()
    p = srf.Params(**kw).c()
    h = C.c_void_p()
    buf = (C.c_double * 30)()
    ptr = C.cast(buf, C.c_void_p)
    st = L.srf_tree_build(10, ptr, ptr, ptr, 3, ptr, 1, C.byref(p), None, C.byref(h))
    return st, L.srf_last_error().decode(), h.value


@pytest.mark.parametrize("kw", [dict(r_cut=0.25), dict(r_cut=0.0), dict(r_cut=float("nan")), dict(eps=0.0),
                                dict(eps=-1.0), dict(theta=-0.1), dict(theta=1.5), dict(n_group=65),
                                dict(n_group=0), dict(n_leaf=0), dict(n_group=8, n_leaf=9), dict(precision=3),
                                dict(G=float("inf")), dict(compensated=2), dict(mac=2)])
def test_invalid_params_rejected_on_host(kw):
    st, msg, h = _build_status(**kw)
    assert st == -1 and msg and h is None


def test_null_and_size_errors():
    L = srf.lib()
    p = srf.Params().c()
    h = C.c_void_p()
    assert L.srf_tree_build(0, None, None, None, 1, None, 1, C.byref(p), None, C.byref(h)) == -1
    assert L.srf_tree_build(5, None, None, None, 1, None, 1, C.byref(p), None, C.byref(h)) == -1
    assert L.srf_tree_build(5, None, None, None, 1, None, 1, None, None, C.byref(h)) == -1
    # sizes past the 32-bit particle index are refused before any pointer is used
    for n in (2 ** 31 - 2, 2 ** 31, 2 ** 40):
        assert L.srf_tree_build(n, None, None, None, 1, None, 1, C.byref(p), None, C.byref(h)) == -1
        assert "n must lie" in L.srf_last_error().decode()
    assert L.srf_kick(-1, None, None, None, 1, None, None, None, 1, 0.1, None) == -1
    assert L.srf_make_lists(None, C.byref(p), None, C.byref(h)) == -1
    assert L.srf_short_range_force(None, None, C.byref(p), None, None, None, 1, None) == -1
    assert L.srf_short_range_potential(None, None, C.byref(p), None, 1, None) == -1
    assert L.srf_short_range_quadrupole(None, None, C.byref(p), None, None, None, 1, None) == -1
    assert L.srf_pm_force(None, 1.0, 0.05, 64, None, None, None, 1, None) == -1
    assert "tree" in L.srf_last_error().decode()
    L.srf_tree_free(None)
    L.srf_lists_free(None)
