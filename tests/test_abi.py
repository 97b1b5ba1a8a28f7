"""CPU checks of the native library's boundary (no GPU compute).

The library must load, export every function declared in include/geraf.h,
and reject invalid arguments with GF_EINVAL before touching the GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1603_09596_amd import geraf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "geraf.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gf_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(geraf.LIB_PATH):
        from paper_1603_09596_amd import build
        build.build()
    return geraf.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("gf_build_forest", "gf_query", "gf_free_forest", "gf_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), f"{name} declared in geraf.h but not exported"
    assert set(geraf.EXPORTED) == set(declared_functions())


def test_version_string(lib):
    assert geraf.version().startswith("geraf-gfx950")


def _status(fn, *args):
    return fn(*args)


def test_build_rejects_bad_arguments_before_hip(lib):
    out = ctypes.c_void_p()
    X = np.zeros((10, 4), np.float32)
    p = X.ctypes.data_as(ctypes.c_void_p)
    B = lib.gf_build_forest
    assert B(None, 10, 4, 2, 2, 2, 0, 0, None, ctypes.byref(out)) == geraf.GF_EINVAL
    assert B(p, 0, 4, 2, 2, 2, 0, 0, None, ctypes.byref(out)) == geraf.GF_EINVAL
    assert B(p, 10, 0, 2, 2, 2, 0, 0, None, ctypes.byref(out)) == geraf.GF_EINVAL
    assert B(p, 10, 4, 0, 2, 2, 0, 0, None, ctypes.byref(out)) == geraf.GF_EINVAL
    assert B(p, 10, 4, 256, 2, 2, 0, 0, None, ctypes.byref(out)) == geraf.GF_EINVAL
    assert B(p, 10, 4, 2, 5, 2, 0, 0, None, ctypes.byref(out)) == geraf.GF_EINVAL
    assert B(p, 10, 4, 2, 0, 2, 0, 0, None, ctypes.byref(out)) == geraf.GF_EINVAL
    assert B(p, 10, 4, 2, 2, 0, 0, 0, None, ctypes.byref(out)) == geraf.GF_EINVAL
    assert B(p, 10, 4, 2, 2, 2, 0, 1 << 7, None, ctypes.byref(out)) == geraf.GF_EINVAL
    assert B(p, 10, 4, 2, 2, 2, 0, 0, None, None) == geraf.GF_EINVAL
    assert b"out" in lib.gf_last_error()
    Xw = np.zeros((100, 80), np.float32)
    assert B(Xw.ctypes.data_as(ctypes.c_void_p), 100, 80, 2, 65, 2, 0, 0, None,
             ctypes.byref(out)) == geraf.GF_EUNSUPPORTED
    # depth above 23: n / leaf > 2^23
    assert B(p, 1 << 25, 4, 2, 2, 1, 0, 0, None, ctypes.byref(out)) == geraf.GF_EUNSUPPORTED


def test_build_ex_rejects_unknown_variants_before_hip(lib):
    out = ctypes.c_void_p()
    X = np.zeros((10, 4), np.float32)
    p = X.ctypes.data_as(ctypes.c_void_p)
    B = lib.gf_build_forest_ex
    assert B(p, 10, 4, 2, 2, 2, 0, 0, 1 << 5, None, ctypes.byref(out)) == geraf.GF_EINVAL
    assert b"variants" in lib.gf_last_error()
    # split-value jitter is a host build without the isometry
    assert B(p, 10, 4, 2, 2, 2, 0, 0, geraf.VARIANT_JITTER | geraf.VARIANT_HOUSEHOLDER, None,
             ctypes.byref(out)) == geraf.GF_EUNSUPPORTED
    assert B(p, 10, 4, 2, 2, 2, 0, geraf.BUILD_DEVICE, geraf.VARIANT_JITTER_EXACT, None,
             ctypes.byref(out)) == geraf.GF_EUNSUPPORTED
    assert B(p, 10, 4, 2, 2, 2, 0, 1 << 7, geraf.VARIANT_HOUSEHOLDER, None,
             ctypes.byref(out)) == geraf.GF_EINVAL
    assert B(None, 10, 4, 2, 2, 2, 0, 0, geraf.VARIANT_HOUSEHOLDER, None,
             ctypes.byref(out)) == geraf.GF_EINVAL


def test_query_rejects_bad_arguments_before_hip(lib):
    Q = np.zeros((3, 4), np.float32)
    ids = np.zeros((3, 2), np.int32)
    dd = np.zeros((3, 2), np.float32)
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    qf = lib.gf_query
    assert qf(None, P(Q), 3, 2, 10, None, 0.0, 0, 0, P(ids), P(dd), None) == geraf.GF_EINVAL
    assert lib.gf_query_trace(None, P(Q), 3, 10, None, 0.0, None, None, None, None) == geraf.GF_EINVAL
    assert lib.gf_forest_info(None, None, None, None, None, None, None) == geraf.GF_EINVAL
    assert lib.gf_export_tree(None, None, None, None, None, None) == geraf.GF_EINVAL
    assert lib.gf_free_forest(None) == geraf.GF_OK


def test_query_multi_rejects_bad_arguments_before_hip(lib):
    M = lib.gf_query_multi
    jobs = (geraf.Job * 1)()
    assert M(None, 1, 0, None) == geraf.GF_EINVAL          # no jobs array
    assert M(jobs, -1, 0, None) == geraf.GF_EINVAL         # negative count
    assert M(jobs, 0, 1 << 5, None) == geraf.GF_EINVAL     # unknown flag bit
    assert M(jobs, 0, 0, None) == geraf.GF_OK              # nothing to do
    Q = np.zeros((3, 4), np.float32)
    jobs[0] = geraf.Job(None, Q.ctypes.data_as(ctypes.c_void_p), 3, 2, 8, None, 0.0, 0, 0, None, None)
    assert M(jobs, 1, 0, None) == geraf.GF_EINVAL          # forest is NULL
    assert b"forest" in lib.gf_last_error()
    b, r, t = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    assert lib.gf_multi_stats(ctypes.byref(b), ctypes.byref(r), ctypes.byref(t)) == geraf.GF_OK


def test_build_refuses_a_near_tie_in_D_before_hip(lib):
    """Columns 2 and 3 hold the same values: their variances are equal, so
    the top-3 set is not determined by the data (the oracle refuses the same
    input)."""
    rng = np.random.default_rng(44)
    X = rng.standard_normal((500, 6)).astype(np.float32)
    X[:, 0] *= 3.0
    X[:, 1] *= 2.0
    X[:, 2] *= 1.5
    X[:, 3] = X[:, 2]
    out = ctypes.c_void_p()
    p = X.ctypes.data_as(ctypes.c_void_p)
    assert lib.gf_build_forest(p, 500, 6, 2, 3, 8, 1, 0, None, ctypes.byref(out)) == geraf.GF_EINVAL
    assert b"near-tie" in lib.gf_last_error()
    assert not out.value


def test_device_memory_cap_refuses_a_build_before_hip(lib, monkeypatch):
    """GF_MAX_DEVICE_BYTES below the FP32 rows: GF_ENOMEM with no HIP call
    (this runs without a GPU)."""
    X = np.zeros((100, 8), np.float32)
    out = ctypes.c_void_p()
    monkeypatch.setenv("GF_MAX_DEVICE_BYTES", "1000")
    st = lib.gf_build_forest(X.ctypes.data_as(ctypes.c_void_p), 100, 8, 2, 2, 4, 0, 0, None,
                             ctypes.byref(out))
    assert st == geraf.GF_ENOMEM
    assert b"GF_MAX_DEVICE_BYTES" in lib.gf_last_error()
    assert lib.gf_device_bytes() == 0
