"""Parity over the (eps, points per leaf) grid that the eps and p sweeps of
bench.py run, on a small noisy-sphere instance: tree arrays, opened leaves
and candidate sets bit-exact with the oracle, neighbours by the acceptance
rule.  p = 1 gives leaves holding zero or one point."""
import numpy as np
import pytest

import oracle
from paper_1603_09596_amd import geraf, workloads as W
from parity import check_knn, ids_from_bits, leaf_set_from_bits, assert_tree_arrays_equal

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

_cache = {}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    geraf.load()
    yield
    for key, val in _cache.items():
        if key != "data":
            val[0].free()
    _cache.clear()


def data():
    if "data" not in _cache:
        _cache["data"] = W.noisy_sphere(4000, 100, 40, 0.1, 11)
    return _cache["data"]


def forests(p):
    if p not in _cache:
        X, _ = data()
        _cache[p] = (geraf.build_forest(X, 8, 5, p, 11), oracle.build_forest(X, 8, 5, p, 11))
    return _cache[p]


@pytest.mark.parametrize("p", [16, 4, 1])
@pytest.mark.parametrize("eps", [0.0, 0.1, 0.5, 0.9])
def test_sweep_grid_bit_exact(p, eps):
    X, Q = data()
    Fg, Fo = forests(p)
    T = Fg.export_tree()
    assert_tree_arrays_equal(T, Fo)
    c = 64
    ref = oracle.search(Fo, X, Q, 1, c, eps=eps, candidates=True)
    nq = len(Q)
    lb = np.zeros((nq, Fg.m, Fg.leaf_words), np.uint32)
    cb = np.zeros((nq, (Fg.n + 31) // 32), np.uint32)
    nc = np.zeros(nq, np.int64)
    geraf.query_trace(Fg, Q, c, leaf_bits=lb, cand_bits=cb, ncand=nc, eps=eps)
    for i in range(nq):
        assert leaf_set_from_bits(lb[i]) == set(ref["opened"][i].tolist()), f"query {i}"
        assert np.array_equal(ids_from_bits(cb[i], Fg.n), ref["cand"][i]), f"query {i}"
    assert np.array_equal(nc, ref["ncand"])
    ids = np.zeros((nq, 1), np.int32)
    dd = np.zeros((nq, 1), np.float32)
    geraf.query(Fg, Q, 1, c, ids, dd, eps=eps)
    check_knn(ids, dd, ref["ids"], ref["dists"], X=X, Q=Q, cand=ref["cand"])
