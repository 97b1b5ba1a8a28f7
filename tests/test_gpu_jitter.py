"""Split-value jitter (Sec. 2.1 "Split value") on the GPU query path against
the FP64 oracle's jittered trees.

Bar: the library's padded layout equals the oracle's layout of its explicit
trees bit for bit (split values, including the +inf pass-through nodes,
dimensions, ids, per-tree leaf offsets); each query's opened leaves and
candidate set equal the oracle's explicit-tree search (rows path, and the
tile path's candidate words); neighbours by the acceptance rule.  Budgets
run from one leaf to every leaf of the trees (never the padding leaves).
"""
import numpy as np
import pytest

import oracle
from paper_1603_09596_amd import geraf, workloads as W
from parity import assert_tree_arrays_equal, check_knn, ids_from_bits, leaf_set_from_bits

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    geraf.load()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def jitter_case(name):
    """(X, Q, m, t, p, diameter)."""
    if name == "uniform-1500-8-exact":
        rng = np.random.default_rng(3)
        X = rng.random((1500, 8)).astype(np.float32)
        Q = rng.random((40, 8)).astype(np.float32)
        return X, Q, 3, 5, 4, "exact"
    if name == "quantised-2000-24":
        rng = np.random.default_rng(5)
        X = rng.integers(0, 6, (2000, 24)).astype(np.float32)
        Q = (X[rng.integers(0, 2000, 40)] + rng.integers(-1, 2, (40, 24))).astype(np.float32)
        return X, Q, 3, 5, 6, "approx"
    if name == "uniform-3000-64":
        rng = np.random.default_rng(7)
        X = rng.random((3000, 64)).astype(np.float32)
        Q = rng.random((30, 64)).astype(np.float32)
        return X, Q, 2, 5, 8, "approx"
    if name == "gauss-2500-16":
        X, Q, _ = W.gauss(2500, 16, 30, 0.2, 11)
        return X, Q, 3, 5, 8, "approx"
    raise KeyError(name)


CASES = ["uniform-1500-8-exact", "quantised-2000-24", "uniform-3000-64", "gauss-2500-16"]
_cache = {}


def forests(name):
    if name not in _cache:
        X, Q, m, t, p, diam = jitter_case(name)
        Fo = oracle.build_forest_jitter(X, m, t, p, 41, diameter=diam)
        Fg = geraf.build_forest(X, m, t, p, 41, forms=("bf16",), jitter=diam)
        _cache[name] = (X, Q, Fg, Fo)
    return _cache[name]


def real_leaves(Fo):
    return sum(int((Fo["dim"][tr, :Fo["nnodes"][tr]] < 0).sum()) for tr in range(Fo["m"]))


@pytest.mark.parametrize("name", CASES)
def test_jitter_layout_bit_exact(name):
    X, Q, Fg, Fo = forests(name)
    T = Fg.export_tree()
    assert_tree_arrays_equal(T, dict(oracle.jitter_layout(Fo), D=Fo["D"], H=Fo["H"]))


@pytest.mark.parametrize("name", CASES)
def test_jitter_opened_leaves_candidates_and_neighbours(name):
    X, Q, Fg, Fo = forests(name)
    L = real_leaves(Fo)
    nq, k = len(Q), 5
    for c in (1, 9, max(2, L // 20), L // 2, L, L + 1000):
        ref = oracle.search(Fo, X, Q, k, c, candidates=True)
        lb = dev(np.zeros((nq, Fg.m, Fg.leaf_words), np.uint32))
        cb = dev(np.zeros((nq, (Fg.n + 31) // 32), np.uint32))
        nc = dev(np.zeros(nq, np.int64))
        geraf.query_trace(Fg, dev(Q), c, leaf_bits=lb, cand_bits=cb, ncand=nc)
        torch.cuda.synchronize()
        lb, cb, nc = lb.cpu().numpy(), cb.cpu().numpy(), nc.cpu().numpy()
        for i in range(nq):
            assert leaf_set_from_bits(lb[i]) == set(ref["opened"][i].tolist()), f"c={c} query {i}"
            assert np.array_equal(ids_from_bits(cb[i], Fg.n), ref["cand"][i]), f"c={c} query {i}"
        assert np.array_equal(nc, ref["ncand"])
        ids = torch.empty((nq, k), dtype=torch.int32, device="cuda:0")
        dd = torch.empty((nq, k), dtype=torch.float32, device="cuda:0")
        geraf.query(Fg, dev(Q), k, c, ids, dd)
        torch.cuda.synchronize()
        check_knn(ids.cpu().numpy(), dd.cpu().numpy(), ref["ids"], ref["dists"], X=X, Q=Q,
                  cand=ref["cand"])


@pytest.mark.parametrize("name", CASES[:2])
def test_jitter_tile_path_candidate_words(name):
    X, Q, Fg, Fo = forests(name)
    c = max(2, real_leaves(Fo) // 10)
    ref = oracle.search(Fo, X, Q, 5, c, candidates=True)
    cb = np.zeros((len(Q), (Fg.n + 31) // 32), np.uint32)
    nc = np.zeros(len(Q), np.int64)
    geraf.query_trace(Fg, Q, c, cand_bits=cb, ncand=nc, path="tile")
    for i in range(len(Q)):
        assert np.array_equal(ids_from_bits(cb[i], Fg.n), ref["cand"][i]), f"query {i}"
    assert np.array_equal(nc, ref["ncand"])


def test_jitter_refused_with_device_build_or_isometry():
    X, _, m, t, p, _ = jitter_case("uniform-1500-8-exact")
    for kw in (dict(device_build=True), dict(householder=True)):
        with pytest.raises(geraf.GerafError) as e:
            geraf.build_forest(X, m, t, p, 1, jitter="approx", **kw)
        assert e.value.status == geraf.GF_EUNSUPPORTED
