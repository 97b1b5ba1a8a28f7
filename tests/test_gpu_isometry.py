"""Parity of the isometry variant (per-tree Householder reflectors, Sec. 2.1
"Rotation" and Sec. 2.2) with the oracle: tree arrays, opened leaves and
candidate sets bit-exact, neighbours by the acceptance rule; the BF16 tile
path on a reflected forest against the oracle's neighbours."""
import numpy as np
import pytest

import oracle
from paper_1603_09596_amd import geraf
from parity import check_knn, ids_from_bits, leaf_set_from_bits, assert_tree_arrays_equal
from test_gpu_parity import case_data

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

_cache = {}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    geraf.load()
    yield
    for Fg, _ in _cache.values():
        Fg.free()
    _cache.clear()


def forests(name, forms=()):
    key = (name, tuple(forms))
    if key not in _cache:
        X, Q, m, t, p = case_data(name)
        seed = 77 + len(name)
        _cache[key] = (geraf.build_forest(X, m, t, p, seed, forms=forms, householder=True),
                       oracle.build_forest(X, m, t, p, seed, householder_variant=True))
    return _cache[key]


CASES = [("gauss-10k-128", 10, 300), ("ragged-3001-77", 7, 100), ("quantised", 5, 150),
         ("quantised", 5, 3), ("desc-60k-960", 10, 4096), ("scales", 10, 200)]


@pytest.mark.parametrize("name,k,c", CASES)
def test_reflected_forest_bit_exact(name, k, c):
    X, Q, _, _, _ = case_data(name)
    Fg, Fo = forests(name)
    T = Fg.export_tree()
    assert_tree_arrays_equal(T, Fo)
    ref = oracle.search(Fo, X, Q, k, c, candidates=True)
    nq = len(Q)
    lb = np.zeros((nq, Fg.m, Fg.leaf_words), np.uint32)
    cb = np.zeros((nq, (Fg.n + 31) // 32), np.uint32)
    nc = np.zeros(nq, np.int64)
    geraf.query_trace(Fg, Q, c, leaf_bits=lb, cand_bits=cb, ncand=nc)
    for i in range(nq):
        assert leaf_set_from_bits(lb[i]) == set(ref["opened"][i].tolist()), f"query {i}"
        assert np.array_equal(ids_from_bits(cb[i], Fg.n), ref["cand"][i]), f"query {i}"
    ids = np.zeros((nq, k), np.int32)
    dd = np.zeros((nq, k), np.float32)
    geraf.query(Fg, Q, k, c, ids, dd)
    check_knn(ids, dd, ref["ids"], ref["dists"], X=X, Q=Q, cand=ref["cand"])


def test_reflected_forest_tile_path(monkeypatch):
    monkeypatch.setenv("GF_SCAN_PATH", "tile")
    X, Q, _, _, _ = case_data("desc-60k-960")
    Fg, Fo = forests("desc-60k-960", forms=("bf16",))
    ref = oracle.search(Fo, X, Q, 10, 4096, trace=False)
    ids = np.zeros((len(Q), 10), np.int32)
    dd = np.zeros((len(Q), 10), np.float32)
    geraf.query(Fg, Q, 10, 4096, ids, dd, form="bf16")
    assert geraf.last_query_timing()["path"] == "tile"
    hits = 0
    for i in range(len(Q)):
        got = ids[i][ids[i] >= 0]
        for j, gid in enumerate(got.tolist()):
            diff = X[gid].astype(np.float64) - Q[i].astype(np.float64)
            true_d = float(diff @ diff)
            assert abs(dd[i][j] - true_d) <= 1e-5 * true_d
        hits += len(set(got.tolist()) & set(ref["ids"][i].tolist()))
    assert hits / ref["ids"].size >= 0.98


def test_reflected_forests_in_the_multi_index_graph():
    """gf_query_multi captures the per-tree query reflection in its graph:
    a reflected forest beside a plain one gives what single calls give, on a
    first launch and on a replay with the buffers refilled."""
    Xr, _, m, t, p = case_data("ragged-3001-77")
    plain = geraf.build_forest(Xr, m, t, p, 5)
    cases = [("gauss-10k-128", forests("gauss-10k-128")[0], 300),
             ("ragged-3001-77", plain, 100),
             ("quantised", forests("quantised")[0], 150)]
    ref, jobs = [], []
    for name, Fg, c in cases:
        _, Q, _, _, _ = case_data(name)
        Qd = torch.from_numpy(Q).to("cuda:0")
        ids = torch.empty((len(Q), 5), dtype=torch.int32, device="cuda:0")
        dd = torch.empty((len(Q), 5), dtype=torch.float32, device="cuda:0")
        geraf.query(Fg, Qd, 5, c, ids, dd)
        torch.cuda.synchronize()
        ref.append((ids.cpu().numpy(), dd.cpu().numpy()))
        jobs.append(dict(forest=Fg, Q=Qd, k=5, checks=c, form="fp32",
                         ids=torch.full((len(Q), 5), -7, dtype=torch.int32, device="cuda:0"),
                         dists=torch.full((len(Q), 5), -7.0, dtype=torch.float32, device="cuda:0")))
    for _ in range(2):
        geraf.query_multi(jobs)
        torch.cuda.synchronize()
        for j, r in zip(jobs, ref):
            assert np.array_equal(j["ids"].cpu().numpy(), r[0])
            assert np.array_equal(j["dists"].cpu().numpy(), r[1])
            j["ids"].fill_(-3)
            j["dists"].fill_(-3.0)
        torch.cuda.synchronize()
    plain.free()
