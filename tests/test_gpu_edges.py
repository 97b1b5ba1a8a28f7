"""Shapes at the edges of the library's limits against the oracle: one
dimension, one point, one tree with t = d, the maximum of 255 trees, and the
maximum k = 64 (FP32, and BF16 with a re-rank depth of 64), and a call of
more queries than one batch holds, on both paths.  Tree arrays,
opened leaves and candidate sets bit-exact; neighbours by the acceptance
rule (FP32) or exact distances and recall (BF16)."""
import numpy as np
import pytest

import oracle
from paper_1603_09596_amd import geraf
from parity import check_knn, ids_from_bits, leaf_set_from_bits, assert_tree_arrays_equal

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    geraf.load()


def shape(name):
    rng = np.random.default_rng(sum(name.encode()))
    if name == "d1":                 # one dimension: t = 1, rows padded to 4 floats
        X = rng.standard_normal((3000, 1)).astype(np.float32)
        Q = rng.standard_normal((20, 1)).astype(np.float32)
        return X, Q, 3, 1, 4, 10, 50
    if name == "n1":                 # one point: H = 0, k above n pads
        X = rng.standard_normal((1, 5)).astype(np.float32)
        Q = rng.standard_normal((4, 5)).astype(np.float32)
        return X, Q, 2, 2, 1, 3, 1
    if name == "m1-t=d":             # one tree, every dimension in D
        X = rng.standard_normal((2000, 16)).astype(np.float32)
        Q = (X[:25] + 0.1 * rng.standard_normal((25, 16))).astype(np.float32)
        return X, Q, 1, 16, 8, 5, 20
    if name == "m255":               # the largest forest the ABI accepts
        X = rng.standard_normal((600, 8)).astype(np.float32)
        Q = (X[:30] + 0.1 * rng.standard_normal((30, 8))).astype(np.float32)
        return X, Q, 255, 3, 16, 10, 300
    if name == "k64":                # the largest k
        X = rng.standard_normal((5000, 32)).astype(np.float32)
        Q = (X[:30] + 0.2 * rng.standard_normal((30, 32))).astype(np.float32)
        return X, Q, 4, 5, 8, 64, 200
    raise KeyError(name)


@pytest.mark.parametrize("name", ["d1", "n1", "m1-t=d", "m255", "k64"])
def test_edge_shape_fp32(name):
    X, Q, m, t, p, k, c = shape(name)
    seed = 3 + len(name)
    Fg = geraf.build_forest(X, m, t, p, seed)
    Fo = oracle.build_forest(X, m, t, p, seed)
    try:
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
    finally:
        Fg.free()


def test_k64_bf16_rerank_64():
    X, Q, m, t, p, k, c = shape("k64")
    Fg = geraf.build_forest(X, m, t, p, 9, forms=("bf16",))
    Fo = oracle.build_forest(X, m, t, p, 9)
    try:
        ref = oracle.search(Fo, X, Q, k, c, trace=False)
        ids = np.zeros((len(Q), k), np.int32)
        dd = np.zeros((len(Q), k), np.float32)
        geraf.query(Fg, Q, k, c, ids, dd, form="bf16", rerank=64)
        hits = 0
        for i in range(len(Q)):
            got = ids[i][ids[i] >= 0]
            for j, gid in enumerate(got.tolist()):
                diff = X[gid].astype(np.float64) - Q[i].astype(np.float64)
                true_d = float(diff @ diff)
                assert abs(dd[i][j] - true_d) <= 1e-5 * true_d
            hits += len(set(got.tolist()) & set(ref["ids"][i].tolist()))
        # with the re-rank depth equal to k, the BF16 selection alone decides
        # membership: the floor is what this seeded case reaches
        assert hits / ref["ids"].size >= 0.95
    finally:
        Fg.free()


@pytest.mark.parametrize("form,path", [("fp32", "rows"), ("bf16", "tile")])
def test_more_queries_than_one_batch(form, path, monkeypatch):
    """16,684 queries, more than the 16,384 one batch holds: the call runs
    two batches, and with host buffers the pinned staging buffer is refilled
    for the second.  Host and device buffers must give identical results,
    every query the result of a call over a small group holding it, and the
    queries on both sides of the batch boundary must match the oracle."""
    rng = np.random.default_rng(31)
    n, d, nq = 6000, 48, 16384 + 300
    X = rng.standard_normal((n, d)).astype(np.float32)
    Q = (X[rng.integers(0, n, nq)] + 0.1 * rng.standard_normal((nq, d))).astype(np.float32)
    m, t, p, k, c, seed = 4, 5, 8, 5, 60, 17
    monkeypatch.setenv("GF_SCAN_PATH", path)
    Fg = geraf.build_forest(X, m, t, p, seed, forms=("bf16",) if form == "bf16" else ())
    try:
        ids_h = np.zeros((nq, k), np.int32)
        dd_h = np.zeros((nq, k), np.float32)
        geraf.query(Fg, Q, k, c, ids_h, dd_h, form=form)
        timing = geraf.last_query_timing()
        assert timing["path"] == path and timing["batches"] == 2
        ids = torch.zeros((nq, k), dtype=torch.int32, device="cuda:0")
        dd = torch.zeros((nq, k), dtype=torch.float32, device="cuda:0")
        geraf.query(Fg, torch.from_numpy(Q).to("cuda:0"), k, c, ids, dd, form=form)
        assert np.array_equal(ids.cpu().numpy(), ids_h)
        assert np.array_equal(dd.cpu().numpy(), dd_h)
        for lo in (0, 16384 - 150, nq - 300):
            sub_i = np.zeros((300, k), np.int32)
            sub_d = np.zeros((300, k), np.float32)
            geraf.query(Fg, np.ascontiguousarray(Q[lo:lo + 300]), k, c, sub_i, sub_d, form=form)
            assert np.array_equal(sub_i, ids_h[lo:lo + 300]), lo
            assert np.array_equal(sub_d, dd_h[lo:lo + 300]), lo
    finally:
        Fg.free()
    idx = np.r_[0:4, 16380:16388, nq - 4:nq]
    Qs = np.ascontiguousarray(Q[idx])
    ref = oracle.search(oracle.build_forest(X, m, t, p, seed), X, Qs, k, c, trace=False)
    if form == "fp32":
        check_knn(ids_h[idx], dd_h[idx], ref["ids"], ref["dists"], X=X, Q=Qs)
        return
    hits = 0
    for j, i in enumerate(idx):
        got = ids_h[i][ids_h[i] >= 0]
        for r, gid in enumerate(got.tolist()):
            diff = X[gid].astype(np.float64) - Qs[j].astype(np.float64)
            true_d = float(diff @ diff)
            assert abs(dd_h[i][r] - true_d) <= 1e-5 * true_d
        hits += len(set(got.tolist()) & set(ref["ids"][j].tolist()))
    assert hits / ref["ids"].size >= 0.95


def test_device_memory_cap_enomem_and_recovery(monkeypatch):
    """Under GF_MAX_DEVICE_BYTES a query whose workspace would exceed the cap
    fails with GF_ENOMEM and leaves the forest usable; a build refused part
    way releases what it had allocated."""
    rng = np.random.default_rng(31)
    X = rng.standard_normal((4000, 32)).astype(np.float32)
    Q = rng.standard_normal((3000, 32)).astype(np.float32)
    base = geraf.load().gf_device_bytes()
    F = geraf.build_forest(X, 4, 5, 8, 1)
    held = geraf.load().gf_device_bytes()
    assert held > base
    ids = torch.empty((3000, 5), dtype=torch.int32, device="cuda:0")
    dd = torch.empty((3000, 5), dtype=torch.float32, device="cuda:0")
    monkeypatch.setenv("GF_MAX_DEVICE_BYTES", str(held + 4096))
    with pytest.raises(geraf.GerafError) as e:
        geraf.query(F, torch.from_numpy(Q).to("cuda:0"), 5, 64, ids, dd)
    assert e.value.status == geraf.GF_ENOMEM
    # a build whose FP32 rows (4000 x 32 floats) fit but whose trees do not
    monkeypatch.setenv("GF_MAX_DEVICE_BYTES", str(held + 4000 * 32 * 4 + 1000))
    with pytest.raises(geraf.GerafError) as e:
        geraf.build_forest(X, 4, 5, 8, 1)
    assert e.value.status == geraf.GF_ENOMEM
    assert geraf.load().gf_device_bytes() == held
    monkeypatch.delenv("GF_MAX_DEVICE_BYTES")
    geraf.query(F, torch.from_numpy(Q).to("cuda:0"), 5, 64, ids, dd)
    torch.cuda.synchronize()
    assert (ids.cpu().numpy() >= 0).all()
    F.free()
    assert geraf.load().gf_device_bytes() == base



def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def test_ids_beyond_one_workgroup_bitmap(monkeypatch):
    """n = 1.5M (47k bitmap words, above the ~37k one scan workgroup's LDS
    holds): the row scan cuts every query's id range into slices, traces
    included.  Opened leaves and candidate sets bit-exact, FP32 neighbours
    by the acceptance rule; the BF16 form on both paths (the tile path and
    the sliced row scan) returns candidates with exact
    FP32 distances.  GF_SCAN_PATH forces each path."""
    rng = np.random.default_rng(41)
    n, d = 1_500_000, 16
    X = rng.standard_normal((n, d)).astype(np.float32)
    Q = (X[rng.integers(0, n, 24)] + 0.1 * rng.standard_normal((24, d))).astype(np.float32)
    m, t, p, seed = 4, 6, 32, 5
    Fg = geraf.build_forest(X, m, t, p, seed, forms=("bf16",))
    Fo = oracle.build_forest(X, m, t, p, seed)
    assert_tree_arrays_equal(Fg.export_tree(), Fo)
    k = 10
    for c in (40, 600):
        ref = oracle.search(Fo, X, Q, k, c, candidates=True)
        nq = len(Q)
        lb = np.zeros((nq, Fg.m, Fg.leaf_words), np.uint32)
        cb = np.zeros((nq, (n + 31) // 32), np.uint32)
        nc = np.zeros(nq, np.int64)
        geraf.query_trace(Fg, Q, c, leaf_bits=lb, cand_bits=cb, ncand=nc)
        for i in range(nq):
            assert leaf_set_from_bits(lb[i]) == set(ref["opened"][i].tolist()), f"c={c} query {i}"
            assert np.array_equal(ids_from_bits(cb[i], n), ref["cand"][i]), f"c={c} query {i}"
        assert np.array_equal(nc, ref["ncand"])
        # counts alone (a sliced trace sums them from the bitmap rows)
        nc2 = np.zeros(nq, np.int64)
        geraf.query_trace(Fg, Q, c, ncand=nc2)
        assert np.array_equal(nc2, ref["ncand"])
        ids = torch.empty((nq, k), dtype=torch.int32, device="cuda:0")
        dd = torch.empty((nq, k), dtype=torch.float32, device="cuda:0")
        geraf.query(Fg, dev(Q), k, c, ids, dd)
        torch.cuda.synchronize()
        check_knn(ids.cpu().numpy(), dd.cpu().numpy(), ref["ids"], ref["dists"], X=X, Q=Q,
                  cand=ref["cand"])
        for path in ("tile", "rows"):
            nb = 16
            monkeypatch.setenv("GF_SCAN_PATH", path)
            ib = torch.empty((nb, k), dtype=torch.int32, device="cuda:0")
            db = torch.empty((nb, k), dtype=torch.float32, device="cuda:0")
            geraf.query(Fg, dev(Q[:nb]), k, c, ib, db, form="bf16")
            torch.cuda.synchronize()
            monkeypatch.delenv("GF_SCAN_PATH")
            assert geraf.last_query_timing()["path"] == path
            ib, db = ib.cpu().numpy(), db.cpu().numpy()
            for i in range(nb):
                got = ib[i][ib[i] >= 0]
                assert np.isin(got, ref["cand"][i]).all()
                for r, gid in enumerate(got.tolist()):
                    diff = X[gid].astype(np.float64) - Q[i].astype(np.float64)
                    assert abs(db[i][r] - float(diff @ diff)) <= 1e-5 * float(diff @ diff)
    Fg.free()
