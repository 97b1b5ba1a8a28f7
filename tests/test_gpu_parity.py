"""GPU parity: the HIP query path (through the C ABI) against the FP64 oracle.

Bar (per case): tree arrays bit-equal; each query's opened leaves and
candidate set bit-equal; neighbours by the acceptance rule of parity.py
(FP64 distances within 1e-5 relative, ids equal up to 1e-6 ties).  The
reduced-precision forms share the candidate sets and are scored by recall
against the oracle's top-k, with every returned distance exact to 1e-5.
"""
import numpy as np
import pytest

import oracle
from paper_1603_09596_amd import geraf, workloads as W
from parity import check_knn, ids_from_bits, leaf_set_from_bits, assert_tree_arrays_equal

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    geraf.load()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def case_data(name):
    """(X, Q, m, t, p) of a named parity case (seeded, several tiles and a
    ragged tail in every dimension that the kernels tile)."""
    if name == "gauss-10k-128":
        w = W.make("gauss-10k-128")
        return w.X, w.Q, w.m, w.t, w.p
    if name == "sphere-20k-1000":
        X, Q, _ = W.sphere(20_000, 1000, 120, 0.3, 1)
        return X, Q, 8, 5, 16
    if name == "desc-60k-960":
        X, Q, _ = W.descriptor(60_000, 960, 80, 0.02, 2)
        return X, Q, 16, 5, 32
    if name == "gauss-4k-10000":
        X, Q, _ = W.gauss(4000, 10_000, 40, 0.05, 4, boost_dims=500, boost=10.0)
        return X, Q, 16, 10, 16
    if name == "ragged-3001-77":
        X, Q, _ = W.gauss(3001, 77, 90, 0.2, 7)
        return X, Q, 3, 7, 5
    if name == "multi-d2048":
        X, Q, _ = W.gauss(9000, 2048, 40, 0.05, 9)
        return X, Q, 8, 5, 16
    if name == "single-leaf":
        X, Q, _ = W.gauss(50, 6, 10, 0.3, 3)
        return X, Q, 2, 2, 64
    if name == "quantised":
        rng = np.random.default_rng(5)
        X = rng.integers(0, 8, (5000, 40)).astype(np.float32)
        Q = (X[rng.integers(0, 5000, 60)] + rng.integers(-1, 2, (60, 40))).astype(np.float32)
        return X, Q, 4, 6, 8
    if name == "scales":
        # per-dimension scales over six decades: trees whose top splits fall
        # on different dimensions have very different eff distributions
        rng = np.random.default_rng(11)
        sc = 10.0 ** rng.uniform(-3, 3, 16)
        X = (rng.standard_normal((8000, 16)) * sc).astype(np.float32)
        Q = (X[rng.integers(0, 8000, 60)] + 0.05 * sc * rng.standard_normal((60, 16))).astype(np.float32)
        return X, Q, 4, 6, 8
    if name == "binary-ties":
        # 0/1 coordinates and queries at 0.5: every gap is +-0.5, so all
        # leaves but the home leaves share one eff (131,070 of them)
        rng = np.random.default_rng(21)
        prob = np.linspace(0.1, 0.45, 8)
        X = (rng.random((40_000, 8)) < prob).astype(np.float32)
        Q = np.full((6, 8), 0.5, np.float32)
        return X, Q, 2, 4, 1
    if name == "quant-h16":
        # integers 0..3, queries at half-integers: gaps take few values, so
        # more than 32,768 leaves share the chain maximum at the threshold
        # (bins narrowed into the (tree, head) bits) and groups of hundreds
        # of leaves under one head cross the budget (deeper levels)
        rng = np.random.default_rng(8)
        X = rng.integers(0, 4, (65536, 8)).astype(np.float32)
        Q = (X[rng.integers(0, 65536, 24)] + rng.integers(-1, 2, (24, 8)) + 0.5).astype(np.float32)
        return X, Q, 2, 4, 1
    if name == "deep-h17":
        # depth 17; one coordinate spans 1000x the others, so for query 4
        # a single group of 37,040 leaves under one head (more than the
        # 32,768-key resolution bin) crosses a budget of 60,000
        rng = np.random.default_rng(5)
        X = rng.standard_normal((1 << 17, 32)).astype(np.float32)
        X[:, 0] *= 1000
        Q = (X[rng.integers(0, 1 << 17, 6)] + 0.05 * rng.standard_normal((6, 32))).astype(np.float32)
        return X, Q, 1, 32, 1
    raise KeyError(name)


SEEDS = {"deep-h17": 0, "quant-h16": 3}

_cache = {}


def forests(name, forms=()):
    key = (name, tuple(forms))
    if key not in _cache:
        X, Q, m, t, p = case_data(name)
        seed = SEEDS.get(name, 1234 + len(name))
        Fg = geraf.build_forest(dev(X), m, t, p, seed, forms=forms)
        Fo = oracle.build_forest(X, m, t, p, seed)
        _cache[key] = (X, Q, Fg, Fo, seed)
    return _cache[key]


CASES = [  # (name, k, c, eps)
    ("gauss-10k-128", 1, 256, 0.0),
    ("gauss-10k-128", 10, 700, 0.0),
    ("sphere-20k-1000", 1, 1024, 0.0),
    ("desc-60k-960", 10, 4096, 0.0),
    ("gauss-4k-10000", 10, 2048, 0.0),
    ("ragged-3001-77", 7, 100, 0.0),
    ("ragged-3001-77", 7, 300, 0.5),
    ("multi-d2048", 10, 512, 0.0),
    ("single-leaf", 4, 1, 0.0),
    ("quantised", 5, 150, 0.0),
    # budgets below the number of trees (the sample's lowest bin), windows
    # that miss the threshold, ties at the threshold crossing the budget, and
    # a bin that stays above the collect capacity down into the (tree, entry) bits
    ("quantised", 5, 1, 0.0),
    ("quantised", 5, 37, 0.0),
    ("ragged-3001-77", 7, 3, 0.0),
    ("scales", 10, 20, 0.0),
    ("scales", 10, 200, 0.0),
    ("scales", 10, 900, 0.0),
    ("binary-ties", 3, 50_000, 0.0),
    # Alg. 2's order inside groups of equal chain maximum: full-key bins
    # whose threshold group crosses the budget, and a group larger than the
    # default resolution bin at depth 17
    ("quant-h16", 5, 20_000, 0.0),
    ("quant-h16", 5, 60_000, 0.0),
    ("deep-h17", 5, 60_000, 0.0),
]


@pytest.mark.parametrize("name", sorted({c[0] for c in CASES}))
def test_tree_arrays_bit_exact(name):
    X, Q, Fg, Fo, _ = forests(name)
    T = Fg.export_tree()
    assert_tree_arrays_equal(T, Fo)


@pytest.mark.parametrize("name,k,c,eps", CASES)
def test_opened_leaves_and_candidates_bit_exact(name, k, c, eps):
    X, Q, Fg, Fo, _ = forests(name)
    ref = oracle.search(Fo, X, Q, k, c, eps=eps, candidates=True)
    nq = len(Q)
    lb = np.zeros((nq, Fg.m, Fg.leaf_words), np.uint32)
    cb = np.zeros((nq, (Fg.n + 31) // 32), np.uint32)
    nc = np.zeros(nq, np.int64)
    lb_d = dev(lb)
    cb_d = dev(cb)
    nc_d = dev(nc)
    geraf.query_trace(Fg, dev(Q), c, leaf_bits=lb_d, cand_bits=cb_d, ncand=nc_d, eps=eps)
    torch.cuda.synchronize()
    lb, cb, nc = lb_d.cpu().numpy(), cb_d.cpu().numpy(), nc_d.cpu().numpy()
    for i in range(nq):
        assert leaf_set_from_bits(lb[i]) == set(ref["opened"][i].tolist()), f"query {i}"
        assert np.array_equal(ids_from_bits(cb[i], Fg.n), ref["cand"][i]), f"query {i}"
    assert np.array_equal(nc, ref["ncand"])


@pytest.mark.parametrize("name,c", [("quant-h16", 20_000), ("deep-h17", 60_000), ("scales", 200)])
def test_opened_leaves_independent_of_batch_size(name, c):
    """Small batches walk each tree in finer leaf ranges (more workgroups per
    tree, more histogram slices per query): a query's opened leaves and
    candidates must be the oracle's whatever batch it comes in."""
    X, Q, Fg, Fo, _ = forests(name)
    ref = oracle.search(Fo, X, Q[:6], 5, c, candidates=True)
    for lo, hi in ((0, 1), (1, 3), (0, 6)):
        nq = hi - lo
        lb_d = dev(np.zeros((nq, Fg.m, Fg.leaf_words), np.uint32))
        cb_d = dev(np.zeros((nq, (Fg.n + 31) // 32), np.uint32))
        geraf.query_trace(Fg, dev(Q[lo:hi]), c, leaf_bits=lb_d, cand_bits=cb_d)
        torch.cuda.synchronize()
        lb, cb = lb_d.cpu().numpy(), cb_d.cpu().numpy()
        for i in range(nq):
            assert leaf_set_from_bits(lb[i]) == set(ref["opened"][lo + i].tolist()), f"batch {lo}:{hi} query {i}"
            assert np.array_equal(ids_from_bits(cb[i], Fg.n), ref["cand"][lo + i]), f"batch {lo}:{hi} query {i}"


@pytest.mark.parametrize("name,c", [("desc-60k-960", 4096), ("gauss-10k-128", 700),
                                    ("sphere-20k-1000", 1024), ("ragged-3001-77", 300),
                                    ("quantised", 37), ("scales", 200), ("quant-h16", 20_000)])
def test_tile_path_candidates_bit_exact(name, c):
    """The per-point candidate words the MFMA tile kernel masks its scores
    with, turned back into per-query rows: bit-equal to the oracle's
    candidate sets (the visited array of Sec. 2.3)."""
    X, Q, Fg, Fo, _ = forests(name, forms=("bf16",))
    ref = oracle.search(Fo, X, Q, 1, c, trace=False, candidates=True)
    nq = len(Q)
    cb = np.zeros((nq, (Fg.n + 31) // 32), np.uint32)
    nc = np.zeros(nq, np.int64)
    lb = np.zeros((nq, Fg.m, Fg.leaf_words), np.uint32)
    geraf.query_trace(Fg, Q, c, leaf_bits=lb, cand_bits=cb, ncand=nc, path="tile")
    for i in range(nq):
        assert np.array_equal(ids_from_bits(cb[i], Fg.n), ref["cand"][i]), f"query {i}"
    assert np.array_equal(nc, ref["ncand"])
    # the same selection as the row path's trace
    lb_rows = np.zeros_like(lb)
    geraf.query_trace(Fg, Q, c, leaf_bits=lb_rows)
    assert np.array_equal(lb, lb_rows)


@pytest.mark.parametrize("name,k,c,eps", CASES)
def test_fp32_neighbours(name, k, c, eps):
    X, Q, Fg, Fo, _ = forests(name)
    ref = oracle.search(Fo, X, Q, k, c, eps=eps, trace=False, candidates=True)
    ids = torch.full((len(Q), k), -7, dtype=torch.int32, device="cuda:0")
    dd = torch.full((len(Q), k), -7.0, dtype=torch.float32, device="cuda:0")
    geraf.query(Fg, dev(Q), k, c, ids, dd, eps=eps)
    torch.cuda.synchronize()
    check_knn(ids.cpu().numpy(), dd.cpu().numpy(), ref["ids"], ref["dists"], X=X, Q=Q,
              cand=ref["cand"])


def test_host_buffers_match_device_buffers():
    X, Q, Fg, Fo, _ = forests("ragged-3001-77")
    ids_h = np.zeros((len(Q), 7), np.int32)
    dd_h = np.zeros((len(Q), 7), np.float32)
    geraf.query(Fg, Q, 7, 100, ids_h, dd_h)
    ids = torch.zeros((len(Q), 7), dtype=torch.int32, device="cuda:0")
    dd = torch.zeros((len(Q), 7), dtype=torch.float32, device="cuda:0")
    geraf.query(Fg, dev(Q), 7, 100, ids, dd)
    assert np.array_equal(ids.cpu().numpy(), ids_h)
    assert np.array_equal(dd.cpu().numpy(), dd_h)


def test_per_query_budgets():
    X, Q, Fg, Fo, _ = forests("gauss-10k-128")
    rng = np.random.default_rng(3)
    cpq = rng.integers(1, 900, len(Q)).astype(np.int32)
    lb = np.zeros((len(Q), Fg.m, Fg.leaf_words), np.uint32)
    geraf.query_trace(Fg, Q, 1, leaf_bits=lb, checks_per_query=cpq)
    ids = np.zeros((len(Q), 3), np.int32)
    dd = np.zeros((len(Q), 3), np.float32)
    geraf.query(Fg, Q, 3, 1, ids, dd, checks_per_query=dev(cpq))
    for i in range(len(Q)):
        ref = oracle.search(Fo, X, Q[i:i + 1], 3, int(cpq[i]))
        assert leaf_set_from_bits(lb[i]) == set(ref["opened"][0].tolist())
        check_knn(ids[i:i + 1], dd[i:i + 1], ref["ids"], ref["dists"], X=X, Q=Q[i:i + 1])


def test_few_queries_left_for_radix_passes():
    """Budgets of one or two leaves (below what the sample walk can place)
    send a handful of queries to radix passes while the rest take the
    window: those passes run split finer than the tree slices, adding into
    the slice histograms."""
    X, Q, Fg, Fo, _ = forests("gauss-10k-128")
    cpq = np.full(len(Q), 256, np.int32)
    cpq[[0, 17, 50, 99]] = [1, 2, 1, 2]
    lb = np.zeros((len(Q), Fg.m, Fg.leaf_words), np.uint32)
    geraf.query_trace(Fg, Q, 1, leaf_bits=lb, checks_per_query=cpq)
    for c in np.unique(cpq):
        sel = np.nonzero(cpq == c)[0]
        ref = oracle.search(Fo, X, np.ascontiguousarray(Q[sel]), 1, int(c))
        for j, i in enumerate(sel):
            assert leaf_set_from_bits(lb[i]) == set(ref["opened"][j].tolist()), f"query {i}"


def test_exhaustive_budget_is_brute_force():
    from oracle import bruteforce as bf
    X, Q, Fg, Fo, _ = forests("ragged-3001-77")
    total = Fg.m << Fg.H
    ids = np.zeros((len(Q), 9), np.int32)
    dd = np.zeros((len(Q), 9), np.float32)
    geraf.query(Fg, Q, 9, total + 5, ids, dd)
    ei, ed = bf.knn_exact(X, Q, 9)
    check_knn(ids, dd, ei, ed, X=X, Q=Q)


def test_fewer_candidates_than_k_pads():
    X, Q, Fg, Fo, _ = forests("ragged-3001-77")
    ids = np.zeros((len(Q), 30), np.int32)
    dd = np.zeros((len(Q), 30), np.float32)
    geraf.query(Fg, Q, 30, 1, ids, dd)          # one leaf of <= 5 points
    ref = oracle.search(Fo, X, Q, 30, 1, trace=False)
    check_knn(ids, dd, ref["ids"], ref["dists"], X=X, Q=Q)
    assert np.all(ids[:, 5:] == -1) and np.all(np.isinf(dd[:, 5:]))


def test_empty_query_batch():
    X, Q, Fg, Fo, _ = forests("ragged-3001-77")
    geraf.query(Fg, Q[:0], 3, 10, np.zeros((0, 3), np.int32), np.zeros((0, 3), np.float32))


def test_non_finite_query_rejected_without_output():
    X, Q, Fg, Fo, _ = forests("ragged-3001-77")
    Qb = Q[:4].copy()
    Qb[2, 5] = np.nan
    ids = np.full((4, 3), 77, np.int32)
    dd = np.full((4, 3), 77.0, np.float32)
    with pytest.raises(geraf.GerafError) as e:
        geraf.query(Fg, Qb, 3, 10, ids, dd)
    assert e.value.status == geraf.GF_EINVAL
    assert np.all(ids == 77) and np.all(dd == 77.0)


def test_repeat_runs_bit_identical():
    X, Q, Fg, Fo, _ = forests("desc-60k-960", forms=("bf16",))
    outs = []
    for _ in range(2):
        ids = torch.zeros((len(Q), 10), dtype=torch.int32, device="cuda:0")
        dd = torch.zeros((len(Q), 10), dtype=torch.float32, device="cuda:0")
        geraf.query(Fg, dev(Q), 10, 4096, ids, dd, form="bf16")
        outs.append((ids.cpu().numpy(), dd.cpu().numpy()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


@pytest.mark.parametrize("name,form,k,c", [("desc-60k-960", "bf16", 10, 4096),
                                           ("multi-d2048", "bf16", 10, 512),
                                           ("gauss-10k-128", "bf16", 10, 700),
                                           ("gauss-4k-10000", "fp8", 10, 2048),
                                           ("gauss-4k-10000", "bf16", 10, 2048),
                                           ("ragged-3001-77", "fp8", 7, 300),
                                           ("sphere-20k-1000", "fp8", 5, 1024)])
def test_reduced_precision_forms(name, form, k, c):
    """Selection in BF16 / FP8, re-rank in FP32: every returned distance is
    exact (1e-5), and the result agrees with the oracle's top-k (recall
    stated; the floor below is what these seeded cases reach)."""
    X, Q, Fg, Fo, _ = forests(name, forms=(form,))
    ref = oracle.search(Fo, X, Q, k, c, trace=False, candidates=True)
    ids = np.zeros((len(Q), k), np.int32)
    dd = np.zeros((len(Q), k), np.float32)
    geraf.query(Fg, Q, k, c, ids, dd, form=form)
    hits = 0
    for i in range(len(Q)):
        got = ids[i][ids[i] >= 0]
        assert np.isin(got, ref["cand"][i]).all(), f"query {i}: a returned id is not a candidate"
        for j, gid in enumerate(got.tolist()):
            diff = X[gid].astype(np.float64) - Q[i].astype(np.float64)
            true_d = float(diff @ diff)
            assert abs(dd[i][j] - true_d) <= 1e-5 * true_d
        hits += len(set(got.tolist()) & set(ref["ids"][i][ref["ids"][i] >= 0].tolist()))
    recall = hits / max(1, int((ref["ids"] >= 0).sum()))
    print(f"{name} {form}: recall vs FP64 oracle = {recall:.4f}")
    assert recall >= 0.98


@pytest.mark.parametrize("form", ["fp32", "bf16"])
def test_wide_rows_query_in_lds_matches_global(form, monkeypatch):
    """Rows wider than the register tiles (d = 10,000): the scan reads the
    query from a copy in LDS, or from global memory where that copy would
    not fit beside the bitmap.  Same chunks, same order: identical output."""
    X, Q, Fg, Fo, _ = forests("gauss-4k-10000", forms=() if form == "fp32" else (form,))
    outs = []
    for where in ("lds", "global"):
        if where == "global":
            monkeypatch.setenv("GF_SCAN_WIDE_QUERY", "global")
        ids = np.zeros((len(Q), 10), np.int32)
        dd = np.zeros((len(Q), 10), np.float32)
        geraf.query(Fg, Q, 10, 2048, ids, dd, form=form)
        outs.append((ids, dd))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])


def test_fp8_hardware_decode_matches_definition():
    hw, sw, _ = geraf.fp8_tables()
    codes = np.arange(256)
    finite = (codes & 0x7F) != 0x7F
    assert np.array_equal(hw[finite], sw[finite])
    assert sw[0x7E] == 448.0 and sw[0x08] == 2.0 ** -6 and sw[0x01] == 2.0 ** -9
    assert sw[0x38] == 1.0 and sw[0xB8] == -1.0


def test_fp8_encoder_is_round_to_nearest_even_saturating():
    # every finite e4m3 value, from the definition
    vals = []
    for c in range(0x7F):
        E, mnt = c >> 3, c & 7
        vals.append(mnt * 2.0 ** -9 if E == 0 else (1 + mnt / 8) * 2.0 ** (E - 7))
    vals = np.array(vals)
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(4000) * 50, rng.standard_normal(2000) * 0.01,
                        vals, (vals[1:] + vals[:-1]) / 2, [500.0, -1e6, 0.0, 448.0, 449.0]])
    x = x.astype(np.float32)
    _, _, enc = geraf.fp8_tables(x)
    for xi, ci in zip(x.tolist(), enc.tolist()):
        a = abs(xi)
        if a >= 448:
            exp_c = 0x7E
        else:
            dist = np.abs(vals - a)
            best = np.nonzero(dist == dist.min())[0]
            exp_c = int(best[0]) if len(best) == 1 else int(best[(best & 1) == 0][0])
        if xi < 0 or (xi == 0 and np.signbit(np.float32(xi))):
            exp_c |= 0x80
        assert ci == exp_c, (xi, ci, exp_c)


@pytest.fixture
def scan_path(monkeypatch):
    def set_path(p):
        monkeypatch.setenv("GF_SCAN_PATH", p)
    return set_path


@pytest.mark.parametrize("name,k,c,nq", [("desc-60k-960", 10, 4096, None),
                                         ("gauss-10k-128", 10, 700, None),
                                         ("sphere-20k-1000", 5, 1024, None),
                                         ("ragged-3001-77", 7, 300, None),
                                         ("desc-600q", 10, 2048, 600)])
def test_tile_path_bf16(name, k, c, nq, scan_path):
    """The MFMA tile path (scores of 128-query blocks, masked by each query's
    visited bitmap) against the oracle and against the per-query BF16 path."""
    if name == "desc-600q":
        X, _, _ = W.descriptor(60_000, 960, 1, 0.02, 2)
        rng = np.random.default_rng(11)
        Q = (X[rng.integers(0, 60_000, nq)] + 0.02 * rng.standard_normal((nq, 960))).astype(np.float32)
        key = ("desc-600q", ("bf16",))
        if key not in _cache:
            Fg = geraf.build_forest(dev(X), 16, 5, 32, 77, forms=("bf16",))
            Fo = oracle.build_forest(X, 16, 5, 32, 77)
            _cache[key] = (X, Q, Fg, Fo, 77)
        X, Q, Fg, Fo, _ = _cache[key]
    else:
        X, Q, Fg, Fo, _ = forests(name, forms=("bf16",))
    ref = oracle.search(Fo, X, Q, k, c, trace=False, candidates=True)
    out = {}
    for path in ("tile", "rows"):
        scan_path(path)
        ids = np.zeros((len(Q), k), np.int32)
        dd = np.zeros((len(Q), k), np.float32)
        geraf.query(Fg, Q, k, c, ids, dd, form="bf16")
        out[path] = (ids, dd)
    ids, dd = out["tile"]
    hits, agree = 0, 0
    for i in range(len(Q)):
        got = ids[i][ids[i] >= 0]
        assert np.isin(got, ref["cand"][i]).all(), f"query {i}: a returned id is not a candidate"
        for j, gid in enumerate(got.tolist()):
            diff = X[gid].astype(np.float64) - Q[i].astype(np.float64)
            true_d = float(diff @ diff)
            assert abs(dd[i][j] - true_d) <= 1e-5 * true_d
        assert np.all(np.diff(dd[i][ids[i] >= 0]) >= 0)
        hits += len(set(got.tolist()) & set(ref["ids"][i][ref["ids"][i] >= 0].tolist()))
        agree += len(set(got.tolist()) & set(out["rows"][0][i][out["rows"][0][i] >= 0].tolist()))
    n_ref = max(1, int((ref["ids"] >= 0).sum()))
    recall, agreement = hits / n_ref, agree / n_ref
    print(f"{name} tile path: recall vs oracle {recall:.4f}, agreement with rows path {agreement:.4f}")
    assert np.array_equal(ids >= 0, ref["ids"] >= 0)
    assert recall >= 0.98 and agreement >= 0.99


@pytest.mark.parametrize("name,k,c", [("gauss-4k-10000", 10, 2048), ("ragged-3001-77", 7, 300),
                                      ("sphere-20k-1000", 5, 1024), ("quantised", 5, 150)])
def test_tile_path_fp8(name, k, c, scan_path):
    """The FP8 tile path (dense FP8 MFMA scores of 128-query blocks, kept for
    each query's candidates) against the oracle and the FP8 row path: every
    returned id a candidate, every distance exact to 1e-5, recall stated."""
    X, Q, Fg, Fo, _ = forests(name, forms=("fp8",))
    ref = oracle.search(Fo, X, Q, k, c, trace=False, candidates=True)
    out = {}
    for path in ("tile", "rows"):
        scan_path(path)
        ids = np.zeros((len(Q), k), np.int32)
        dd = np.zeros((len(Q), k), np.float32)
        geraf.query(Fg, Q, k, c, ids, dd, form="fp8")
        assert geraf.last_query_timing()["path"] == path
        out[path] = (ids, dd)
    ids, dd = out["tile"]
    hits = agree = 0
    for i in range(len(Q)):
        got = ids[i][ids[i] >= 0]
        assert np.isin(got, ref["cand"][i]).all(), f"query {i}: a returned id is not a candidate"
        for j, gid in enumerate(got.tolist()):
            diff = X[gid].astype(np.float64) - Q[i].astype(np.float64)
            true_d = float(diff @ diff)
            assert abs(dd[i][j] - true_d) <= 1e-5 * true_d
        assert np.all(np.diff(dd[i][ids[i] >= 0]) >= 0)
        hits += len(set(got.tolist()) & set(ref["ids"][i][ref["ids"][i] >= 0].tolist()))
        agree += len(set(got.tolist()) & set(out["rows"][0][i][out["rows"][0][i] >= 0].tolist()))
    n_ref = max(1, int((ref["ids"] >= 0).sum()))
    recall, agreement = hits / n_ref, agree / n_ref
    print(f"{name} fp8 tile path: recall vs oracle {recall:.4f}, agreement with rows path {agreement:.4f}")
    assert np.array_equal(ids >= 0, ref["ids"] >= 0)
    assert recall >= 0.97 and agreement >= 0.97


@pytest.mark.parametrize("name,form,k,c", [("gauss-10k-128", "fp32", 10, 700),
                                           ("ragged-3001-77", "fp32", 7, 300),
                                           ("desc-60k-960", "bf16", 10, 4096),
                                           ("gauss-4k-10000", "fp8", 10, 2048),
                                           ("gauss-4k-10000", "fp32", 10, 2048)])
def test_sliced_row_scan_equals_one_workgroup_per_query(name, form, k, c, monkeypatch):
    """Small batches cut each query's id range into slices (one workgroup
    each) whose lists are merged: the result must be bit-equal to one
    workgroup per query, for the default slice count and a forced odd one."""
    X, Q, Fg, Fo, _ = forests(name, forms=() if form == "fp32" else (form,))
    monkeypatch.setenv("GF_SCAN_PATH", "rows")
    out = []
    for slices in ("1", None, "7"):
        if slices is None:
            monkeypatch.delenv("GF_SCAN_SLICES", raising=False)
        else:
            monkeypatch.setenv("GF_SCAN_SLICES", slices)
        ids = np.zeros((len(Q), k), np.int32)
        dd = np.zeros((len(Q), k), np.float32)
        geraf.query(Fg, Q, k, c, ids, dd, form=form)
        out.append((ids, dd))
    for ids, dd in out[1:]:
        assert np.array_equal(ids, out[0][0]) and np.array_equal(dd, out[0][1])


def test_row_scan_bitmap_prepass_boundary(monkeypatch):
    """Sliced row scans of batches of up to 64 queries read a candidate bitmap
    built once per query; larger batches expand the opened leaves in every
    slice.  The first 64 queries' results agree bit for bit across that
    boundary, and a single query's with both."""
    X, Q, Fg, Fo, _ = forests("desc-60k-960", forms=("bf16",))
    monkeypatch.setenv("GF_SCAN_PATH", "rows")
    monkeypatch.delenv("GF_SCAN_SLICES", raising=False)
    res = {}
    for nq in (1, 64, 65):
        ids = np.zeros((nq, 10), np.int32)
        dd = np.zeros((nq, 10), np.float32)
        geraf.query(Fg, Q[:nq], 10, 4096, ids, dd, form="bf16")
        res[nq] = (ids, dd)
    assert np.array_equal(res[64][0], res[65][0][:64]) and np.array_equal(res[64][1], res[65][1][:64])
    assert np.array_equal(res[1][0], res[65][0][:1]) and np.array_equal(res[1][1], res[65][1][:1])


@pytest.mark.parametrize("k", [1, 5, 10, 12])
def test_tile_path_bf16_independent_of_split_count(k, monkeypatch):
    """The BF16 tile path's lists are exact: the kk best scores of each
    query over its candidates do not depend on how the points are split
    among workgroups (one split: no shared bound; two or three: the rank
    bound as well; four: the worst-entry bound alone), so the neighbours and
    distances are bit-identical for every split count, at every list
    capacity kk = 4 k (k = 12 fills all 48 positions)."""
    X, Q, Fg, Fo, _ = forests("desc-60k-960", forms=("bf16",))
    monkeypatch.setenv("GF_SCAN_PATH", "tile")
    out = []
    for ns in (1, 2, 3, 4):
        monkeypatch.setenv("GF_TILE_SPLITS", str(ns))
        ids = np.zeros((len(Q), k), np.int32)
        dd = np.zeros((len(Q), k), np.float32)
        geraf.query(Fg, Q, k, 4096, ids, dd, form="bf16")
        assert geraf.last_query_timing()["path"] == "tile"
        out.append((ids, dd))
    for ns, (ids, dd) in zip((2, 3, 4), out[1:]):
        assert np.array_equal(ids, out[0][0]), f"{ns} splits"
        assert np.array_equal(dd.view(np.uint32), out[0][1].view(np.uint32)), f"{ns} splits"
    ref = oracle.search(Fo, X, Q, k, 4096, trace=False, candidates=True)
    for i in range(len(Q)):
        got = out[0][0][i][out[0][0][i] >= 0]
        assert np.isin(got, ref["cand"][i]).all()
