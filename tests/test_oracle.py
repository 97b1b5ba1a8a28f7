"""CPU pins for the FP64 oracle (no GPU).

Each test checks the oracle against something other than itself: published
RNG outputs, a hand-worked example, numpy's textbook routines, closed forms of
the split and search rules, brute force, and structural invariants.  A
plausible mistake in the oracle (a dropped term, a flipped comparison, a wrong
child index or key) fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import bruteforce as bf

GOLD = os.path.join(os.path.dirname(__file__), "golden")
M64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def py_mix(z):
    """splitmix64's mixing function, as published (used as a helper below;
    the published outputs in golden/splitmix64.json pin it)."""
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def py_draw(seed, stream, tree, idx):
    h = py_mix((seed + GAMMA) & M64)
    h = py_mix(((h ^ stream) + GAMMA) & M64)
    h = py_mix(((h ^ tree) + GAMMA) & M64)
    return py_mix(((h ^ idx) + GAMMA) & M64)


# --------------------------------------------------------------------- RNG

def test_splitmix64_published_outputs():
    g = json.load(open(os.path.join(GOLD, "splitmix64.json")))
    for i, hx in enumerate(g["state0_outputs_hex"]):
        assert oracle.splitmix64((i * GAMMA) & M64) == int(hx, 16)
        assert py_mix(((i + 1) * GAMMA) & M64) == int(hx, 16)


def test_draw_is_keyed_composition():
    rng = np.random.default_rng(7)
    for _ in range(200):
        s, a, b, c = (int(x) for x in rng.integers(0, 2**63, 4))
        assert oracle.draw(s, a % 5, b % 300, c) == py_draw(s, a % 5, b % 300, c)


# --------------------------------------------------- variance and top dims

def test_variance_matches_numpy():
    rng = np.random.default_rng(1)
    X = (rng.standard_normal((777, 19)) * rng.uniform(0.1, 5, 19) + 3.0).astype(np.float32)
    V = oracle.variance(X)
    ref = np.var(X.astype(np.float64), axis=0, ddof=1)
    assert np.allclose(V, ref, rtol=1e-12, atol=0)


def test_variance_fewer_than_two_points_is_zero():
    assert np.all(oracle.variance(np.ones((1, 4), np.float32) * 3) == 0)


def test_top_dims_ties_go_to_lower_index_and_sorted():
    V = np.array([1.0, 5.0, 3.0, 5.0, 2.0, 3.0])
    assert oracle.top_dims(V, 1).tolist() == [1]
    assert oracle.top_dims(V, 2).tolist() == [1, 3]
    assert oracle.top_dims(V, 3).tolist() == [1, 2, 3]
    assert oracle.top_dims(V, 4).tolist() == [1, 2, 3, 5]
    assert oracle.top_dims(V, 6).tolist() == [0, 1, 2, 3, 4, 5]


# ------------------------------------------------------------------ depth

def _near_tie_data(kind):
    rng = np.random.default_rng(44)
    X = rng.standard_normal((500, 6)).astype(np.float32)
    X[:, 0] *= 3.0
    X[:, 1] *= 2.0                                  # ranks 1 and 2 well separated
    if kind == "duplicate":
        X[:, 3] = X[:, 2] * np.float32(1.5)
        X[:, 2] = X[:, 3]                           # ranks 3 and 4 equal exactly
    elif kind == "permuted":
        X[:, 2] *= 1.5
        X[:, 3] = X[::-1, 2]                        # same values, other order: equal up to rounding
    elif kind == "one-ulp":
        X[:, 2] *= 1.5
        X[:, 3] = X[:, 2]
        X[7, 3] = np.nextafter(X[7, 3], np.float32(np.inf))   # ~3e-11 relative: resolvable
    elif kind == "zero-columns":
        X[:, 3:] = 0.0                              # ranks 4.. all exactly 0
    return X


@pytest.mark.parametrize("kind,t,ambiguous", [("duplicate", 3, True), ("permuted", 3, True),
                                              ("one-ulp", 3, False), ("duplicate", 2, False),
                                              ("duplicate", 4, False), ("zero-columns", 4, False),
                                              ("separated", 3, False)])
def test_build_refuses_a_near_tie_at_rank_t(kind, t, ambiguous):
    X = _near_tie_data(kind)
    assert oracle.dims_ambiguous(X, t) == ambiguous
    if ambiguous:
        with pytest.raises(oracle.NearTieError):
            oracle.build_forest(X, 2, t, 8, 1)
    else:
        F = oracle.build_forest(X, 2, t, 8, 1)
        V = np.var(X.astype(np.float64), axis=0, ddof=1)
        assert set(F["D"].tolist()) == set(np.argsort(-V, kind="stable")[:t].tolist())


def test_build_near_tie_guard_exempts_single_point():
    X = np.zeros((1, 5), np.float32)
    F = oracle.build_forest(X, 2, 2, 1, 3)            # V = 0 by definition: D = {0, 1}
    assert F["D"].tolist() == [0, 1]


@pytest.mark.parametrize("n,p,H", [(10_000, 8, 11), (100_000, 16, 13), (1_000_000, 32, 15),
                                   (200_000, 16, 14), (5, 5, 0), (5, 9, 0), (6, 5, 1),
                                   (1, 1, 0), (2, 1, 1), (9, 2, 3), (8, 2, 2), (17, 4, 3)])
def test_depth_closed_form(n, p, H):
    assert oracle.depth(n, p) == H
    assert math.ceil(n / 2**H) <= p and (H == 0 or math.ceil(n / 2**(H - 1)) > p)


# ------------------------------------------------------------------- build

def node_sizes(n, H):
    """Point count of every node, level by level (left floor, right ceil)."""
    sizes = [n]
    for _ in range(H):
        sizes = [s for z in sizes for s in (z // 2, z - z // 2)]
    return sizes


def subtree_points(F, tree, v):
    """Point ids in the subtree of node v (from the leaf ranges)."""
    H = F["H"]
    lo, hi = v, v
    while lo < (1 << H) - 1:
        lo, hi = 2 * lo + 1, 2 * hi + 2
    L0, L1 = lo - ((1 << H) - 1), hi - ((1 << H) - 1)
    off = F["leaf_off"]
    return F["perm"][tree, off[L0]:off[L1 + 1]]


def check_build_invariants(F, X):
    n, d = X.shape
    m, t, H = F["m"], F["t"], F["H"]
    D = F["D"]
    # D = the t largest sample variances (numpy), as a set
    V = np.var(X.astype(np.float64), axis=0, ddof=1)
    order = sorted(range(d), key=lambda j: (-V[j], j))
    assert sorted(order[:t]) == D.tolist()
    # leaf offsets follow the floor/ceil size recursion; every leaf <= p
    sizes = node_sizes(n, H)
    assert F["leaf_off"].tolist() == [0] + np.cumsum(sizes).tolist()
    assert max(sizes) <= F["p"]
    keys = None
    for tr in range(m):
        perm = F["perm"][tr]
        assert np.array_equal(np.sort(perm), np.arange(n))
        for j in range(1 << H):
            seg = perm[F["leaf_off"][j]:F["leaf_off"][j + 1]]
            assert np.all(np.diff(seg.astype(np.int64)) > 0)       # ascending ids
        keys = np.array([py_draw(F["seed"], 2, tr, i) for i in range(n)], dtype=np.uint64)
        for v in range((1 << H) - 1):
            s = int(F["split_dim"][tr, v])
            assert s == int(D[py_draw(F["seed"], 1, tr, v) % t])
            pts = subtree_points(F, tr, v)
            left = subtree_points(F, tr, 2 * v + 1)
            right = subtree_points(F, tr, 2 * v + 2)
            assert len(left) == len(pts) // 2
            # closed form of the median split: the left child holds the
            # floor(|P|/2) smallest points under (x_s, tie key, id)
            srt = sorted(pts.tolist(), key=lambda i: (float(X[i, s]), int(keys[i]), i))
            assert set(srt[:len(pts) // 2]) == set(left.tolist())
            val = F["split_val"][tr, v]
            assert val == X[srt[len(pts) // 2], s]
            if len(left):
                assert X[left, s].max() <= val
            assert X[right, s].min() == val


@pytest.mark.parametrize("n,d,m,t,p,seed", [(300, 7, 3, 3, 5, 11), (257, 12, 2, 5, 4, 3),
                                            (64, 4, 2, 4, 1, 0)])
def test_build_invariants_continuous(n, d, m, t, p, seed):
    X = np.random.default_rng(seed).standard_normal((n, d)).astype(np.float32)
    X[:, 1] *= 3
    F = oracle.build_forest(X, m, t, p, seed)
    check_build_invariants(F, X)


def test_build_invariants_quantised_ties():
    # SIFT-like byte values: many equal coordinates, so the tie key decides
    rng = np.random.default_rng(5)
    X = rng.integers(0, 4, (200, 6)).astype(np.float32)
    X[:, 2] *= 3
    F = oracle.build_forest(X, 3, 3, 3, 99)
    check_build_invariants(F, X)
    # shuffling: different trees split the tied values differently
    assert not np.array_equal(F["perm"][0], F["perm"][1])


def test_build_t1_contiguous_rank_blocks():
    # t = 1: every split is on D[0], so each tree's leaves are contiguous
    # blocks of the order by (x_D0, tie key, id), block sizes from leaf_off
    rng = np.random.default_rng(8)
    X = rng.standard_normal((500, 5)).astype(np.float32)
    X[:, 3] *= 4
    X[::7, 3] = 0.5                                   # plus ties
    F = oracle.build_forest(X, 3, 1, 6, 21)
    assert F["D"].tolist() == [3]
    for tr in range(3):
        keys = [py_draw(21, 2, tr, i) for i in range(500)]
        srt = sorted(range(500), key=lambda i: (float(X[i, 3]), keys[i], i))
        off = F["leaf_off"]
        for j in range(len(off) - 1):
            assert sorted(srt[off[j]:off[j + 1]]) == F["perm"][tr, off[j]:off[j + 1]].tolist()


def test_build_hand_worked_example():
    g = json.load(open(os.path.join(GOLD, "tiny_2d.json")))
    X = np.array(g["X"], dtype=np.float32)
    F = oracle.build_forest(X, g["m"], g["t"], g["p"], g["seed"])
    tr = g["tree"]
    assert F["H"] == tr["H"]
    assert F["D"].tolist() == tr["D"]
    assert F["split_dim"][0].tolist() == tr["split_dim"]
    assert F["split_val"][0].tolist() == tr["split_val"]
    assert F["leaf_off"].tolist() == tr["leaf_off"]
    assert F["perm"][0].tolist() == tr["perm"]


# ------------------------------------------------------------------ search

def _inf(v):
    return math.inf if v == "inf" else float(v)


def search_hand_example(eff_key):
    g = json.load(open(os.path.join(GOLD, "tiny_2d.json")))
    X = np.array(g["X"], dtype=np.float32)
    q = np.array([g["q"]], dtype=np.float32)
    F = oracle.build_forest(X, g["m"], g["t"], g["p"], g["seed"])
    for c in range(1, 5):
        r = oracle.search(F, X, q, 3, c, eff_key=eff_key)
        assert (r["opened"][0] & 0xFFFFFF).tolist() == g["pops"]["leaves"][:c]
        assert r["opened_key"][0].tolist() == g["pops"]["keys"][:c]
        exp = g["k3_by_c"][str(c)]
        assert r["ids"][0].tolist() == exp["ids"]
        assert r["dists"][0].tolist() == [_inf(x) for x in exp["dists"]]


def test_search_hand_worked_example():
    search_hand_example(False)


def test_search_hand_worked_example_max_key_variant():
    # one split dimension: the gaps grow along every chain, so the diagnostic
    # max-key variant pops the same sequence
    search_hand_example(True)


def _golden_forest(name):
    g = json.load(open(os.path.join(GOLD, name)))
    X = np.array(g["X"], dtype=np.float32)
    q = np.array([g["q"]], dtype=np.float32)
    F = oracle.build_forest(X, g["m"], g["t"], g["p"], g["seed"])
    tr = g["tree"]
    assert F["H"] == tr["H"] and F["D"].tolist() == tr["D"]
    for i in range(g["m"]):
        assert F["split_dim"][i].tolist() == tr["split_dim"]
        assert F["split_val"][i].tolist() == tr["split_val"]
        assert F["perm"][i].tolist() == tr["perm"]
    assert F["leaf_off"].tolist() == tr["leaf_off"]
    return g, X, q, F


def test_search_far_gap_below_its_entry_key():
    """Alg. 2 keys a left-behind child by its own |gap|, which can be below the
    key of the entry whose descent pushed it; the max-key variant would pop
    another leaf third and return another best 3 at c = 3."""
    g, X, q, F = _golden_forest("gap_below_entry_2d.json")
    B = len(g["pops"]["leaves"])
    r = oracle.search(F, X, q, 3, B)
    assert (r["opened"][0] & 0xFFFFFF).tolist() == g["pops"]["leaves"]
    assert r["opened_key"][0].tolist() == g["pops"]["keys"]
    for c, exp in g["k3_by_c"].items():
        r = oracle.search(F, X, q, 3, int(c))
        assert r["ids"][0].tolist() == exp["ids"], c
        assert r["dists"][0].tolist() == [_inf(x) for x in exp["dists"]], c
    v = oracle.search(F, X, q, 3, B, eff_key=True)
    assert (v["opened"][0] & 0xFFFFFF).tolist() == g["pops_max_key_variant"]["leaves"]
    assert v["opened_key"][0].tolist() == g["pops_max_key_variant"]["keys"]
    v3 = oracle.search(F, X, q, 3, 3, eff_key=True)
    assert v3["ids"][0].tolist() == g["k3_c3_max_key_variant"]["ids"]


def test_search_zero_gap_descends_right_and_ties_go_to_lower_tree():
    g, X, q, F = _golden_forest("zero_gap_two_trees.json")
    B = len(g["pops"]["leaves"])
    r = oracle.search(F, X, q, 2, B, candidates=True)
    assert (r["opened"][0] >> 24).tolist() == g["pops"]["trees"]
    assert (r["opened"][0] & 0xFFFFFF).tolist() == g["pops"]["leaves"]
    assert r["opened_key"][0].tolist() == g["pops"]["keys"]
    for c, exp in g["k2_by_c"].items():
        rc = oracle.search(F, X, q, 2, int(c))
        assert rc["ids"][0].tolist() == exp["ids"], c
        assert rc["dists"][0].tolist() == exp["dists"], c
    for c, nc in g["ncand_by_c"].items():
        rc = oracle.search(F, X, q, 1, int(c), candidates=True)
        assert int(rc["ncand"][0]) == nc, c


def _leaf_chains(F, q):
    """Every leaf's chain of (|gap|, tree, entry node) from an independent
    top-down traversal: the root contributes (0, tree, 0); each node where
    the leaf lies on the far side contributes (|q_s - v| as float32, tree,
    far child).  Yields (tree, leaf, chain)."""
    H, m = F["H"], F["m"]
    nint = (1 << H) - 1
    for tr in range(m):
        stack = [(0, [(0.0, tr, 0)])]
        while stack:
            v, chain = stack.pop()
            if v >= nint:
                yield tr, v - nint, chain
                continue
            s = F["split_dim"][tr, v]
            g = np.float32(q[s]) - np.float32(F["split_val"][tr, v])
            near, far = (2 * v + 1, 2 * v + 2) if g < 0 else (2 * v + 2, 2 * v + 1)
            stack.append((near, chain))
            stack.append((far, chain + [(float(abs(g)), tr, far)]))


def static_leaf_order_gap(F, q):
    """Static characterisation of Alg. 2's pop order.  A leaf's key is the
    subsequence of its chain made of the entries strictly larger than every
    entry after them (the strictly decreasing suffix maxima), compared
    lexicographically by (|gap|, tree, node), a prefix first.  Reason: pops
    come in non-decreasing order of the chain maximum; among equal maxima,
    the entries at that value head groups that the queue empties one after
    the other, in (tree, node) order (a child head has a larger node index);
    inside a group the same argument applies to the chain below its head.
    Returns the leaf codes in that order and each one's last chain key (the
    key it is popped with)."""
    items = []
    for tr, leaf, chain in _leaf_chains(F, q):
        seq, best = [], -1.0
        for e in reversed(chain):
            if e[0] > best:
                seq.append(e)
                best = e[0]
        seq.reverse()
        items.append((seq, (tr << 24) | leaf, chain[-1][0]))
    items.sort(key=lambda it: it[0])
    return [it[1] for it in items], [it[2] for it in items]


def static_leaf_order_eff(F, q):
    """The diagnostic max-key variant: every leaf's (eff, tree, entry), eff
    the largest |gap| on its chain, entry its deepest far child."""
    items = []
    for tr, leaf, chain in _leaf_chains(F, q):
        eff = max(e[0] for e in chain)
        items.append((eff, tr, chain[-1][2], (tr << 24) | leaf))
    items.sort()
    return [it[3] for it in items], [it[0] for it in items]


SEARCH_CASES = [(2000, 24, 4, 5, 8, 100, 0, "gauss"),
                (1000, 16, 3, 2, 3, 333, 1, "gauss"),
                (333, 8, 5, 8, 2, 50, 2, "gauss"),
                (1500, 12, 3, 4, 4, 120, 3, "quantised"),
                (2400, 6, 2, 4, 1, 900, 4, "binary")]


def _search_case_data(n, d, seed, kind):
    rng = np.random.default_rng(seed)
    if kind == "gauss":
        X = rng.standard_normal((n, d)).astype(np.float32)
        Q = (X[rng.integers(0, n, 12)] + 0.1 * rng.standard_normal((12, d))).astype(np.float32)
    elif kind == "quantised":
        # integer coordinates: equal gaps at different nodes and trees
        X = rng.integers(0, 4, (n, d)).astype(np.float32)
        Q = (X[rng.integers(0, n, 12)] + rng.integers(-1, 2, (12, d))).astype(np.float32)
    else:
        # 0/1 coordinates, queries at 0.5: every gap is 0.5
        X = (rng.random((n, d)) < np.linspace(0.1, 0.45, d)).astype(np.float32)
        Q = np.full((4, d), 0.5, np.float32)
    return X, Q


@pytest.mark.parametrize("n,d,m,t,p,c,seed,kind", SEARCH_CASES)
def test_search_pop_order_equals_static_leaf_ranking(n, d, m, t, p, c, seed, kind):
    X, Q = _search_case_data(n, d, seed, kind)
    F = oracle.build_forest(X, m, t, p, seed)
    r = oracle.search(F, X, Q, 3, c)
    for i in range(len(Q)):
        codes, keys = static_leaf_order_gap(F, Q[i])
        assert r["opened"][i].tolist() == codes[:r["B"]]
        assert r["opened_key"][i].tolist() == keys[:r["B"]]


@pytest.mark.parametrize("n,d,m,t,p,c,seed,kind", SEARCH_CASES)
def test_search_max_key_variant_equals_its_static_ranking(n, d, m, t, p, c, seed, kind):
    X, Q = _search_case_data(n, d, seed, kind)
    F = oracle.build_forest(X, m, t, p, seed)
    r = oracle.search(F, X, Q, 3, c, eff_key=True)
    for i in range(len(Q)):
        codes, keys = static_leaf_order_eff(F, Q[i])
        assert r["opened"][i].tolist() == codes[:r["B"]]
        assert r["opened_key"][i].tolist() == keys[:r["B"]]


def test_search_key_variants_open_different_leaves():
    # with several split dimensions the two keys disagree inside groups of
    # equal chain maximum: the reference must not be the variant
    X, Q = _search_case_data(2000, 24, 0, "gauss")
    F = oracle.build_forest(X, 4, 5, 8, 0)
    a = oracle.search(F, X, Q, 3, 100)
    b = oracle.search(F, X, Q, 3, 100, eff_key=True)
    differ = sum(set(a["opened"][i].tolist()) != set(b["opened"][i].tolist())
                 for i in range(len(Q)))
    assert differ >= 1


def test_search_1d_closed_form_nearest_cells():
    # m = t = 1: leaves are intervals of x_s; a leaf's key is the 1-D distance
    # from q_s to its cell [lower split, upper split), so the opened leaves
    # are the B cells nearest to q_s, in that order.
    rng = np.random.default_rng(4)
    X = rng.standard_normal((600, 3)).astype(np.float32)
    X[:, 0] *= 5
    F = oracle.build_forest(X, 1, 1, 4, 8)
    s = int(F["D"][0])
    perm, off = F["perm"][0], F["leaf_off"]
    L = len(off) - 1
    keys = [py_draw(8, 2, 0, i) for i in range(600)]
    srt = sorted(range(600), key=lambda i: (float(X[i, s]), keys[i], i))
    lower = [None] + [X[srt[off[j]], s] for j in range(1, L)]          # cell boundaries
    Q = (X[rng.integers(0, 600, 20)] + 0.3 * rng.standard_normal((20, 3))).astype(np.float32)
    B = 37
    r = oracle.search(F, X, Q, 1, B)
    for i in range(len(Q)):
        qs = Q[i, s]
        dist = []
        for j in range(L):
            lo = lower[j]
            hi = lower[j + 1] if j + 1 < L else None
            if lo is not None and qs < lo:
                dist.append((float(np.float32(lo) - qs), j))
            elif hi is not None and qs >= hi:
                dist.append((float(qs - np.float32(hi)), j))
            else:
                dist.append((0.0, j))
        dist.sort()
        got = sorted((r["opened"][i] & 0xFFFFFF).tolist())
        exp_keys = sorted(k for k, _ in dist)
        assert r["opened_key"][i].tolist() == exp_keys[:B]
        assert set(got) == {j for _, j in dist[:B]} or exp_keys[B - 1] == exp_keys[B]


def test_search_nesting_and_count():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((3000, 32)).astype(np.float32)
    Q = (X[:10] + 0.05).astype(np.float32)
    F = oracle.build_forest(X, 4, 5, 8, 2)
    total = 4 << F["H"]
    prev = None
    for c in [1, 7, 64, 300, total, total + 50]:
        r = oracle.search(F, X, Q, 2, c)
        assert r["B"] == min(c, total)
        assert r["opened"].shape[1] == min(c, total)
        for i in range(10):
            assert len(set(r["opened"][i].tolist())) == r["B"]        # distinct leaves
        if prev is not None:
            assert np.array_equal(r["opened"][:, :prev.shape[1]], prev)   # nested in c
        prev = r["opened"]


def test_search_budget_with_eps():
    assert oracle.budget(100, 0.0, 10**6) == 100
    assert oracle.budget(100, 0.5, 10**6) == 67          # ceil(100 / 1.5)
    assert oracle.budget(100, 1.0, 10**6) == 50
    assert oracle.budget(101, 1.0, 10**6) == 51
    assert oracle.budget(100, 0.0, 40) == 40


def test_search_candidates_union_and_topk_over_them():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((4000, 40)).astype(np.float32)
    Q = (X[rng.integers(0, 4000, 15)] + 0.05 * rng.standard_normal((15, 40))).astype(np.float32)
    F = oracle.build_forest(X, 4, 5, 8, 3)
    r = oracle.search(F, X, Q, 7, 90, candidates=True)
    for i in range(15):
        union = set()
        for code in r["opened"][i].tolist():
            tr, leaf = code >> 24, code & 0xFFFFFF
            union |= set(F["perm"][tr, F["leaf_off"][leaf]:F["leaf_off"][leaf + 1]].tolist())
        assert sorted(union) == r["cand"][i].tolist()
    ei, ed = bf.knn_exact(X, Q, 7, subset=r["cand"])
    assert np.array_equal(r["ids"], ei)
    assert np.allclose(r["dists"], ed, rtol=1e-13, atol=0)


@pytest.mark.parametrize("eff_key", [False, True])
def test_search_exhaustive_budget_is_exact_knn(eff_key):
    rng = np.random.default_rng(6)
    X = rng.standard_normal((1500, 20)).astype(np.float32)
    Q = rng.standard_normal((25, 20)).astype(np.float32)
    F = oracle.build_forest(X, 3, 4, 6, 6)
    r = oracle.search(F, X, Q, 10, 3 << F["H"], eff_key=eff_key, candidates=True)
    assert all(len(cq) == 1500 for cq in r["cand"])
    ei, ed = bf.knn_exact(X, Q, 10)
    assert np.array_equal(r["ids"], ei)
    assert np.allclose(r["dists"], ed, rtol=1e-13, atol=0)


def test_search_single_leaf_tree_is_exact_knn():
    # p >= n: H = 0, each tree is one leaf holding every point
    rng = np.random.default_rng(9)
    X = rng.standard_normal((50, 6)).astype(np.float32)
    Q = rng.standard_normal((5, 6)).astype(np.float32)
    F = oracle.build_forest(X, 2, 2, 64, 1)
    assert F["H"] == 0
    r = oracle.search(F, X, Q, 4, 1)
    ei, ed = bf.knn_exact(X, Q, 4)
    assert np.array_equal(r["ids"], ei) and np.allclose(r["dists"], ed, rtol=1e-13)


def test_search_pads_when_fewer_than_k_candidates():
    rng = np.random.default_rng(10)
    X = rng.standard_normal((100, 4)).astype(np.float32)
    F = oracle.build_forest(X, 1, 2, 3, 1)
    r = oracle.search(F, X, X[:3], 8, 1, candidates=True)
    for i in range(3):
        nc = int(r["ncand"][i])
        assert nc <= 3
        assert r["ids"][i, nc:].tolist() == [-1] * (8 - nc)
        assert np.all(np.isinf(r["dists"][i, nc:]))
        assert r["ids"][i, 0] == i and r["dists"][i, 0] == 0.0


def test_search_home_leaves_first():
    # the first m pops are the m home leaves (key 0), in tree order
    rng = np.random.default_rng(11)
    X = rng.standard_normal((800, 10)).astype(np.float32)
    Q = rng.standard_normal((6, 10)).astype(np.float32)
    F = oracle.build_forest(X, 5, 3, 4, 4)
    for eff_key in (False, True):
        r = oracle.search(F, X, Q, 1, 40, eff_key=eff_key)
        assert np.all(r["opened_key"][:, :5] == 0)
        assert ((r["opened"][:, :5] >> 24) == np.arange(5)).all()


def test_search_threads_do_not_change_results():
    w_rng = np.random.default_rng(12)
    X = w_rng.standard_normal((2500, 30)).astype(np.float32)
    Q = w_rng.standard_normal((40, 30)).astype(np.float32)
    F1 = oracle.build_forest(X, 4, 5, 8, 5, nthreads=1)
    F4 = oracle.build_forest(X, 4, 5, 8, 5, nthreads=4)
    for key in ("split_dim", "split_val", "perm", "leaf_off", "D"):
        assert np.array_equal(F1[key], F4[key])
    r1 = oracle.search(F1, X, Q, 5, 77, nthreads=1)
    r4 = oracle.search(F1, X, Q, 5, 77, nthreads=4)
    for key in ("ids", "dists", "opened", "opened_key"):
        assert np.array_equal(r1[key], r4[key])


# ---------------------------------------------------------------- isometry
# The variant of Sec. 2.1 ("Rotation") with the Householder reflector of
# Sec. 2.2: tree i splits the coordinates of (I - 2 u_i u_i') x.


def test_householder_vectors_unit_deterministic_distinct():
    u0 = oracle.householder(7, 0, 300)
    assert np.array_equal(u0, oracle.householder(7, 0, 300))
    assert abs(float(np.dot(u0, u0)) - 1.0) < 1e-14
    u1 = oracle.householder(7, 1, 300)
    assert not np.allclose(u0, u1)
    # the reflector is an isometry and an involution (FP64, to rounding)
    rng = np.random.default_rng(2)
    x, y = rng.standard_normal(300), rng.standard_normal(300)
    P = lambda v: v - 2.0 * np.dot(u0, v) * u0
    assert abs(np.linalg.norm(P(x) - P(y)) - np.linalg.norm(x - y)) < 1e-12
    assert np.allclose(P(P(x)), x, rtol=0, atol=1e-13)


def test_householder_e0_is_the_plain_method_on_a_negated_column():
    # u = e_0 reflects across the plane x_0 = 0: every reflected coordinate is
    # exact (-x_0, and x_s for s != 0), variances are unchanged, and so are
    # all distances.  The forest and every search must equal the plain ones
    # on the data with column 0 negated.
    rng = np.random.default_rng(4)
    X = rng.standard_normal((2000, 8)).astype(np.float32)
    X[:, 0] *= 3.0                        # column 0 among the top-variance dims
    Q = rng.standard_normal((30, 8)).astype(np.float32)
    Xn, Qn = X.copy(), Q.copy()
    Xn[:, 0] = -Xn[:, 0]
    Qn[:, 0] = -Qn[:, 0]
    m = 3
    U = np.zeros((m, 8))
    U[:, 0] = 1.0
    Fi = oracle.build_forest(X, m, 4, 8, 21, u=U)
    Fp = oracle.build_forest(Xn, m, 4, 8, 21)
    assert 0 in Fi["D"].tolist()
    for key in ("D", "split_dim", "split_val", "perm", "leaf_off"):
        assert np.array_equal(Fi[key], Fp[key]), key
    for c in (1, 5, 40):
        ri = oracle.search(Fi, X, Q, 5, c, candidates=True)
        rp = oracle.search(Fp, Xn, Qn, 5, c, candidates=True)
        assert np.array_equal(ri["opened"], rp["opened"])
        assert np.array_equal(ri["ids"], rp["ids"])
        assert np.array_equal(ri["dists"], rp["dists"])


def test_householder_forest_differs_and_exhaustive_budget_is_exact_knn():
    rng = np.random.default_rng(8)
    X = rng.standard_normal((1500, 20)).astype(np.float32)
    Q = rng.standard_normal((25, 20)).astype(np.float32)
    Fi = oracle.build_forest(X, 3, 4, 6, 6, householder_variant=True)
    Fp = oracle.build_forest(X, 3, 4, 6, 6)
    assert np.array_equal(Fi["D"], Fp["D"])           # D comes from X itself
    assert not np.array_equal(Fi["perm"], Fp["perm"])
    for tr in range(3):                                 # every tree partitions all points
        assert np.array_equal(np.sort(Fi["perm"][tr]), np.arange(1500, dtype=np.uint32))
    assert set(Fi["split_dim"].ravel().tolist()) <= set(Fi["D"].tolist())
    r = oracle.search(Fi, X, Q, 10, 3 << Fi["H"], candidates=True)
    assert all(len(cq) == 1500 for cq in r["cand"])
    ei, ed = bf.knn_exact(X, Q, 10)
    assert np.array_equal(r["ids"], ei)
    assert np.allclose(r["dists"], ed, rtol=1e-13, atol=0)
    # a small budget opens different leaves than the plain forest does
    ri = oracle.search(Fi, X, Q, 10, 4)
    rp = oracle.search(Fp, X, Q, 10, 4)
    assert not np.array_equal(ri["opened"], rp["opened"])


# ------------------------------------------------ sharding the trees (design)
# Across GPUs the trees would be split into groups.  Each group ranks its own
# leaves by the static key of Alg. 2's order (a leaf's strictly decreasing
# suffix maxima of (|gap|, tree, node)) and keeps its B smallest; the B
# smallest of the union are the opened set, because every key of the global
# B smallest is among its own group's B smallest.  Each group then takes the
# best k of its own candidates, and merging those lists with duplicates
# removed (a point can be a candidate in several groups, with the same
# distance) gives the global best k.


@pytest.mark.parametrize("groups", [2, 3, 5])
def test_tree_sharding_merge_equals_global_selection(groups):
    rng = np.random.default_rng(17)
    X = rng.standard_normal((3000, 12)).astype(np.float32)
    Q = (X[rng.integers(0, 3000, 8)] + 0.1 * rng.standard_normal((8, 12))).astype(np.float32)
    m, c, k = 6, 40, 5
    F = oracle.build_forest(X, m, 5, 8, 23)
    r = oracle.search(F, X, Q, k, c, candidates=True)
    B = r["B"]
    lo = F["leaf_off"].astype(np.int64)
    for i in range(len(Q)):
        # every leaf in Alg. 2's static order; a leaf's position in this
        # list stands for its full key
        codes, _ = static_leaf_order_gap(F, Q[i])
        trees = np.array([cd >> 24 for cd in codes])
        shard_of_tree = np.arange(m) % groups
        merged, local_best = [], []
        for g in range(groups):
            mine = [j for j in range(len(codes)) if shard_of_tree[trees[j]] == g][:B]
            merged += mine                                   # this group's B smallest keys
        opened = [codes[j] for j in sorted(merged)[:B]]
        assert opened == r["opened"][i].tolist()
        # per group: candidates of its own opened leaves, best k, then merge
        for g in range(groups):
            ids = set()
            for code in opened:
                if shard_of_tree[code >> 24] == g:
                    leaf = code & 0xFFFFFF
                    ids.update(F["perm"][code >> 24][lo[leaf]:lo[leaf + 1]].tolist())
            ids = np.array(sorted(ids), dtype=np.int64)
            if ids.size:
                diff = X[ids].astype(np.float64) - Q[i].astype(np.float64)
                dd = np.einsum("ij,ij->i", diff, diff)
                order = np.lexsort((ids, dd))[:k]
                local_best += list(zip(dd[order].tolist(), ids[order].tolist()))
        best = sorted(set(local_best))[:k]                   # duplicates are identical pairs
        assert [b[1] for b in best] == r["ids"][i][:len(best)].tolist()
        assert np.allclose([b[0] for b in best], r["dists"][i][:len(best)], rtol=1e-12, atol=0)


# ---------------------------------------------------------------- split-value jitter (Sec. 2.1)

JITTER_CASES = [("gauss", 2500, 16, 3, 5, 8, "approx"),
                ("gauss", 600, 40, 2, 6, 4, "exact"),
                ("quantised", 1800, 24, 3, 5, 6, "approx"),
                ("wide", 900, 300, 2, 8, 5, "approx")]


def _jitter_data(kind, n, d, seed=3):
    rng = np.random.default_rng(seed)
    if kind == "quantised":
        return rng.integers(0, 6, (n, d)).astype(np.float32)
    if kind == "wide":
        return (rng.standard_normal((n, d)) * np.linspace(0.5, 2.0, d)).astype(np.float32)
    if kind == "uniform":
        return rng.random((n, d)).astype(np.float32)
    return rng.standard_normal((n, d)).astype(np.float32)


def _subtree_ids(F, tr, i):
    """The point ids under explicit node i of tree tr."""
    out, stack = [], [i]
    while stack:
        j = stack.pop()
        if F["dim"][tr, j] < 0:
            a = int(F["off"][tr, j])
            out.extend(F["perm"][tr, a:a + int(F["len"][tr, j])].tolist())
        else:
            stack += [int(F["left"][tr, j]), int(F["right"][tr, j])]
    return np.array(sorted(out), np.int64)


def _diameter(P):
    g = P.astype(np.float64)
    sq = (g * g).sum(1)
    d2 = np.maximum(sq[:, None] + sq[None, :] - 2.0 * g @ g.T, 0.0)
    return math.sqrt(float(d2.max()))


@pytest.mark.parametrize("kind,n,d,m,t,p,diam", JITTER_CASES)
def test_jitter_splits_leaves_and_delta_range(kind, n, d, m, t, p, diam):
    """Every internal node: its points split at the value (left < v <= right),
    or, where that would leave a side empty, at the median with the median's
    own value; v lies within 3 Delta / sqrt(d) of the median (Delta the
    brute-force diameter, which bounds both readings of it); internal nodes
    hold > p points, leaves <= p, ascending, and each tree's leaves partition
    the ids.  Heap indices follow the tree's shape."""
    X = _jitter_data(kind, n, d)
    seed = 17
    F = oracle.build_forest_jitter(X, m, t, p, seed, diameter=diam)
    assert F["H"] <= 23
    for tr in range(m):
        nn = int(F["nnodes"][tr])
        leaves = []
        for i in range(nn):
            ids = _subtree_ids(F, tr, i)
            if F["dim"][tr, i] < 0:
                assert len(ids) <= p
                a = int(F["off"][tr, i])
                seg = F["perm"][tr, a:a + int(F["len"][tr, i])]
                assert np.all(np.diff(seg.astype(np.int64)) > 0)
                leaves.append(seg)
                continue
            assert len(ids) > p
            s, v = int(F["dim"][tr, i]), np.float32(F["val"][tr, i])
            assert s in F["D"].tolist()
            L = _subtree_ids(F, tr, int(F["left"][tr, i]))
            R = _subtree_ids(F, tr, int(F["right"][tr, i]))
            assert len(L) > 0 and len(R) > 0 and len(L) + len(R) == len(ids)
            h = int(F["heap"][tr, i])
            assert F["heap"][tr, F["left"][tr, i]] == 2 * h + 1
            assert F["heap"][tr, F["right"][tr, i]] == 2 * h + 2
            # the median item under (coordinate, tie key, id)
            keys = sorted((float(X[j, s]), oracle.draw(seed, 2, tr, int(j)), int(j)) for j in ids)
            med = np.float32(keys[len(ids) // 2][0])
            if np.all(X[L, s] < v) and np.all(X[R, s] >= v):
                bound = 3.0 * _diameter(X[ids]) / math.sqrt(d)
                assert abs(float(v) - float(med)) <= bound * (1 + 1e-12) + float(np.spacing(np.float32(abs(v))))
            else:
                # the median split of the plain build
                assert v == med
                assert set(L.tolist()) == {k[2] for k in keys[:len(ids) // 2]}
        allids = np.sort(np.concatenate(leaves))
        assert np.array_equal(allids, np.arange(n))


def test_jitter_delta_spans_its_range_and_the_approximate_diameter_bounds():
    """On nearly collinear points in d = 900 (so 3 Delta / sqrt(d) = Delta / 10
    keeps every split value inside the data), the root's |v - median| over 40
    seeds, divided by 3 Delta / sqrt(d) with Delta the brute-force diameter,
    stays below 1 for both readings, exceeds 0.8 for the exact one (w spans
    [-1, 1)) and 0.4 for the approximate one (its Delta is >= Delta / 2)."""
    rng = np.random.default_rng(8)
    d = 900
    X = (1e-3 * rng.standard_normal((60, d))).astype(np.float32)
    X[:, 0] = rng.uniform(-1.0, 1.0, 60).astype(np.float32)
    dm = _diameter(X)
    ratios = {"approx": [], "exact": []}
    for diam in ("approx", "exact"):
        for seed in range(40):
            F = oracle.build_forest_jitter(X, 1, 1, 59, seed, diameter=diam)
            assert F["D"].tolist() == [0]
            v = float(F["val"][0, 0])
            keys = sorted((float(X[j, 0]), oracle.draw(seed, 2, 0, j), j) for j in range(60))
            med = keys[30][0]
            ratios[diam].append(abs(v - med) / (3.0 * dm / math.sqrt(d)))
    assert max(ratios["exact"]) <= 1.0 + 1e-6 and max(ratios["approx"]) <= 1.0 + 1e-6
    assert max(ratios["exact"]) > 0.8
    assert max(ratios["approx"]) > 0.4


@pytest.mark.parametrize("kind,n,d,m,t,p,diam", [("uniform", 1500, 8, 3, 5, 4, "exact"),
                                                  ("quantised", 2000, 24, 3, 5, 6, "approx"),
                                                  ("uniform", 3000, 64, 2, 5, 8, "approx")])
def test_jitter_pop_order_equals_static_key_on_the_padded_layout(kind, n, d, m, t, p, diam):
    """The explicit-tree queue's pops equal the static-key order computed on
    the padded perfect layout (pass-through nodes of value +inf, whose far
    sides carry an infinite gap): the layout reproduces the trees."""
    X = _jitter_data(kind, n, d)
    F = oracle.build_forest_jitter(X, m, t, p, 29, diameter=diam)
    assert F["H"] <= 16
    Lay = dict(oracle.jitter_layout(F), H=F["H"], m=m)
    rng = np.random.default_rng(4)
    Q = (X[rng.integers(0, n, 4)] + 0.3 * rng.standard_normal((4, d))).astype(np.float32)
    nleaves = sum(int((F["dim"][tr, :F["nnodes"][tr]] < 0).sum()) for tr in range(m))
    for c in (1, 7, nleaves // 3, nleaves):
        r = oracle.search(F, X, Q, 3, c)
        for i in range(len(Q)):
            order, keys = static_leaf_order_gap(Lay, Q[i])
            assert np.all(np.isfinite(keys[:nleaves])) and not np.any(np.isfinite(keys[nleaves:]))
            assert r["opened"][i].tolist() == order[:r["B"]]


@pytest.mark.parametrize("diam", ["approx", "exact"])
def test_jitter_exhaustive_budget_is_exact_knn(diam):
    rng = np.random.default_rng(12)
    X = rng.standard_normal((700, 12)).astype(np.float32)
    Q = rng.standard_normal((15, 12)).astype(np.float32)
    F = oracle.build_forest_jitter(X, 3, 4, 5, 2, diameter=diam)
    r = oracle.search(F, X, Q, 8, 10 ** 9, candidates=True)
    assert all(len(cq) == 700 for cq in r["cand"])
    ei, ed = bf.knn_exact(X, Q, 8)
    assert np.array_equal(r["ids"], ei)
    assert np.allclose(r["dists"], ed, rtol=1e-13, atol=0)
