"""Comparison rules shared by the GPU parity tests (no method arithmetic)."""
import numpy as np


def leaf_set_from_bits(bits_row: np.ndarray) -> set:
    """Opened (tree << 24 | leaf) codes from one query's [m][W] leaf bitmap."""
    out = set()
    m, W = bits_row.shape
    for tree in range(m):
        for w in range(W):
            b = int(bits_row[tree, w])
            while b:
                j = (b & -b).bit_length() - 1
                out.add((tree << 24) | (w * 32 + j))
                b &= b - 1
    return out


def ids_from_bits(bits_row: np.ndarray, n: int) -> np.ndarray:
    bits = np.unpackbits(bits_row.view(np.uint8), bitorder="little")[:n]
    return np.nonzero(bits)[0]


def check_knn(got_ids, got_d, ref_ids, ref_d64, rel=1e-5, tie=1e-6, X=None, Q=None, cand=None):
    """The acceptance rule for neighbours: let dk be the oracle's k-th FP64
    distance; every oracle id with distance < dk(1 - tie) must be returned,
    every returned id's true distance must be <= dk(1 + tie), returned
    distances must be within `rel` of the oracle's (relative), and padding
    must agree.  With cand (the oracle's candidate set of each query, sorted
    ids) every returned id must also be one of the query's candidates.
    Returns the number of queries checked."""
    nq, k = ref_ids.shape
    for i in range(nq):
        if cand is not None:
            got_all = got_ids[i][got_ids[i] >= 0]
            inside = np.isin(got_all, cand[i])
            assert inside.all(), f"query {i}: ids {got_all[~inside].tolist()} are not candidates"
        valid = ref_ids[i] >= 0
        assert np.array_equal(got_ids[i] >= 0, valid), f"query {i}: padding differs"
        if not valid.any():
            continue
        dk = ref_d64[i][valid][-1]
        must = set(ref_ids[i][valid][ref_d64[i][valid] < dk * (1 - tie)].tolist())
        got = got_ids[i][got_ids[i] >= 0]
        assert must <= set(got.tolist()), f"query {i}: missing {must - set(got.tolist())}"
        assert len(set(got.tolist())) == len(got), f"query {i}: duplicate ids"
        ref_map = dict(zip(ref_ids[i].tolist(), ref_d64[i].tolist()))
        for j, gid in enumerate(got.tolist()):
            if gid in ref_map:
                true_d = ref_map[gid]
            else:
                diff = X[gid].astype(np.float64) - Q[i].astype(np.float64)
                true_d = float(diff @ diff)
            assert true_d <= dk * (1 + tie), f"query {i}: id {gid} beyond the k-th distance"
            assert abs(float(got_d[i][j]) - true_d) <= rel * true_d, \
                f"query {i}: distance of id {gid}: {got_d[i][j]} vs {true_d}"
        assert np.all(np.diff(got_d[i][got_ids[i] >= 0]) >= 0), f"query {i}: not sorted"
    return nq


def assert_tree_arrays_equal(T, Fo):
    """The library's exported tree arrays against the oracle's: D, split
    dimensions, leaf-ordered ids, split values bit for bit, and per-tree leaf
    offsets (the oracle's plain build holds one row shared by every tree)."""
    assert T["H"] == Fo["H"]
    for key in ("D", "split_dim", "perm"):
        assert np.array_equal(T[key], Fo[key]), key
    assert np.array_equal(T["split_val"].view(np.uint32), Fo["split_val"].view(np.uint32)), "split_val"
    lo = np.asarray(Fo["leaf_off"])
    if lo.ndim == 1:
        lo = np.broadcast_to(lo, T["leaf_off"].shape)
    assert np.array_equal(T["leaf_off"], lo), "leaf_off"
