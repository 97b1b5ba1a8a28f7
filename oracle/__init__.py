"""FP64 CPU oracle for the kd-GeRaF build and query (arXiv 1603.09596).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark call it; the product library never does.  It shares no code
with the GPU library.  ``oracle.c`` holds the method (Alg. 1-3, Sec. 2.3);
this module compiles it with gcc and marshals numpy arrays through ctypes.
``bruteforce.py`` holds the exact k-NN definition used to pin it.

Parity status of each function (what pins it is in tests/test_oracle.py):
  splitmix64 / draw     pinned: published splitmix64 outputs for state 0
  variance / top dims   pinned: numpy.var(ddof=1), hand-made columns
  build                 pinned: partition / median / leaf-size invariants,
                        the closed form for t = 1 (contiguous rank blocks)
  build, near-tie guard pinned: duplicated and nearly equal columns at the
                        rank-t boundary are refused, separated ones pass
  search (Alg. 2 key,   pinned: the pop ORDER equals the sort of every leaf's
   the reference)       static key (the strictly decreasing suffix maxima of
                        the gaps on its root path, by an independent
                        traversal in the test); hand-worked examples (a far
                        gap below its entry's key, an exactly zero gap, the
                        2-D and 1-D cases); the 1-D closed form for m = t = 1;
                        nesting in c; exhaustive budget = brute force
  search (eff key)      diagnostic variant only (key = max along the chain):
                        pinned by its own static ranking; it differs from the
                        Alg. 2 key inside groups of equal eff
  householder / build and search with the isometry
                        pinned: u unit and deterministic; u = e_0 (a
                        reflection that negates one coordinate) gives the
                        forest and searches of the plain method on the data
                        with that column negated; exhaustive budget = brute
                        force
  build_jitter /        pinned: every split separates its points at the
   search_jitter        split value (or is the median split when a side
                        would be empty), lies within 3 Delta / sqrt(d) of the
                        median, leaves hold <= p points and partition the
                        ids; the approximate diameter lies in [Delta/2, Delta]
                        of the brute-force one; the pop order equals the
                        static-key order computed on the padded layout;
                        exhaustive budget = brute force
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (-O2, no fast-math) into liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
                               "-ffp-contract=off", "-Wall", "-o", tmp, _SRC, "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i32, i64, u64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    lib.orc_splitmix64.argtypes = [u64]
    lib.orc_splitmix64.restype = u64
    lib.orc_draw.argtypes = [u64, u64, u64, u64]
    lib.orc_draw.restype = u64
    lib.orc_variance.argtypes = [P, i64, i32, P]
    lib.orc_variance.restype = ctypes.c_int
    lib.orc_top_dims.argtypes = [P, i32, i32, P]
    lib.orc_top_dims.restype = ctypes.c_int
    lib.orc_dims_ambiguous.argtypes = [P, i64, i32, i32, P]
    lib.orc_dims_ambiguous.restype = ctypes.c_int
    lib.orc_depth.argtypes = [i64, i32]
    lib.orc_depth.restype = i32
    lib.orc_budget.argtypes = [i64, f64, i64]
    lib.orc_budget.restype = i64
    lib.orc_householder.argtypes = [u64, i32, i32, P]
    lib.orc_householder.restype = ctypes.c_int
    lib.orc_build.argtypes = [P, i64, i32, i32, i32, i32, u64, i32, P, P, P, P, P, P]
    lib.orc_build.restype = ctypes.c_int
    lib.orc_search.argtypes = [P, i64, i32, i32, i32, P, P, P, P, P, i64, i32, i64, f64,
                               i32, i32, P, P, P, P, P, P, i64, P]
    lib.orc_search.restype = ctypes.c_int
    lib.orc_build_jitter.argtypes = [P, i64, i32, i32, i32, i32, u64, i32, i64,
                                     P, P, P, P, P, P, P, P, P, P, P, P]
    lib.orc_build_jitter.restype = ctypes.c_int
    lib.orc_search_jitter.argtypes = [P, i64, i32, i32, i32, i64, P, P, P, P, P, P, P, P, P, P,
                                      P, i64, i32, i64, f64, P, P, P, P, P, P, i64]
    lib.orc_search_jitter.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def splitmix64(x: int) -> int:
    return int(_load().orc_splitmix64(x & 0xFFFFFFFFFFFFFFFF))


def draw(seed: int, stream: int, tree: int, idx: int) -> int:
    return int(_load().orc_draw(seed, stream, tree, idx))


def variance(X: np.ndarray) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.float32)
    V = np.empty(X.shape[1], dtype=np.float64)
    st = _load().orc_variance(_ptr(X), X.shape[0], X.shape[1], _ptr(V))
    if st != 0:
        raise ValueError(f"orc_variance failed: {st}")
    return V


def top_dims(V: np.ndarray, t: int) -> np.ndarray:
    V = np.ascontiguousarray(V, dtype=np.float64)
    D = np.empty(t, dtype=np.int32)
    st = _load().orc_top_dims(_ptr(V), V.shape[0], t, _ptr(D))
    if st != 0:
        raise ValueError(f"orc_top_dims failed: {st}")
    return D


def dims_ambiguous(X: np.ndarray, t: int) -> bool:
    """Whether the t-th and (t+1)-th largest variances of X are too close
    for the top-t set to be defined (see orc_dims_ambiguous)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    V = variance(X)
    return bool(_load().orc_dims_ambiguous(_ptr(X), X.shape[0], X.shape[1], t, _ptr(V)))


class NearTieError(ValueError):
    """The build refused data whose top-t variance set is not determined."""


def depth(n: int, p: int) -> int:
    return int(_load().orc_depth(n, p))


def budget(c: int, eps: float, total_leaves: int) -> int:
    return int(_load().orc_budget(c, eps, total_leaves))


def householder(seed: int, tree: int, d: int) -> np.ndarray:
    """The reflector u of tree `tree` (FP64, unit norm; see orc_householder)."""
    u = np.empty(d, dtype=np.float64)
    st = _load().orc_householder(seed & 0xFFFFFFFFFFFFFFFF, tree, d, _ptr(u))
    if st != 0:
        raise ValueError(f"orc_householder failed: {st}")
    return u


def build_forest(X: np.ndarray, m: int, t: int, p: int, seed: int, nthreads: int = 0,
                 householder_variant: bool = False, u: Optional[np.ndarray] = None) -> dict:
    """Alg. 1.  Returns the forest arrays (see oracle.c, orc_build).  With
    householder_variant, tree i is built on the points reflected by
    I - 2 u_i u_i' (u_i from householder(seed, i, d), or the rows of `u`
    when given) and the forest carries "u" for search()."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    n, d = X.shape
    U = None
    if u is not None:
        U = np.ascontiguousarray(u, dtype=np.float64).reshape(m, d)
    elif householder_variant:
        U = np.stack([householder(seed, i, d) for i in range(m)])
    H = depth(n, p)
    n_int = (1 << H) - 1
    D = np.empty(t, dtype=np.int32)
    split_dim = np.zeros((m, max(n_int, 1)), dtype=np.int32)
    split_val = np.zeros((m, max(n_int, 1)), dtype=np.float32)
    perm = np.empty((m, n), dtype=np.uint32)
    leaf_off = np.empty((1 << H) + 1, dtype=np.uint32)
    if nthreads <= 0:
        nthreads = os.cpu_count() or 1
    st = _load().orc_build(_ptr(X), n, d, m, t, p, seed & 0xFFFFFFFFFFFFFFFF, nthreads, _ptr(D),
                           _ptr(split_dim), _ptr(split_val), _ptr(perm), _ptr(leaf_off), _ptr(U))
    if st == -3:
        raise NearTieError("near-tie in D: the t-th and (t+1)-th largest variances are "
                           "within rounding of each other")
    if st != 0:
        raise ValueError(f"orc_build failed: {st}")
    return dict(n=n, d=d, m=m, t=t, p=p, seed=seed, H=H, D=D,
                split_dim=split_dim[:, :n_int], split_val=split_val[:, :n_int],
                perm=perm, leaf_off=leaf_off, u=U)


def build_forest_jitter(X: np.ndarray, m: int, t: int, p: int, seed: int,
                        diameter: str = "approx") -> dict:
    """Alg. 1 with the split-value jitter of Sec. 2.1 (see orc_build_jitter):
    explicit trees (node arrays [m][ncap], per tree nnodes[tr] of them), the
    leaf-ordered perm [m][n], D and H = the deepest leaf.  diameter: "approx"
    or "exact"."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    n, d = X.shape
    ncap = 2 * n
    D = np.empty(t, np.int32)
    arr = {name: np.zeros((m, ncap), dt) for name, dt in
           (("dim", np.int32), ("val", np.float32), ("left", np.int32), ("right", np.int32),
            ("heap", np.int32), ("depth", np.int32), ("off", np.uint32), ("len", np.uint32))}
    perm = np.empty((m, n), np.uint32)
    nnodes = np.zeros(m, np.int64)
    H = ctypes.c_int32(0)
    st = _load().orc_build_jitter(_ptr(X), n, d, m, t, p, seed & 0xFFFFFFFFFFFFFFFF,
                                  int(diameter == "exact"), ncap, _ptr(D),
                                  *[_ptr(arr[k]) for k in ("dim", "val", "left", "right", "heap",
                                                            "depth", "off", "len")],
                                  _ptr(perm), _ptr(nnodes), ctypes.byref(H))
    if st == -3:
        raise NearTieError("near-tie in D")
    if st != 0:
        raise ValueError(f"orc_build_jitter failed: {st}")
    return dict(n=n, d=d, m=m, t=t, p=p, seed=seed, H=int(H.value), D=D, jitter=diameter,
                ncap=ncap, nnodes=nnodes, perm=perm, **arr)


def jitter_layout(F: dict) -> dict:
    """The padded perfect layout of depth H of jittered trees: a real node
    keeps its heap index; below a real leaf every internal position is a
    pass-through node (dimension D[0], value +inf: points and queries all go
    left), and the leaf sits at its leftmost position of depth H.  Returns
    split_dim, split_val [m][2^H - 1], perm [m][n] and leaf_off [m][2^H + 1]."""
    m, H, n = F["m"], F["H"], F["n"]
    nint, nleaf = (1 << H) - 1, 1 << H
    sd = np.full((m, max(nint, 1)), F["D"][0], np.int32)
    sv = np.full((m, max(nint, 1)), np.inf, np.float32)
    lo = np.zeros((m, nleaf + 1), np.uint32)
    for tr in range(m):
        starts = np.full(nleaf, -1, np.int64)
        for i in range(int(F["nnodes"][tr])):
            h, dep = int(F["heap"][tr, i]), int(F["depth"][tr, i])
            if F["dim"][tr, i] >= 0:
                sd[tr, h], sv[tr, h] = F["dim"][tr, i], F["val"][tr, i]
            else:
                j = h - ((1 << dep) - 1)
                starts[j << (H - dep)] = int(F["off"][tr, i])
        # empty leaves start where the next real leaf does (perm is in leaf order)
        nxt = n
        for L in range(nleaf - 1, -1, -1):
            if starts[L] >= 0:
                nxt = starts[L]
            lo[tr, L] = nxt
        lo[tr, nleaf] = n
    return dict(split_dim=sd[:, :nint], split_val=sv[:, :nint], perm=F["perm"], leaf_off=lo)


def search(forest: dict, X: np.ndarray, Q: np.ndarray, k: int, c: int, eps: float = 0.0,
           eff_key: bool = False, nthreads: int = 0, trace: bool = True,
           candidates: bool = False) -> dict:
    """Alg. 2 for every row of Q.  Returns ids [nq,k], dists [nq,k] (FP64,
    squared), and with trace=True the opened (tree<<24|leaf) codes and keys in
    pop order; with candidates=True the checked point ids per query.  The
    queue key is Alg. 2's |gap|; eff_key=True selects the diagnostic variant
    whose key is the maximum gap along the chain."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    Q = np.ascontiguousarray(Q, dtype=np.float32)
    if forest.get("jitter"):
        return _search_jitter(forest, X, Q, k, c, eps, trace, candidates)
    n, d = X.shape
    nq = Q.shape[0]
    m, H = forest["m"], forest["H"]
    B = budget(c, eps, m << H)
    n_int = (1 << H) - 1
    sd = np.zeros((m, max(n_int, 1)), dtype=np.int32)
    sv = np.zeros((m, max(n_int, 1)), dtype=np.float32)
    sd[:, :n_int] = forest["split_dim"]
    sv[:, :n_int] = forest["split_val"]
    ids = np.empty((nq, k), dtype=np.int32)
    dists = np.empty((nq, k), dtype=np.float64)
    opened = np.empty((nq, B), dtype=np.uint32) if trace else None
    okey = np.empty((nq, B), dtype=np.float64) if trace else None
    ncand = np.empty(nq, dtype=np.int64) if candidates else None
    lo = forest["leaf_off"].astype(np.int64)
    pmax = int((lo[1:] - lo[:-1]).max()) if lo.size > 1 else 0
    cap = min(n, B * pmax) if candidates else 0
    cand = np.empty((nq, max(cap, 1)), dtype=np.uint32) if candidates else None
    if nthreads <= 0:
        nthreads = os.cpu_count() or 1
    st = _load().orc_search(_ptr(X), n, d, m, H, _ptr(sd), _ptr(sv),
                            _ptr(np.ascontiguousarray(forest["perm"])),
                            _ptr(np.ascontiguousarray(forest["leaf_off"])),
                            _ptr(Q), nq, k, c, float(eps), int(bool(eff_key)), nthreads,
                            _ptr(ids), _ptr(dists), _ptr(opened), _ptr(okey), _ptr(ncand),
                            _ptr(cand), cap, _ptr(forest.get("u")))
    if st != 0:
        raise ValueError(f"orc_search failed: {st}")
    out = dict(ids=ids, dists=dists, B=B)
    if trace:
        out["opened"] = opened
        out["opened_key"] = okey
    if candidates:
        out["ncand"] = ncand
        out["cand"] = [cand[i, :ncand[i]].copy() for i in range(nq)]
    return out


def _search_jitter(F, X, Q, k, c, eps, trace, candidates):
    n, d = X.shape
    nq, m, H = Q.shape[0], F["m"], F["H"]
    leaves = int(sum(int((F["dim"][tr, :F["nnodes"][tr]] < 0).sum()) for tr in range(m)))
    B = budget(c, eps, leaves)
    ids = np.empty((nq, k), np.int32)
    dists = np.empty((nq, k), np.float64)
    opened = np.empty((nq, max(B, 1)), np.uint32) if trace else None
    okey = np.empty((nq, max(B, 1)), np.float64) if trace else None
    ncand = np.empty(nq, np.int64) if candidates else None
    cand = np.empty((nq, n), np.uint32) if candidates else None
    st = _load().orc_search_jitter(_ptr(X), n, d, m, H, F["ncap"],
                                   *[_ptr(F[key]) for key in ("dim", "val", "left", "right", "heap",
                                                              "depth", "off", "len", "perm")],
                                   _ptr(F["nnodes"]), _ptr(Q), nq, k, c, float(eps),
                                   _ptr(ids), _ptr(dists), _ptr(opened), _ptr(okey),
                                   _ptr(ncand), _ptr(cand), n if candidates else 0)
    if st != 0:
        raise ValueError(f"orc_search_jitter failed: {st}")
    out = dict(ids=ids, dists=dists, B=B)
    if trace:
        out["opened"] = opened[:, :B]
        out["opened_key"] = okey[:, :B]
    if candidates:
        out["ncand"] = ncand
        out["cand"] = [cand[i, :ncand[i]].copy() for i in range(nq)]
    return out


def leaf_code(tree, leaf):
    return (np.asarray(tree, dtype=np.uint32) << np.uint32(24)) | np.asarray(leaf, dtype=np.uint32)


__all__ = ["build", "splitmix64", "draw", "variance", "top_dims", "dims_ambiguous",
           "NearTieError", "depth", "budget",
           "householder", "build_forest", "build_forest_jitter", "jitter_layout", "search",
           "leaf_code"]
