"""Exact k nearest neighbours by definition (Def. 1 with eps = 0): every
point's squared Euclidean distance to the query, in FP64, then the k smallest
(distance, id) pairs ascending.  TEST INFRASTRUCTURE ONLY.

``knn_exact`` is the plain definition (direct differences, FP64); it pins the
oracle's search when the budget covers every leaf.  ``knn_ground_truth`` is the
same definition made affordable for a million points: a float32 inner-product
pre-selection keeps the ``keep`` best per query, which are then re-measured
exactly in FP64 and ranked; it is used only to score recall.
"""
from __future__ import annotations

import numpy as np


def sqdist_fp64(Q: np.ndarray, X: np.ndarray) -> np.ndarray:
    """[nq, n] squared distances sum_j (q_j - x_j)^2 in FP64."""
    Q64 = np.asarray(Q, dtype=np.float64)
    X64 = np.asarray(X, dtype=np.float64)
    out = np.empty((Q64.shape[0], X64.shape[0]), dtype=np.float64)
    for i in range(Q64.shape[0]):
        diff = X64 - Q64[i]
        out[i] = np.einsum("ij,ij->i", diff, diff)
    return out


def topk_rows(dist: np.ndarray, ids: np.ndarray, k: int):
    """k smallest (dist, id) per row, ascending; pads with (-1, inf)."""
    nq = dist.shape[0]
    out_i = np.full((nq, k), -1, dtype=np.int64)
    out_d = np.full((nq, k), np.inf, dtype=np.float64)
    for r in range(nq):
        order = np.lexsort((ids[r], dist[r]))[:k]
        out_i[r, :order.size] = ids[r][order]
        out_d[r, :order.size] = dist[r][order]
    return out_i, out_d


def knn_exact(X: np.ndarray, Q: np.ndarray, k: int, subset=None):
    """Exact k-NN of every query over X (or over the given id subset per
    query, a list of int arrays)."""
    nq = np.asarray(Q).shape[0]
    out_i = np.full((nq, k), -1, dtype=np.int64)
    out_d = np.full((nq, k), np.inf, dtype=np.float64)
    for r in range(nq):
        ids = np.arange(X.shape[0]) if subset is None else np.asarray(subset[r], dtype=np.int64)
        if ids.size == 0:
            continue
        diff = np.asarray(X, dtype=np.float64)[ids] - np.asarray(Q[r], dtype=np.float64)
        d = np.einsum("ij,ij->i", diff, diff)
        order = np.lexsort((ids, d))[:k]
        out_i[r, :order.size] = ids[order]
        out_d[r, :order.size] = d[order]
    return out_i, out_d


def knn_ground_truth(X: np.ndarray, Q: np.ndarray, k: int, keep: int = 64,
                     chunk: int = 65536):
    """Exact k-NN for large X: float32 inner-product pre-selection of `keep`
    candidates per query, then exact FP64 re-measurement and ranking."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    Q = np.ascontiguousarray(Q, dtype=np.float32)
    n = X.shape[0]
    nq = Q.shape[0]
    keep = min(keep, n)
    best_s = np.full((nq, keep), np.inf, dtype=np.float32)
    best_i = np.zeros((nq, keep), dtype=np.int64)
    for a in range(0, n, chunk):
        xb = X[a:a + chunk]
        xn = np.einsum("ij,ij->i", xb, xb)
        s = xn[None, :] - 2.0 * (Q @ xb.T)           # ||x||^2 - 2 q.x (rank-equivalent)
        cat_s = np.concatenate([best_s, s], axis=1)
        cat_i = np.concatenate([best_i, np.broadcast_to(np.arange(a, a + xb.shape[0]),
                                                        s.shape)], axis=1)
        sel = np.argpartition(cat_s, keep - 1, axis=1)[:, :keep]
        best_s = np.take_along_axis(cat_s, sel, axis=1)
        best_i = np.take_along_axis(cat_i, sel, axis=1)
    out_i = np.empty((nq, k), dtype=np.int64)
    out_d = np.empty((nq, k), dtype=np.float64)
    for r in range(nq):
        ids = best_i[r]
        diff = X[ids].astype(np.float64) - Q[r].astype(np.float64)
        d = np.einsum("ij,ij->i", diff, diff)
        order = np.lexsort((ids, d))[:k]
        out_i[r] = ids[order]
        out_d[r] = d[order]
    return out_i, out_d
