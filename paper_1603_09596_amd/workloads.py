"""Seeded synthetic workloads shaped like the paper's experiments (Sec. 4).

This module only draws inputs: it holds none of the method's arithmetic and
is shared by the GPU tests, the oracle tests and the benchmark.

The paper's datasets (MNIST, SIFT, GIST) are not available, so these
generators stand in for them with the same shapes; no dataset item is
reproduced.  Every draw comes from numpy's PCG64 through a SeedSequence
tree: the root SeedSequence(seed) spawns [parameters, data, queries]; the
data child spawns one generator per 65,536-row chunk, so the result does
not depend on how many threads fill the chunks.  Gaussians are drawn in
float32.

Workloads (name: shape; points; queries; forest/search parameters):
  gauss-10k-128     10,000 x 128 iid N(0,1); 100 queries = point + N(0, 0.05^2);
                    m=4 t=5 p=8 c=256 k=1
  sphere-100k-1000  100,000 x 1,000 uniform on the unit sphere; 1,000 queries
                    planted at distance 0.3 from a point; m=8 t=5 p=16 c=1024 k=1
  desc-1m-960       1,000,000 x 960 descriptor-like |N(0,1)| * s_j with per-dim
                    scale s_j ~ LogNormal(0, 0.5), rows L2-normalised; 10,000
                    queries = point + N(0, 0.02^2); m=16 t=5 p=32 c=4096 k=10
                    (stands in for GIST 10^6 x 960)
  gauss-200k-10000  200,000 x 10,000 iid N(0,1), 500 random dims scaled x10;
                    2,000 queries = point + N(0, 0.05^2); m=16 t=10 p=16 c=2048 k=10
  multi-20          20 indexes, n log-uniform in [1e4, 5e5], d from
                    {128, 512, 960, 2048}, iid N(0,1); 100..5,000 queries each
                    (point + N(0, 0.05^2)), per-query c uniform in [256, 8192];
                    m=8 t=5 p=16 k=10
  noisy sphere      (for the eps and points-per-leaf sweeps) points uniform on
                    the unit sphere plus N(0, sigma^2) on every coordinate, and
                    queries drawn the same way (not planted), as the synthetic
                    Sphere sets of Sec. 4 are described; queries are then
                    nearly equidistant from the points
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

CHUNK = 65536


@dataclass
class Workload:
    name: str
    X: np.ndarray                  # [n, d] float32
    Q: np.ndarray                  # [nq, d] float32
    src: np.ndarray                # [nq] int64, the point each query was planted at
    m: int
    t: int
    p: int
    c: int
    k: int
    seed: int
    checks: np.ndarray | None = None   # per-query budgets, when they vary
    extra: dict = field(default_factory=dict)


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _fill_rows(n: int, d: int, data_ss: np.random.SeedSequence, make_chunk) -> np.ndarray:
    """Fill an [n, d] float32 matrix chunk by chunk, each chunk from its own
    spawned generator; make_chunk(rng, rows, d) returns float32 [rows, d]."""
    nchunks = max(1, math.ceil(n / CHUNK))
    kids = data_ss.spawn(nchunks)
    X = np.empty((n, d), dtype=np.float32)

    def work(ci):
        a = ci * CHUNK
        b = min(n, a + CHUNK)
        X[a:b] = make_chunk(np.random.default_rng(kids[ci]), b - a, d)

    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(work, range(nchunks)))
    return X


def _normalise_rows(A: np.ndarray) -> np.ndarray:
    nrm = np.sqrt(np.einsum("ij,ij->i", A, A, dtype=np.float32))
    nrm[nrm == 0] = 1.0
    return (A / nrm[:, None]).astype(np.float32)


def gauss(n: int, d: int, nq: int, noise: float, seed: int, boost_dims: int = 0,
          boost: float = 1.0):
    """iid N(0,1) points (optionally `boost_dims` random columns scaled by
    `boost`); queries = a random point + iid N(0, noise^2)."""
    root = np.random.SeedSequence(seed)
    par_ss, data_ss, q_ss = root.spawn(3)
    scale = None
    if boost_dims > 0:
        prng = np.random.default_rng(par_ss)
        cols = prng.choice(d, boost_dims, replace=False)
        scale = np.ones(d, dtype=np.float32)
        scale[cols] = boost

    def chunk(rng, rows, dd):
        a = rng.standard_normal((rows, dd), dtype=np.float32)
        if scale is not None:
            a *= scale
        return a

    X = _fill_rows(n, d, data_ss, chunk)
    qrng = np.random.default_rng(q_ss)
    src = qrng.integers(0, n, nq)
    Q = (X[src] + noise * qrng.standard_normal((nq, d), dtype=np.float32)).astype(np.float32)
    return X, Q, src


def sphere(n: int, d: int, nq: int, qdist: float, seed: int):
    """Points uniform on the unit sphere (normalised Gaussians); each query is
    a random point moved by `qdist` along a uniform random direction."""
    root = np.random.SeedSequence(seed)
    _, data_ss, q_ss = root.spawn(3)
    X = _fill_rows(n, d, data_ss,
                   lambda rng, rows, dd: _normalise_rows(rng.standard_normal((rows, dd),
                                                                             dtype=np.float32)))
    qrng = np.random.default_rng(q_ss)
    src = qrng.integers(0, n, nq)
    u = _normalise_rows(qrng.standard_normal((nq, d), dtype=np.float32))
    Q = (X[src] + qdist * u).astype(np.float32)
    return X, Q, src


def noisy_sphere(n: int, d: int, nq: int, sigma: float, seed: int):
    """Points and queries alike: uniform on the unit sphere, then N(0, sigma^2)
    added to every coordinate.  Returns X, Q (no planted source)."""
    root = np.random.SeedSequence(seed)
    _, data_ss, q_ss = root.spawn(3)

    def chunk(rng, rows, dd):
        u = _normalise_rows(rng.standard_normal((rows, dd), dtype=np.float32))
        return (u + sigma * rng.standard_normal((rows, dd), dtype=np.float32)).astype(np.float32)

    X = _fill_rows(n, d, data_ss, chunk)
    Q = chunk(np.random.default_rng(q_ss), nq, d)
    return X, Q


def descriptor(n: int, d: int, nq: int, noise: float, seed: int):
    """Descriptor-like rows |N(0,1)| * s_j, s_j ~ LogNormal(0, 0.5) per column
    (drawn first), L2-normalised; queries = point + N(0, noise^2)."""
    root = np.random.SeedSequence(seed)
    par_ss, data_ss, q_ss = root.spawn(3)
    s = np.random.default_rng(par_ss).lognormal(0.0, 0.5, d).astype(np.float32)

    def chunk(rng, rows, dd):
        a = np.abs(rng.standard_normal((rows, dd), dtype=np.float32)) * s
        return _normalise_rows(a)

    X = _fill_rows(n, d, data_ss, chunk)
    qrng = np.random.default_rng(q_ss)
    src = qrng.integers(0, n, nq)
    Q = (X[src] + noise * qrng.standard_normal((nq, d), dtype=np.float32)).astype(np.float32)
    return X, Q, src


def make(name: str, n: int | None = None, nq: int | None = None) -> Workload:
    """One of the named workloads; `n` / `nq` shrink it (same recipe, same
    seed) for tests that need a smaller instance."""
    if name == "gauss-10k-128":
        n = n or 10_000
        X, Q, src = gauss(n, 128, nq or 100, 0.05, 0)
        return Workload(name, X, Q, src, m=4, t=5, p=8, c=256, k=1, seed=0)
    if name == "sphere-100k-1000":
        n = n or 100_000
        X, Q, src = sphere(n, 1000, nq or 1000, 0.3, 1)
        return Workload(name, X, Q, src, m=8, t=5, p=16, c=1024, k=1, seed=1)
    if name == "desc-1m-960":
        n = n or 1_000_000
        X, Q, src = descriptor(n, 960, nq or 10_000, 0.02, 2)
        return Workload(name, X, Q, src, m=16, t=5, p=32, c=4096, k=10, seed=2)
    if name == "gauss-200k-10000":
        n = n or 200_000
        X, Q, src = gauss(n, 10_000, nq or 2000, 0.05, 4, boost_dims=500, boost=10.0)
        return Workload(name, X, Q, src, m=16, t=10, p=16, c=2048, k=10, seed=4)
    raise KeyError(name)


def multi_index(seed: int = 3, count: int = 20, scale: float = 1.0):
    """The uneven batch: `count` indexes with n log-uniform in [1e4, 5e5]
    (times `scale`, for smaller test instances), d drawn from {128, 512, 960,
    2048}, iid N(0,1) points; 100..5,000 queries each (times `scale`), each
    with its own budget uniform in [256, 8192].  m=8 t=5 p=16 k=10."""
    root = np.random.SeedSequence(seed)
    par_ss, *idx_ss = root.spawn(count + 1)
    prng = np.random.default_rng(par_ss)
    out = []
    for i in range(count):
        n = int(round(math.exp(prng.uniform(math.log(1e4), math.log(5e5))) * scale))
        d = int(prng.choice([128, 512, 960, 2048]))
        nq = int(max(1, round(prng.integers(100, 5001) * scale)))
        n = max(n, 64)
        seed_i = int(idx_ss[i].generate_state(1)[0])
        X, Q, src = gauss(n, d, nq, 0.05, seed_i)
        crng = np.random.default_rng(idx_ss[i].spawn(1)[0])
        checks = crng.integers(256, 8193, nq).astype(np.int32)
        out.append(Workload(f"multi-20/{i}", X, Q, src, m=8, t=5, p=16, c=int(checks.max()),
                            k=10, seed=seed_i, checks=checks))
    return out
