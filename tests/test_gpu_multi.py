"""The multi-index launch (gf_query_multi) against single gf_query calls and
the oracle.

Each job of a multi call must give exactly what gf_query gives for the same
arguments on the same path (the same kernels run, launched from one graph),
in graph mode and eagerly, on the first call and when a cached graph is
reused, also over several replays with eager calls between them.  An FP32 job is also checked against the FP64 oracle by the
acceptance rule, and the autotuned choice must reproduce one of the two
single-call paths.
"""
import numpy as np
import pytest

import oracle
from paper_1603_09596_amd import geraf, workloads as W
from parity import check_knn

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    geraf.load()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


@pytest.fixture(scope="module")
def indexes():
    """Six indexes of uneven n and d (the multi-20 recipe at 1/20 scale)
    plus one BF16 index big enough in queries for the tile path."""
    ws = W.multi_index(seed=3, count=6, scale=0.05)
    out = []
    for i, w in enumerate(ws):
        form = ("fp32", "bf16", "fp8")[i % 3]
        forms = {"fp32": (), "bf16": ("bf16",), "fp8": ("fp8",)}[form]
        F = geraf.build_forest(w.X, w.m, w.t, w.p, w.seed, forms=forms)
        out.append(dict(w=w, F=F, form=form, checks=w.checks, scalar=None))
    # one budget for the whole job: the path rule can then see the candidate share
    X, Q, _ = W.descriptor(30_000, 256, 300, 0.02, 11)
    F = geraf.build_forest(X, 8, 5, 16, 11, forms=("bf16",))
    w = W.Workload("desc-30k-256", X, Q, np.arange(len(Q)), m=8, t=5, p=16, c=1024, k=10, seed=11,
                   checks=np.full(len(Q), 1024, np.int32))
    out.append(dict(w=w, F=F, form="bf16", checks=w.checks, scalar=1024))
    yield out
    for e in out:
        e["F"].free()


def jobs_of(indexes):
    jobs = []
    for e in indexes:
        w = e["w"]
        nq = len(w.Q)
        per_q = None if e["scalar"] else dev(e["checks"])
        jobs.append(dict(forest=e["F"], Q=dev(w.Q), k=w.k, checks=e["scalar"] or 1,
                         checks_per_query=per_q, form=e["form"],
                         ids=torch.full((nq, w.k), -7, dtype=torch.int32, device="cuda:0"),
                         dists=torch.full((nq, w.k), -7.0, dtype=torch.float32, device="cuda:0")))
    return jobs


def single(e):
    w = e["w"]
    nq = len(w.Q)
    ids = torch.empty((nq, w.k), dtype=torch.int32, device="cuda:0")
    dd = torch.empty((nq, w.k), dtype=torch.float32, device="cuda:0")
    per_q = None if e["scalar"] else dev(e["checks"])
    geraf.query(e["F"], dev(w.Q), w.k, e["scalar"] or 1, ids, dd, checks_per_query=per_q,
                form=e["form"])
    torch.cuda.synchronize()
    return ids.cpu().numpy(), dd.cpu().numpy(), geraf.last_query_timing()["path"]


def test_multi_equals_single_calls(indexes):
    ref = [single(e) for e in indexes]
    assert any(r[2] == "tile" for r in ref), "no job took the tile path"
    before = geraf.multi_stats()
    for eager in (False, True):
        jobs = jobs_of(indexes)
        geraf.query_multi(jobs, eager=eager)
        torch.cuda.synchronize()
        for e, j, r in zip(indexes, jobs, ref):
            assert np.array_equal(j["ids"].cpu().numpy(), r[0]), e["w"].name
            assert np.array_equal(j["dists"].cpu().numpy(), r[1]), e["w"].name
    after = geraf.multi_stats()
    assert after["graphs_built"] == before["graphs_built"] + 1


def test_multi_graph_reuse(indexes):
    jobs = jobs_of(indexes)
    geraf.query_multi(jobs)
    first = [(j["ids"].cpu().numpy().copy(), j["dists"].cpu().numpy().copy()) for j in jobs]
    before = geraf.multi_stats()
    for j in jobs:
        j["ids"].fill_(-3)
        j["dists"].fill_(-3.0)
    geraf.query_multi(jobs)
    after = geraf.multi_stats()
    assert after["graphs_reused"] == before["graphs_reused"] + 1
    assert after["graphs_built"] == before["graphs_built"]
    for j, f in zip(jobs, first):
        assert np.array_equal(j["ids"].cpu().numpy(), f[0])
        assert np.array_equal(j["dists"].cpu().numpy(), f[1])


def test_multi_graph_replays_match_eager(indexes):
    """Four launches of one cached graph, with eager single-index calls and
    host synchronisations between them: every replay must reproduce the
    eager results exactly (replays after the first start from the
    workspace contents the previous call and the eager work left)."""
    ref = [single(e) for e in indexes]
    jobs = jobs_of(indexes)
    geraf.query_multi(jobs)
    torch.cuda.synchronize()
    before = geraf.multi_stats()
    for rep in range(4):
        for j in jobs:
            j["ids"].fill_(-3 - rep)
            j["dists"].fill_(-3.0 - rep)
        geraf.query_multi(jobs)
        torch.cuda.synchronize()
        for e, j, r in zip(indexes, jobs, ref):
            assert np.array_equal(j["ids"].cpu().numpy(), r[0]), (rep, e["w"].name)
            assert np.array_equal(j["dists"].cpu().numpy(), r[1]), (rep, e["w"].name)
        # the program's own eager work between replays, on the same forests
        e = indexes[rep % len(indexes)]
        got = single(e)
        r = ref[rep % len(indexes)]
        assert np.array_equal(got[0], r[0]) and np.array_equal(got[1], r[1])
    after = geraf.multi_stats()
    assert after["graphs_reused"] == before["graphs_reused"] + 4
    assert after["graphs_built"] == before["graphs_built"]


def test_multi_every_job_against_oracle(indexes):
    """Every job of one graph launch against the FP64 oracle on a sample of
    its queries (each with its own budget): FP32 jobs by the acceptance rule,
    BF16 / FP8 jobs by exact returned distances and recall; in every form a
    returned id must be one of the query's candidates."""
    jobs = jobs_of(indexes)
    geraf.query_multi(jobs)
    torch.cuda.synchronize()
    for e, j in zip(indexes, jobs):
        w = e["w"]
        Fo = oracle.build_forest(w.X, w.m, w.t, w.p, w.seed)
        got_i, got_d = j["ids"].cpu().numpy(), j["dists"].cpu().numpy()
        sample = np.linspace(0, len(w.Q) - 1, min(len(w.Q), 24)).astype(np.int64)
        hits = total = 0
        for i in sample:
            Qs = np.ascontiguousarray(w.Q[i:i + 1])
            ref = oracle.search(Fo, w.X, Qs, w.k, int(w.checks[i]), trace=False, candidates=True)
            if e["form"] == "fp32":
                check_knn(got_i[i:i + 1], got_d[i:i + 1], ref["ids"], ref["dists"], X=w.X, Q=Qs,
                          cand=ref["cand"])
                continue
            got = got_i[i][got_i[i] >= 0]
            assert np.isin(got, ref["cand"][0]).all(), (w.name, int(i))
            for r, gid in enumerate(got.tolist()):
                diff = w.X[gid].astype(np.float64) - Qs[0].astype(np.float64)
                true_d = float(diff @ diff)
                assert abs(got_d[i][r] - true_d) <= 1e-5 * true_d, (w.name, int(i))
            hits += len(set(got.tolist()) & set(ref["ids"][0][ref["ids"][0] >= 0].tolist()))
            total += int((ref["ids"][0] >= 0).sum())
        if total:
            print(f"{w.name} {e['form']}: recall vs FP64 oracle {hits / total:.4f}")
            assert hits / total >= 0.95, w.name


def test_multi_graph_64_replays_with_radix_passes():
    """A budget of 37 leaves on quantised data sends queries through radix
    passes (and their list of queries) in every replay.  64 launches of the
    cached graph with nothing between them must all equal the eager call."""
    rng = np.random.default_rng(5)
    X = rng.integers(0, 8, (5000, 40)).astype(np.float32)
    Q = (X[rng.integers(0, 5000, 60)] + rng.integers(-1, 2, (60, 40))).astype(np.float32)
    F = geraf.build_forest(X, 4, 6, 8, 1234 + len("quantised"))
    try:
        e = dict(w=W.Workload("quantised", X, Q, np.arange(60), m=4, t=6, p=8, c=37, k=5,
                              seed=0, checks=np.full(60, 37, np.int32)),
                 F=F, form="fp32", checks=np.full(60, 37, np.int32), scalar=37)
        r = single(e)
        jobs = jobs_of([e])
        geraf.query_multi(jobs)
        torch.cuda.synchronize()
        for rep in range(64):
            jobs[0]["ids"].fill_(-3)
            jobs[0]["dists"].fill_(-3.0)
            geraf.query_multi(jobs)
            assert np.array_equal(jobs[0]["ids"].cpu().numpy(), r[0]), rep
            assert np.array_equal(jobs[0]["dists"].cpu().numpy(), r[1]), rep
    finally:
        F.free()


def test_multi_autotune_matches_a_path(indexes, monkeypatch):
    e = indexes[-1]
    per_path = {}
    for path in ("rows", "tile"):
        monkeypatch.setenv("GF_SCAN_PATH", path)
        per_path[path] = single(e)
    monkeypatch.delenv("GF_SCAN_PATH")
    before = geraf.multi_stats()
    jobs = jobs_of([e])
    geraf.query_multi(jobs, autotune=True)
    after = geraf.multi_stats()
    assert after["tuned"] == before["tuned"] + 1
    got_i, got_d = jobs[0]["ids"].cpu().numpy(), jobs[0]["dists"].cpu().numpy()
    assert any(np.array_equal(got_i, r[0]) and np.array_equal(got_d, r[1]) for r in per_path.values())
    geraf.query_multi(jobs, autotune=True)   # the choice is kept: nothing measured again
    assert geraf.multi_stats()["tuned"] == after["tuned"]


def test_multi_rejects_nan_before_running(indexes):
    jobs = jobs_of(indexes[:2])
    jobs[1]["Q"][0, 0] = float("nan")
    with pytest.raises(geraf.GerafError):
        geraf.query_multi(jobs)
    assert int(jobs[0]["ids"][0, 0]) == -7   # nothing ran
