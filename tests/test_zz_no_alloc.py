"""gf_query_noalloc (the allocation-free variant of gf_query, whose workspace
is the library's static device array) against gf_query on the same path.

Each case makes two calls in a row, the second with fewer queries, and both
must equal gf_query's row path exactly (the same kernels run); one case has
more queries than one scratch-sized batch holds, and one uses per-query
device budgets.  The outputs are also checked against the FP64 oracle."""
import numpy as np
import pytest

import oracle
from paper_1603_09596_amd import geraf
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


def run(fn, F, Q, k, c, form, cpq=None):
    nq = Q.shape[0]
    ids = torch.full((nq, k), -9, dtype=torch.int32, device="cuda:0")
    dd = torch.full((nq, k), -9.0, dtype=torch.float32, device="cuda:0")
    fn(F, Q, k, c, ids, dd, checks_per_query=cpq, form=form)
    torch.cuda.synchronize()
    return ids.cpu().numpy(), dd.cpu().numpy()


@pytest.mark.parametrize("form,nq,nq2,c", [("fp32", 300, 41, 120), ("bf16", 700, 130, 300),
                                           ("fp8", 200, 7, 90), ("fp32", 2600, 5, 64)])
def test_noalloc_equals_query_on_two_calls(form, nq, nq2, c, monkeypatch):
    monkeypatch.setenv("GF_SCAN_PATH", "rows")
    rng = np.random.default_rng(nq)
    n, d = 20_000, 96
    X = rng.standard_normal((n, d)).astype(np.float32)
    Qa = (X[rng.integers(0, n, nq)] + 0.05 * rng.standard_normal((nq, d))).astype(np.float32)
    Qb = (X[rng.integers(0, n, nq2)] + 0.05 * rng.standard_normal((nq2, d))).astype(np.float32)
    forms = () if form == "fp32" else (form,)
    F = geraf.build_forest(X, 8, 5, 8, 21, forms=forms)
    Fo = oracle.build_forest(X, 8, 5, 8, 21)
    try:
        for Q in (Qa, Qb):                    # the second call is the smaller one
            Qd = dev(Q)
            got = run(geraf.query_noalloc, F, Qd, 10, c, form)
            ref = run(geraf.query, F, Qd, 10, c, form)
            assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
            sample = np.linspace(0, len(Q) - 1, 12).astype(np.int64)
            Qs = np.ascontiguousarray(Q[sample])
            r = oracle.search(Fo, X, Qs, 10, c, trace=False, candidates=True)
            if form == "fp32":
                check_knn(got[0][sample], got[1][sample], r["ids"], r["dists"], X=X, Q=Qs,
                          cand=r["cand"])
            else:
                for j, i in enumerate(sample):
                    g = got[0][i][got[0][i] >= 0]
                    assert np.isin(g, r["cand"][j]).all()
    finally:
        F.free()


def test_noalloc_per_query_budgets_and_deep_collect(monkeypatch):
    """Per-query device budgets on a forest whose selection takes radix
    passes and deeper tie levels (integer data)."""
    monkeypatch.setenv("GF_SCAN_PATH", "rows")
    rng = np.random.default_rng(8)
    X = rng.integers(0, 4, (65536, 8)).astype(np.float32)
    Q = (X[rng.integers(0, 65536, 24)] + rng.integers(-1, 2, (24, 8)) + 0.5).astype(np.float32)
    F = geraf.build_forest(X, 2, 4, 1, 3)
    try:
        cpq = dev(rng.integers(1, 60_000, 24).astype(np.int32))
        for Q2 in (Q, Q[:9]):
            Qd = dev(Q2)
            c2 = cpq[:len(Q2)].contiguous()
            got = run(geraf.query_noalloc, F, Qd, 5, 1, "fp32", cpq=c2)
            ref = run(geraf.query, F, Qd, 5, 1, "fp32", cpq=c2)
            assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
    finally:
        F.free()


def test_noalloc_rejects_host_buffers():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((1000, 8)).astype(np.float32)
    F = geraf.build_forest(X, 2, 3, 8, 1)
    try:
        Q = X[:4].copy()
        with pytest.raises(geraf.GerafError) as e:
            geraf.query_noalloc(F, Q, 3, 10, np.zeros((4, 3), np.int32), np.zeros((4, 3), np.float32))
        assert e.value.status == geraf.GF_EINVAL
    finally:
        F.free()
