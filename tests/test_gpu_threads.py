"""Calls from several host threads at once.  Calls on one forest share its
workspace and wait for each other; calls on different forests run side by
side on their own streams.  Every result must equal the one the same call
gives alone, on both query paths."""
import ctypes
import threading

import numpy as np
import pytest

from paper_1603_09596_amd import geraf

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    geraf.load()


def test_threads_on_shared_and_separate_forests():
    rng = np.random.default_rng(41)
    nq, k, c = 400, 5, 40
    cases = []
    for i, (n, d) in enumerate(((8000, 64), (5000, 200))):
        X = rng.standard_normal((n, d)).astype(np.float32)
        Q = (X[rng.integers(0, n, nq)] + 0.1 * rng.standard_normal((nq, d))).astype(np.float32)
        cases.append((geraf.build_forest(X, 4, 5, 8, 50 + i, forms=("bf16",)), Q))
    kinds = [(ci, form) for ci in (0, 1) for form in ("fp32", "bf16")]

    def run(kind, stream=None):
        F, Q = cases[kind[0]]
        ids = np.zeros((nq, k), np.int32)
        dd = np.zeros((nq, k), np.float32)
        geraf.query(F, Q, k, c, ids, dd, form=kind[1], stream=stream)
        return ids, dd, geraf.last_query_timing()["path"]

    try:
        ref = {kind: run(kind) for kind in kinds}
        assert {r[2] for r in ref.values()} == {"rows", "tile"}
        results, errors = {}, []

        def worker(tid):
            try:
                st = torch.cuda.Stream(device="cuda:0")
                for rep in range(3):
                    kind = kinds[(tid + rep) % len(kinds)]
                    results[(tid, rep)] = (kind, run(kind, ctypes.c_void_p(st.cuda_stream)))
            except Exception as e:  # reported below
                errors.append(repr(e))

        threads = [threading.Thread(target=worker, args=(t,)) for t in range(4)]
        for t in threads:
            t.start()
        for t in threads:
            t.join(timeout=120)
        assert not errors, errors
        assert len(results) == 12
        for (tid, rep), (kind, got) in results.items():
            assert np.array_equal(got[0], ref[kind][0]), (tid, rep, kind)
            assert np.array_equal(got[1], ref[kind][1]), (tid, rep, kind)
            assert got[2] == ref[kind][2]
    finally:
        for F, _ in cases:
            F.free()
