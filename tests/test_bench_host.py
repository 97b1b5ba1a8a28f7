"""Host logic of bench.py: the single-GPU guard and the algorithmic byte
model behind roofline.achieved on the row path (no GPU needed)."""
import os
import subprocess
import sys
from types import SimpleNamespace

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


@pytest.mark.parametrize("form,row", [("fp32", 1000 * 4), ("bf16", 1024 * 2 + 4), ("fp8", 1008 + 8)])
def test_scan_bytes_per_candidate_row(form, row):
    # d = 1000: FP32 rows padded to 1000 floats, BF16 to 1024 (one MFMA k
    # step is 32), FP8 to 1008 bytes plus the row's scale and norm
    F = SimpleNamespace(d=1000, n=4096, H=8, m=4, leaf_words=8)
    base = bench.scan_bytes_per_launch(F, 3, 0, form, 10, 40, 64)
    more = bench.scan_bytes_per_launch(F, 3, 7, form, 10, 40, 64)
    assert more - base == 7 * row


def test_scan_bytes_count_rerank_only_for_reduced_forms():
    F = SimpleNamespace(d=960, n=1 << 20, H=15, m=16, leaf_words=1024)
    nq, kk = 5, 40
    b32 = bench.scan_bytes_per_launch(F, nq, 0, "fp32", 10, kk, 1)
    b16 = bench.scan_bytes_per_launch(F, nq, 0, "bf16", 10, kk, 1)
    # query rows differ by the BF16 copy (960 x 2 B); the re-rank reads kk FP32 rows
    assert b16 - b32 == nq * 960 * 2 + nq * kk * 960 * 4


def test_nn_quality_tie_rule_and_eps_bound():
    # squared distances: exact nearest 1, 4, 9, 16; reported 1 (exact), 4 up
    # to a last-bit difference (a tie counts as correct), 9.5, no answer
    d_true = [1.0, 4.0, 9.0, 16.0]
    d_got = [1.0, 4.0 * (1 + 1e-15), 9.5, float("inf")]
    miss, fail = bench.nn_quality(d_true, d_got, 0.0)
    assert miss == pytest.approx(50.0) and fail == pytest.approx(50.0)
    # eps = 0.1 bounds the distance by 1.1 * 3 = 3.3, i.e. the square by 10.89
    miss, fail = bench.nn_quality(d_true, d_got, 0.1)
    assert miss == pytest.approx(50.0) and fail == pytest.approx(25.0)
    miss, fail = bench.nn_quality([9.0], [9.0 * 1.1 ** 2], 0.1)
    assert fail == 0.0 and miss == 100.0
    _, fail = bench.nn_quality([9.0], [9.0 * 1.1 ** 2 * (1 + 1e-9)], 0.1)
    assert fail == 100.0


def test_sweep_settings_cover_the_paper_tables():
    # the four eps values and the eight points-per-leaf values of the tables
    assert bench.SWEEPS["eps"]["eps"] == (0.0, 0.1, 0.5, 0.9)
    assert bench.SWEEPS["p"]["p"] == (256, 128, 64, 32, 16, 4, 2, 1)
    # the budget grid starts at the smallest c of the protocol and holds the headline c
    b = bench.SWEEPS["c"]["budgets"]
    assert b[0] == 4096 and bench.CHECKS_AT_090 in b and list(b) == sorted(set(b))


def test_pmc_traffic_reads_the_record_of_the_named_kernel():
    # the committed records: the tile kernel of the headline workload and the
    # FP8 scan of the 10,000-dim one; no record for an unknown kernel
    for kernel, workload in (("k_tile_bf16", "desc-1m-960"), ("k_scan (fp8)", "gauss-200k-10000")):
        v = bench.pmc_traffic(kernel, workload)
        assert v is None or v > 1e9
    assert bench.pmc_traffic("no_such_kernel", "desc-1m-960") is None


def test_pmc_traffic_is_null_once_kernel_or_launch_source_changes(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    (tmp_path / "k.hip").write_text("kernel v1")
    (tmp_path / "l.hip").write_text("launch v1")
    import hashlib
    h = lambda t: hashlib.sha256(t.encode()).hexdigest()
    rec = ("kernel: k_x\nsource_file: k.hip\nsource_sha256: %s\n"
           "launch_file: l.hip\nlaunch_sha256: %s\nhbm_bytes_per_dispatch: 5000000000\n")
    (tmp_path / "profiles" / "pmc_w.txt").write_text(rec % (h("kernel v1"), h("launch v1")))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.pmc_traffic("k_x", "w") == 5e9
    (tmp_path / "l.hip").write_text("launch v2")
    assert bench.pmc_traffic("k_x", "w") is None
    (tmp_path / "l.hip").write_text("launch v1")
    (tmp_path / "k.hip").write_text("kernel v2")
    assert bench.pmc_traffic("k_x", "w") is None


def test_vs_oracle_recall_and_distance_errors():
    import numpy as np
    X = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 2.0], [3.0, 0.0]], np.float32)
    Q = np.array([[0.0, 0.0], [1.0, 0.0]], np.float32)
    # oracle's 2 best: query 0 -> ids 0, 1; query 1 -> ids 1, 0
    ref = {"ids": np.array([[0, 1], [1, 0]]), "dists": np.array([[0.0, 1.0], [0.0, 1.0]])}
    ids = np.array([[0, 1], [1, 3]], np.int32)           # query 1 misses id 0
    dists = np.array([[0.0, 1.0], [0.0, 4.0 * (1 + 1e-6)]], np.float32)
    out = bench.vs_oracle(X, Q, ids, dists, ref)
    assert out["recall@2"] == pytest.approx(0.75)
    assert out["queries"] == 2
    assert 5e-7 < out["max_rel_dist_err"] < 2e-6
