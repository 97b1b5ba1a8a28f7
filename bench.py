"""Benchmark of the kd-GeRaF query path on one MI355X.

Workload desc-1m-960: 1,000,000 descriptor-like points in 960 dimensions,
10,000 planted queries, a forest of 16 trees (t = 5, leaf <= 32), k = 10; the
budget c is the smallest tested that reaches recall@10 >= 0.90 (see
CHECKS_AT_090).  A step is one gf_query call over all queries: leaf
selection, candidate expansion, gathers and distances, best-k, re-rank and
tie re-check, with data and queries already in HBM.  The headline value is
the BF16 form; the FP32 form is timed the same way beside it.

Prints one JSON line.  Also reports:
  roofline      the dominant kernel of the path taken: on the tile path the
                MFMA score kernel (2*nq*n*d flops per launch, against 2.5
                PFLOP/s dense BF16), on the row path the scan kernel
                (algorithmic bytes per launch, against 8 TB/s); its mean
                duration comes from HIP events the library records on the
                query stream during the timed steps;
  cpu_baseline  the FP64 oracle, searching a bounded sample of the same
                queries on the host's cores (its own forest build excluded).

`--workload` runs one of the other recipes in its own form and at its own
budget instead (gauss-10k-128 and sphere-100k-1000 in FP32, gauss-200k-10000
in FP8 with FP32 re-rank of the best 40), with the same line and the same
roofline and baseline objects; the FP32 form is timed beside the FP8 one.

`--sweep eps|p` measures accuracy and time against the approximation factor
eps or the points per leaf p on noisy-sphere stand-ins shaped like the
paper's synthetic Sphere sets (k = 1): miss %, eps-failure %, build and
search time per setting, in one line with a row per setting.  `--sweep c`
gives the recall-against-budget curve of the headline recipe (recall@10,
1-recall@10, candidates per query and queries/s per c).

`--multi` measures the multi-index launch instead and prints its own line:
the multi-20 recipe (20 indexes of uneven n and d, per-query budgets,
scaled by --multi-scale), FP32 form, as one gf_query_multi graph launch,
as the same launches issued eagerly, and as one gf_query call per index.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "desc-1m-960"
CHECKS_AT_090 = 114688         # smallest c on a 8192 grid with recall@10 >= 0.90 (oracle 200-query and GPU 500-query samples)
# the form each recipe is measured in (the FP32 form is timed beside the reduced ones)
FORMS = {"desc-1m-960": "bf16", "gauss-200k-10000": "fp8",
         "sphere-100k-1000": "fp32", "gauss-10k-128": "fp32"}
HBM_PEAK_GBS = 8000.0
MFMA_BF16_PEAK_TFLOPS = 2500.0   # MI355X dense BF16
MFMA_FP8_PEAK_TFLOPS = 5000.0    # MI355X dense FP8
TILE_KERNELS = {"bf16": ("k_tile_bf16", MFMA_BF16_PEAK_TFLOPS), "fp8": ("k_tile_fp8", MFMA_FP8_PEAK_TFLOPS)}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_threads() -> int:
    n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        n = min(n, int(env))
    return max(1, n)


def recall_at(ids: np.ndarray, gt: np.ndarray) -> float:
    k = gt.shape[1]
    return float(np.mean([len(set(ids[i].tolist()) & set(gt[i].tolist())) / k
                          for i in range(len(gt))]))


def scan_bytes_per_launch(F, nq, ncand_total, form, k, kk, checks):
    """Algorithmic HBM bytes of one scan launch over nq queries: candidate
    rows (+ their norms), opened leaves' point ids, leaf-bitmap words, the
    FP32 rows re-measured by the re-rank, the query rows, the outputs."""
    ld32 = (F.d + 3) // 4 * 4
    ld16 = (F.d + 31) // 32 * 32
    ld8 = (F.d + 15) // 16 * 16
    if form == "bf16":
        row = ld16 * 2 + 4
        rerank = nq * kk * ld32 * 4
        qrow = ld16 * 2 + ld32 * 4
    elif form == "fp8":
        row = ld8 + 8                      # e4m3 row, its scale and its norm
        rerank = nq * kk * ld32 * 4
        qrow = ld8 + ld32 * 4
    else:
        row = ld32 * 4
        rerank = 0
        qrow = ld32 * 4
    leaf_pts = F.n / (1 << F.H)
    perm = nq * checks * leaf_pts * 4
    bits = nq * F.m * F.leaf_words * 4
    return ncand_total * row + rerank + perm + bits + nq * qrow + nq * k * 8


def nn_quality(d_true, d_got, eps, tie=1e-12):
    """Accuracy of 1-NN answers as Sec. 4 measures it, from squared FP64
    distances: miss % is the share of queries whose reported neighbour is
    farther than the exact nearest (a point at the same distance counts as
    correct); eps-failure % is the share whose reported distance exceeds
    (1 + eps) times the nearest distance (Def. 1).  A query with no answer
    (distance inf) counts as both."""
    d_true = np.asarray(d_true, dtype=np.float64)
    d_got = np.asarray(d_got, dtype=np.float64)
    miss = ~(d_got <= d_true * (1.0 + tie))
    fail = ~(d_got <= d_true * (1.0 + eps) ** 2 * (1.0 + tie))
    return 100.0 * float(miss.mean()), 100.0 * float(fail.mean())


# eps sweep: the two Sphere shapes of the paper's search table; p sweep: the
# shape of its points-per-leaf table (there on a Klein bottle, here a sphere)
SWEEPS = {
    "eps": dict(cases=[(1000, 10000), (100000, 100)], eps=(0.0, 0.1, 0.5, 0.9), p=(16,)),
    "p": dict(cases=[(10000, 100)], eps=(0.0,), p=(256, 128, 64, 32, 16, 4, 2, 1)),
    # recall against the budget on the headline recipe: the curve that fixes its c
    "c": dict(budgets=(4096, 8192, 16384, 32768, 65536, 98304, 106496, 114688, 131072)),
}
SWEEP_M, SWEEP_T, SWEEP_NQ, SWEEP_SEED, SWEEP_SIGMA = 8, 5, 1000, 5, 0.1


def sweep_bench(args, torch, geraf, workloads, dev):
    """eps or p sweep on noisy-sphere stand-ins (FP32 form, k = 1)."""
    from oracle import bruteforce as bf
    spec = SWEEPS[args.sweep]
    m, t, nq, seed = SWEEP_M, SWEEP_T, SWEEP_NQ, SWEEP_SEED
    rows = []
    for n, d in spec["cases"]:
        X, Q = workloads.noisy_sphere(n, d, nq, SWEEP_SIGMA, seed)
        _, gt_d = bf.knn_ground_truth(X, Q, 1)
        Qd = torch.from_numpy(Q).to(dev)
        ids = torch.empty((nq, 1), dtype=torch.int32, device=dev)
        dd = torch.empty((nq, 1), dtype=torch.float32, device=dev)
        for p in spec["p"]:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            F = geraf.build_forest(X, m, t, p, seed)
            torch.cuda.synchronize()
            build_s = time.perf_counter() - t0
            leaves = m << F.H
            c = args.checks if args.checks is not None else (
                256 if args.sweep == "p" else max(1, leaves // 16))
            for eps in spec["eps"]:
                geraf.query(F, Qd, 1, c, ids, dd, eps=eps)
                torch.cuda.synchronize()
                times = []
                for _ in range(max(1, args.steps)):
                    t0 = time.perf_counter()
                    geraf.query(F, Qd, 1, c, ids, dd, eps=eps)
                    torch.cuda.synchronize()
                    times.append(time.perf_counter() - t0)
                ms = 1e3 * float(np.median(times))
                got = ids.cpu().numpy()[:, 0].astype(np.int64)
                d_got = np.full(nq, np.inf)
                ok = got >= 0
                diff = X[got[ok]].astype(np.float64) - Q[ok].astype(np.float64)
                d_got[ok] = np.einsum("ij,ij->i", diff, diff)
                miss, fail = nn_quality(gt_d[:, 0], d_got, eps)
                budget = min(int(np.ceil(c / (1.0 + eps))), leaves)
                rows.append(dict(dataset=f"noisy-sphere-{n}x{d}", n=n, d=d, p=p, H=int(F.H),
                                 eps=eps, checks=c, leaves_opened=budget,
                                 build_s=round(build_s, 4), search_ms=round(ms, 3),
                                 us_per_query=round(1e3 * ms / nq, 3),
                                 miss_pct=round(miss, 1), eps_fail_pct=round(fail, 1)))
                log(f"[bench] sweep {rows[-1]}")
            F.free()
    first = rows[0]
    out = {
        "metric": f"{args.sweep} sweep: miss %, eps-failure % and search time (noisy-sphere)",
        "value": round(nq / (first["search_ms"] / 1e3), 2), "unit": "queries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": first["search_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"noisy-sphere {args.sweep} sweep", "m": m, "t": t, "k": 1,
                   "nq": nq, "sigma": SWEEP_SIGMA, "seed": seed, "form": "fp32"},
        "rows": rows,
    }
    print(json.dumps(out), flush=True)


def c_sweep_bench(args, torch, geraf, workloads, dev):
    """recall@10, 1-recall@10, candidates per query and queries/s against the
    budget c on the headline recipe (desc-1m-960, BF16 form with FP32
    re-rank of 4k): the curve from which the headline c is the smallest
    budget on the grid reaching recall@10 >= 0.90."""
    from oracle import bruteforce as bf
    w = workloads.make(WORKLOAD, nq=args.nq)
    F = geraf.build_forest(w.X, w.m, w.t, w.p, w.seed, forms=("bf16",))
    Q = torch.from_numpy(w.Q).to(dev)
    nq, k = len(w.Q), w.k
    idx = np.linspace(0, nq - 1, min(args.recall_sample, nq)).astype(np.int64)
    gt, _ = bf.knn_ground_truth(w.X, w.Q[idx], k)
    Qs = torch.from_numpy(np.ascontiguousarray(w.Q[idx])).to(dev)
    ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
    dists = torch.empty((nq, k), dtype=torch.float32, device=dev)
    nc = torch.empty(len(idx), dtype=torch.int64, device=dev)
    rows = []
    for c in SWEEPS["c"]["budgets"]:
        geraf.query(F, Q, k, c, ids, dists, form="bf16")
        torch.cuda.synchronize()
        times = []
        for _ in range(max(1, args.steps)):
            t0 = time.perf_counter()
            geraf.query(F, Q, k, c, ids, dists, form="bf16")
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        path = geraf.last_query_timing()["path"]
        ms = 1e3 * float(np.median(times))
        got = ids.cpu().numpy()[idx]
        geraf.query_trace(F, Qs, c, ncand=nc)
        torch.cuda.synchronize()
        one = float(np.mean([gt[i, 0] in set(got[i].tolist()) for i in range(len(idx))]))
        rows.append(dict(checks=c, **{f"recall@{k}": round(recall_at(got, gt), 4),
                                     f"1-recall@{k}": round(one, 4)},
                         mean_candidates=round(float(nc.float().mean().item()), 1),
                         path=path, ms=round(ms, 2), queries_per_s=round(nq / (ms / 1e3), 1)))
        log(f"[bench] c sweep {rows[-1]}")
    F.free()
    head = next(r for r in rows if r["checks"] == CHECKS_AT_090)
    out = {
        "metric": f"recall@{k} and queries/s against the budget c, {WORKLOAD}, BF16 form",
        "value": head["queries_per_s"], "unit": "queries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": head["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": f"{WORKLOAD} c sweep", "nq": nq, "k": k, "form": "bf16",
                   "recall_sample": len(idx)},
        "rows": rows,
    }
    print(json.dumps(out), flush=True)


def pmc_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from a committed rocprofv3 --pmc
    summary of `workload` (profiles/pmc_<workload>.txt or
    profiles/pmc_<workload>_<part>.txt), or None when none records that
    kernel, or the one that does was taken on a different source of it (the
    kernel's source_file and, where recorded, the launch_file that chooses
    its launch shape)."""
    import glob
    paths = sorted(glob.glob(os.path.join(ROOT, "profiles", f"pmc_{glob.escape(workload)}*.txt")))
    for path in paths:
        vals = {}
        for line in open(path):
            if ":" in line:
                key, v = line.split(":", 1)
                vals[key.strip()] = v.strip()
        src = vals.get("source_file")
        if vals.get("kernel") != kernel or not src:
            continue
        for fkey, hkey in (("source_file", "source_sha256"), ("launch_file", "launch_sha256")):
            f = vals.get(fkey)
            if f is None:
                continue
            cur = hashlib.sha256(open(os.path.join(ROOT, f), "rb").read()).hexdigest()
            if vals.get(hkey) != cur:
                return None
        try:
            return float(vals["hbm_bytes_per_dispatch"])
        except (KeyError, ValueError):
            return None
    return None


def cpu_baseline(w, idx_all, checks, seconds, threads, householder=False):
    import oracle
    t0 = time.perf_counter()
    F = oracle.build_forest(w.X, w.m, w.t, w.p, w.seed, nthreads=threads,
                            householder_variant=householder)
    log(f"[bench] oracle build {time.perf_counter() - t0:.1f}s")
    # calibrate on one query per thread, then size the sample to ~`seconds`
    probe = idx_all[:threads]
    t0 = time.perf_counter()
    oracle.search(F, w.X, w.Q[probe], w.k, checks, nthreads=threads, trace=False)
    dt = time.perf_counter() - t0
    per_q = dt / len(probe)
    nsample = int(max(threads, min(len(idx_all), seconds / max(per_q, 1e-9))))
    nsample = (nsample + threads - 1) // threads * threads
    sample = idx_all[:nsample]
    t0 = time.perf_counter()
    ref = oracle.search(F, w.X, w.Q[sample], w.k, checks, nthreads=threads, trace=False)
    dt = time.perf_counter() - t0
    # one thread, on the first queries of the same sample (about 5 s)
    n1 = int(max(1, min(len(sample), 5.0 / max(per_q * threads, 1e-9))))
    t0 = time.perf_counter()
    oracle.search(F, w.X, w.Q[sample[:n1]], w.k, checks, nthreads=1, trace=False)
    dt1 = time.perf_counter() - t0
    return dict(value=round(len(sample) / dt, 3), unit="queries/s", cores=threads, kind="oracle",
                single_thread=dict(value=round(n1 / dt1, 3), queries=n1),
                sample=f"first {len(sample)} of the {len(w.Q)} queries (evenly spaced), "
                       f"c={checks}, k={w.k}; FP64 sequential queue per query, one query per "
                       f"thread; forest build excluded"), sample, ref


def hbm_probe(torch, geraf, dev, gib=4, reps=5):
    """Streaming read bandwidth of this machine, beside the 8 TB/s peak: the
    library's read probe (gf_hbm_probe: 16-byte non-temporal loads over
    contiguous 64 KB spans, sixteen in flight per thread, nothing written)
    over a `gib` GiB device buffer, `reps` timed launches after a warm-up."""
    buf = torch.empty(gib << 30, dtype=torch.uint8, device=dev)
    rate = geraf.hbm_probe(buf, reps)
    torch.cuda.synchronize()
    del buf
    torch.cuda.empty_cache()
    return {"read_GB_s": round(rate, 1), "frac_of_peak": round(rate / HBM_PEAK_GBS, 4),
            "gib": gib, "kernel": "k_read_probe"}


def vs_oracle(X, Q, ids, dists, ref):
    """The GPU answers of the oracle's sample against the oracle: recall of
    the oracle's k (its FP64 top-k at the same budget) and the relative error
    of every returned distance against its FP64 value."""
    hits, errs = 0, []
    for j in range(len(Q)):
        got = ids[j][ids[j] >= 0]
        hits += len(set(got.tolist()) & set(ref["ids"][j][ref["ids"][j] >= 0].tolist()))
        for r, gid in enumerate(got.tolist()):
            diff = X[gid].astype(np.float64) - Q[j].astype(np.float64)
            true_d = float(diff @ diff)
            errs.append(abs(float(dists[j][r]) - true_d) / true_d if true_d > 0 else 0.0)
    n_ref = max(1, int((ref["ids"] >= 0).sum()))
    return {f"recall@{ids.shape[1]}": round(hits / n_ref, 4),
            "max_rel_dist_err": float(f"{max(errs):.3g}") if errs else 0.0,
            "mean_rel_dist_err": float(f"{np.mean(errs):.3g}") if errs else 0.0,
            "queries": len(Q)}


def multi_bench(args, torch, geraf, workloads, dev):
    """The multi-index launch over the multi-20 recipe: FP32 and BF16 jobs
    (alternating by index), per-query budgets, as one gf_query_multi graph
    launch (path by rule, then autotuned), as the same launches issued
    eagerly, and as one gf_query call per index; then every job against the
    FP64 oracle on a sample of its queries."""
    import oracle
    t0 = time.perf_counter()
    ws = workloads.multi_index(seed=3, count=20, scale=args.multi_scale)
    forms = ["bf16" if i % 2 else "fp32" for i in range(len(ws))]
    forests = [geraf.build_forest(w.X, w.m, w.t, w.p, w.seed, forms=() if f == "fp32" else (f,))
               for w, f in zip(ws, forms)]
    log(f"[bench] multi-20 x{args.multi_scale}: {sum(len(w.Q) for w in ws)} queries over "
        f"{len(ws)} indexes, {sum(w.X.nbytes for w in ws) / 1e9:.1f} GB of rows, data + forests "
        f"{time.perf_counter() - t0:.1f}s")
    jobs = []
    for w, F, f in zip(ws, forests, forms):
        nq = len(w.Q)
        jobs.append(dict(forest=F, Q=torch.from_numpy(w.Q).to(dev), k=w.k, checks=1,
                         checks_per_query=torch.from_numpy(w.checks).to(dev), form=f,
                         ids=torch.empty((nq, w.k), dtype=torch.int32, device=dev),
                         dists=torch.empty((nq, w.k), dtype=torch.float32, device=dev)))
    total = sum(len(w.Q) for w in ws)

    def per_index():
        for j in jobs:
            geraf.query(j["forest"], j["Q"], j["k"], 1, j["ids"], j["dists"],
                        checks_per_query=j["checks_per_query"], form=j["form"])

    modes = {"graph": lambda: geraf.query_multi(jobs),
             "graph_autotuned": lambda: geraf.query_multi(jobs, autotune=True),
             "eager": lambda: geraf.query_multi(jobs, eager=True),
             "per_index_calls": per_index}
    res = {}
    for name, fn in modes.items():
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        res[name] = dict(value=round(total / dt, 2), ms_per_step=round(dt * 1e3, 3))
        log(f"[bench] multi {name}: {dt * 1e3:.2f} ms per step, {total / dt:.0f} queries/s")
    # every job against the oracle on a sample of its queries (graph results)
    geraf.query_multi(jobs)
    torch.cuda.synchronize()
    parity = []
    t0 = time.perf_counter()
    for w, j, f in zip(ws, jobs, forms):
        Fo = oracle.build_forest(w.X, w.m, w.t, w.p, w.seed, nthreads=host_threads())
        got_i, got_d = j["ids"].cpu().numpy(), j["dists"].cpu().numpy()
        sample = np.linspace(0, len(w.Q) - 1, min(len(w.Q), args.multi_sample)).astype(np.int64)
        hits = total_ref = 0
        max_err = 0.0
        not_cand = 0
        for i in sample:
            Qs = np.ascontiguousarray(w.Q[i:i + 1])
            ref = oracle.search(Fo, w.X, Qs, w.k, int(w.checks[i]), trace=False, candidates=True,
                                nthreads=1)
            g = got_i[i][got_i[i] >= 0]
            not_cand += int((~np.isin(g, ref["cand"][0])).sum())
            r = ref["ids"][0][ref["ids"][0] >= 0]
            hits += len(set(g.tolist()) & set(r.tolist()))
            total_ref += len(r)
            for rr, gid in enumerate(g.tolist()):
                diff = w.X[gid].astype(np.float64) - Qs[0].astype(np.float64)
                true_d = float(diff @ diff)
                max_err = max(max_err, abs(float(got_d[i][rr]) - true_d) / true_d if true_d > 0 else 0.0)
        parity.append(dict(index=w.name, form=f, n=int(w.X.shape[0]), d=int(w.X.shape[1]),
                           queries=len(sample), recall_vs_oracle=round(hits / max(1, total_ref), 4),
                           max_rel_dist_err=float(f"{max_err:.3g}"), ids_not_candidates=not_cand))
    log(f"[bench] multi oracle comparison {time.perf_counter() - t0:.1f}s")
    out = {
        "metric": "queries/s over a batch of 20 indexes with per-query budgets (multi-20)",
        "value": res["graph"]["value"], "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res["graph"]["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+bf16",
        "data": "synthetic",
        "config": {"workload": "multi-20", "scale": args.multi_scale, "indexes": len(ws),
                   "queries": total, "n": [len(w.X) for w in ws], "d": [w.X.shape[1] for w in ws],
                   "forms": forms, "m": 8, "t": 5, "leaf": 16, "k": 10,
                   "checks": "uniform 256..8192 per query"},
        "graph_autotuned": res["graph_autotuned"], "eager": res["eager"],
        "per_index_calls": res["per_index_calls"],
        "graph_stats": geraf.multi_stats(),
        "vs_oracle": parity,
    }
    print(json.dumps(out), flush=True)
    for F in forests:
        F.free()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=WORKLOAD, choices=sorted(FORMS),
                    help="recipe to measure (default: the headline desc-1m-960, BF16 form)")
    ap.add_argument("--checks", type=int, default=None,
                    help="budget c (default: the smallest c reaching recall@10 >= 0.90 on "
                         "desc-1m-960, the recipe's own c otherwise)")
    ap.add_argument("--nq", type=int, default=None)
    ap.add_argument("--recall-sample", type=int, default=500)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-probe", action="store_true",
                    help="skip the streaming-bandwidth probe reported beside the rooflines")
    ap.add_argument("--no-exhaustive", action="store_true",
                    help="skip the exhaustive comparator (every leaf opened) on the tile path")
    ap.add_argument("--no-small-batches", action="store_true",
                    help="skip the per-call times of 1, 16, 128 and 1024 queries on both paths")
    ap.add_argument("--no-build-compare", action="store_true",
                    help="skip the GPU forest build timed beside the host build")
    ap.add_argument("--householder", action="store_true",
                    help="build the forest with the per-tree Householder isometry variant")
    ap.add_argument("--sweep", choices=sorted(SWEEPS),
                    help="accuracy/time sweep over eps or points per leaf (noisy-sphere), "
                         "or recall against the budget c on desc-1m-960")
    ap.add_argument("--multi", action="store_true",
                    help="measure the multi-index launch (multi-20 recipe) instead")
    ap.add_argument("--multi-scale", type=float, default=1.0,
                    help="size factor of the multi-20 indexes and query counts")
    ap.add_argument("--multi-sample", type=int, default=4,
                    help="queries per index compared with the FP64 oracle")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (a plain copy "
                         "kernel of known size that scales rocprofv3 FETCH_SIZE/WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the query path is "
              "measured on a single MI355X; sharding across GPUs is not implemented.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from oracle import bruteforce as bf
    from paper_1603_09596_amd import geraf, workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    geraf.load()
    if args.multi:
        return multi_bench(args, torch, geraf, workloads, dev)
    if args.sweep == "c":
        return c_sweep_bench(args, torch, geraf, workloads, dev)
    if args.sweep:
        return sweep_bench(args, torch, geraf, workloads, dev)
    name = args.workload
    form = FORMS[name]
    t0 = time.perf_counter()
    w = workloads.make(name, nq=args.nq)
    log(f"[bench] workload {name}: X {w.X.shape} Q {w.Q.shape} in {time.perf_counter() - t0:.1f}s")
    t0 = time.perf_counter()
    F = geraf.build_forest(w.X, w.m, w.t, w.p, w.seed, forms=() if form == "fp32" else (form,),
                           householder=args.householder)
    host_build_s = time.perf_counter() - t0
    log(f"[bench] forest build + upload {host_build_s:.1f}s (H={F.H})")
    build = None
    if not args.no_build_compare:
        # the same forest built on the GPU from device rows (GF_BUILD_DEVICE):
        # wall time of the whole call, and its arrays against the host build's
        Xd = torch.from_numpy(w.X).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Fd = geraf.build_forest(Xd, w.m, w.t, w.p, w.seed, forms=() if form == "fp32" else (form,),
                                householder=args.householder, device_build=True)
        torch.cuda.synchronize()
        dev_build_s = time.perf_counter() - t0
        Th, Td = F.export_tree(), Fd.export_tree()
        same = all(np.array_equal(Th[key], Td[key]) for key in ("D", "split_dim", "perm", "leaf_off")) \
            and np.array_equal(Th["split_val"].view(np.uint32), Td["split_val"].view(np.uint32))
        Fd.free()
        del Xd, Th, Td
        build = {"host_s": round(host_build_s, 3), "device_s": round(dev_build_s, 3),
                 "host_input": "numpy rows", "device_input": "device rows", "arrays_equal": bool(same)}
        log(f"[bench] forest build on the GPU {dev_build_s:.3f}s, arrays equal to the host build: {same}")
    Q = torch.from_numpy(w.Q).to(dev)
    nq, k = len(w.Q), w.k
    c = args.checks if args.checks is not None else (CHECKS_AT_090 if name == WORKLOAD else w.c)
    kk = min(64, 4 * k)
    ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
    dists = torch.empty((nq, k), dtype=torch.float32, device=dev)
    if args.copy_probe_mb > 0:
        src = torch.ones(args.copy_probe_mb << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: {args.copy_probe_mb} MiB device-to-device")
        del src, dst
    nc = torch.empty(nq, dtype=torch.int64, device=dev)
    geraf.query_trace(F, Q, c, ncand=nc)
    torch.cuda.synchronize()
    ncand_total = int(nc.sum().item())
    log(f"[bench] c={c}: mean candidates/query {ncand_total / nq:.0f}")

    def timed(form, steps, warmup):
        for _ in range(warmup):
            geraf.query(F, Q, k, c, ids, dists, form=form)
        torch.cuda.synchronize()
        phases = []
        t0 = time.perf_counter()
        for _ in range(steps):
            geraf.query(F, Q, k, c, ids, dists, form=form)
            tm = geraf.last_query_timing()
            phases.append(tm)
            log(f"[bench] {form} step ({tm['path']} path): prep {tm['prep_ms']:.1f} ms, select "
                f"{tm['select_ms']:.1f} ms, scan/expand {tm['scan_or_expand_ms']:.1f} ms, tile "
                f"{tm['tile_ms']:.1f} ms, merge {tm['merge_ms']:.1f} ms")
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        mean = {key: float(np.mean([p[key] for p in phases]))
                for key in ("prep_ms", "select_ms", "scan_or_expand_ms", "tile_ms", "merge_ms")}
        mean["path"] = phases[-1]["path"]
        return wall, mean, ids.cpu().numpy(), dists.cpu().numpy()

    def scan_roofline(f, ms):
        # the row scan (gathers + distances + best-k): algorithmic bytes per launch
        algo = scan_bytes_per_launch(F, nq, ncand_total, f, k, kk, c)
        achieved = algo / (ms / 1000.0) / 1e9
        return dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=pmc_traffic(f"k_scan ({f})", name),
                    kernel=f"k_scan ({f})", bytes_per_launch=int(algo), ms_per_launch=round(ms, 3))

    wall, ph, ids_main, dists_main = timed(form, args.steps, args.warmup)
    value = args.steps * nq / wall
    fp32 = None
    if form != "fp32" and not args.no_fp32:
        wall32, ph32, ids_fp32, _ = timed("fp32", max(1, args.steps), 1)
        fp32 = dict(value=round(args.steps * nq / wall32, 2), path=ph32["path"],
                    scan_ms=round(ph32["scan_or_expand_ms"], 2),
                    ms_per_step=round(1000 * wall32 / max(1, args.steps), 2))
        if ph32["path"] == "rows":
            # the candidate gathers of the FP32 form against the HBM peak
            fp32["roofline"] = scan_roofline("fp32", ph32["scan_or_expand_ms"])

    # recall@10 on a query sample against exact FP64 neighbours
    idx = np.linspace(0, nq - 1, min(args.recall_sample, nq)).astype(np.int64)
    t0 = time.perf_counter()
    gt, gt_dist = bf.knn_ground_truth(w.X, w.Q[idx], k)
    log(f"[bench] ground truth for {len(idx)} queries {time.perf_counter() - t0:.1f}s")
    rec_main = recall_at(ids_main[idx], gt)
    one_main = float(np.mean([gt[i, 0] in set(ids_main[j].tolist()) for i, j in enumerate(idx)]))
    # the paper's 1-NN miss rate (Sec. 4): the first answer farther than the exact nearest
    first = ids_main[idx, 0].astype(np.int64)
    d_first = np.full(len(idx), np.inf)
    ok = first >= 0
    diff = w.X[first[ok]].astype(np.float64) - w.Q[idx[ok]].astype(np.float64)
    d_first[ok] = np.einsum("ij,ij->i", diff, diff)
    miss_1nn, _ = nn_quality(gt_dist[:, 0], d_first, 0.0)
    if fp32 is not None:
        fp32[f"recall@{k}"] = round(recall_at(ids_fp32[idx], gt), 4)

    if ph["path"] == "tile":
        # dominant kernel: the MFMA score kernel.  It scores every (query,
        # point) pair of its blocks, 2*nq*n*d flops per launch (dense); the
        # method's own work is 2*d flops per (query, candidate) pair, beside it
        kname, peak = TILE_KERNELS[form]
        flops = 2.0 * nq * F.n * F.d
        achieved = flops / (ph["tile_ms"] / 1000.0) / 1e12
        mflops = 2.0 * F.d * ncand_total
        m_ach = mflops / (ph["tile_ms"] / 1000.0) / 1e12
        roofline = dict(bound="mfma", achieved=round(achieved, 1), peak=peak,
                        unit="TFLOP/s", frac=round(achieved / peak, 4),
                        traffic=pmc_traffic(kname, name), kernel=kname,
                        flops_per_launch=int(flops), ms_per_launch=round(ph["tile_ms"], 3),
                        method_work=dict(flops_per_launch=int(mflops), achieved=round(m_ach, 1),
                                         frac=round(m_ach / peak, 4),
                                         share_of_dense=round(mflops / flops, 4)))
    else:
        roofline = scan_roofline(form, ph["scan_or_expand_ms"])

    # the same tile kernel with every candidate bit set (the whole forest
    # opened: exhaustive reduced-precision search, FP32 re-rank), timed the
    # same way, with its recall: the comparator of the forest's budget
    exhaustive = None
    if ph["path"] == "tile" and not args.no_exhaustive:
        call = m_total = F.m << F.H
        for _ in range(args.warmup):
            geraf.query(F, Q, k, call, ids, dists, form=form)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            geraf.query(F, Q, k, call, ids, dists, form=form)
        torch.cuda.synchronize()
        ex_wall = (time.perf_counter() - t0) / args.steps
        ex_ph = geraf.last_query_timing()
        ex_ids = ids.cpu().numpy()
        exhaustive = dict(checks=m_total, value=round(nq / ex_wall, 2), ms_per_step=round(1e3 * ex_wall, 2),
                          tile_ms=round(ex_ph["tile_ms"], 3), path=ex_ph["path"],
                          **{f"recall@{k}": round(recall_at(ex_ids[idx], gt), 4)})
        log(f"[bench] exhaustive comparator: {exhaustive}")

    # small batches, the forest's own regime (the paper searches one query at
    # a time): per-call time of nq in {1, 16, 128, 1024} on each path
    small = None
    if not args.no_small_batches:
        small = []
        for b in (1, 16, 128, 1024):
            Qb = Q[:b].contiguous()
            ib = torch.empty((b, k), dtype=torch.int32, device=dev)
            db = torch.empty((b, k), dtype=torch.float32, device=dev)
            row = dict(nq=b)
            for path in ("rows", "tile"):
                os.environ["GF_SCAN_PATH"] = path
                geraf.query(F, Qb, k, c, ib, db, form=form)
                torch.cuda.synchronize()
                reps = 5 if b <= 128 else 2
                t0 = time.perf_counter()
                for _ in range(reps):
                    geraf.query(F, Qb, k, c, ib, db, form=form)
                torch.cuda.synchronize()
                dt = (time.perf_counter() - t0) / reps
                tm = geraf.last_query_timing()
                row[f"{path}_ms"] = round(1e3 * dt, 3)
                row[f"{path}_qps"] = round(b / dt, 1)
                row[f"{path}_phases_ms"] = [round(tm[key], 3) for key in
                                            ("prep_ms", "select_ms", "scan_or_expand_ms", "tile_ms", "merge_ms")]
            os.environ.pop("GF_SCAN_PATH", None)
            small.append(row)
            log(f"[bench] small batch {row}")

    probe = None if args.no_probe else hbm_probe(torch, geraf, dev)
    if probe:
        log(f"[bench] streaming read probe: {probe['read_GB_s']} GB/s")

    cpu, oracle_cmp = None, None
    if not args.no_cpu_baseline:
        cpu, sample, ref = cpu_baseline(w, idx, c, args.cpu_seconds, host_threads(), args.householder)
        oracle_cmp = vs_oracle(w.X, w.Q[sample], ids_main[sample], dists_main[sample], ref)

    if name == WORKLOAD and not args.householder:
        metric = "queries/s at recall@10>=0.90, 1Mx960, 16 trees; BF16 vs FP32 form"
    else:
        metric = f"queries/s, {name}, {form.upper()} form, c={c}, k={k}" + (
            ", Householder isometry variant" if args.householder else "")
    out = {
        "metric": metric,
        "value": round(value, 2),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000 * wall / args.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": form,
        "data": "synthetic",
        "config": {"workload": name, "n": int(F.n), "d": int(F.d), "m": int(F.m),
                   "t": int(F.t), "leaf": int(F.leaf), "checks": c, "k": k, "nq": nq,
                   "form": form, "rerank": kk if form != "fp32" else None,
                   "variant": "householder" if args.householder else None},
        f"recall@{k}": round(rec_main, 4),
        f"1-recall@{k}": round(one_main, 4),
        "miss_pct_1nn": round(miss_1nn, 2),
        "vs_oracle": oracle_cmp,
        "recall_sample": len(idx),
        "mean_candidates": round(ncand_total / nq, 1),
        "path": ph["path"],
        "phases_ms": {key: round(v, 2) for key, v in ph.items() if key != "path"},
        "fp32_form": fp32,
        "roofline": roofline,
        "forest_build": build,
        "exhaustive_comparator": exhaustive,
        "small_batches": small,
        "hbm_probe": probe,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    F.free()


if __name__ == "__main__":
    main()
