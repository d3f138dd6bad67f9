"""Benchmark: QPS at recall@10 >= 0.95 of PEOs-routed graph search on one GPU,
against the same search with the routing test off (exhaustive-neighbour).

Workload (default): 1,000,000 x 128 integer-valued vectors (0..255) from a
skewed mixture of 100 exponential clusters (a synthetic stand-in for SIFT),
10,000 queries from the same mixture, pruned 64-NN graph of degree 32,
L = 8 subspaces, m = 16 directions, eps = 0.1, k = 10, squared l2.

A step = one pass of the whole hot path over the 10,000-query batch: the
projection tables (matrix cores) and the search kernel, inputs resident in
HBM.  The list size ef is the smallest swept value whose mean recall@10
reaches 0.95 (each mode gets its own).  Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="sift_like_1m_d128")
    ap.add_argument("--n", type=int, default=None, help="override base size (testing)")
    ap.add_argument("--nq", type=int, default=None, help="override query count (testing)")
    ap.add_argument("--eps", type=float, default=None)
    ap.add_argument("--pool", type=int, default=0, help="candidate-list capacity, 0 = unbounded queue")
    ap.add_argument("--target", type=float, default=0.95)
    ap.add_argument("--efs", default="16,24,32,48,64,96,128,192,256")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="oracle CPU-baseline budget")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-only", action="store_true",
                    help="skip the sweep; time the search at --ef (for profiler runs)")
    ap.add_argument("--ef", type=int, default=None)
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; the multi-GPU sharding "
                                   "is a design (see DESIGN.md), not a code path",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    import paper_2402_11354_amd as P
    import workloads as W
    from workloads.graph import recall_at_k

    dev = torch.device("cuda:0")
    w = W.WORKLOADS[args.workload]
    w = w.with_sizes(n=args.n, nq=args.nq)
    eps = args.eps if args.eps is not None else w.eps
    t0 = time.time()
    x = W.make_base(w)
    q = W.make_queries(w)
    A, B = W.directions_for(w)
    log(f"data {w.name} n={w.n} nq={w.nq} d={w.d} in {time.time() - t0:.1f}s")
    t0 = time.time()
    g, entry = W.build_graph(x, w.R, w.cand, device=dev, log=lambda m: log("graph:", m))
    deg = (g >= 0).sum(1)
    log(f"graph R={w.R} mean degree {deg.mean():.2f} entry={entry} in {time.time() - t0:.1f}s")
    xt = torch.from_numpy(x).to(dev)
    qt = torch.from_numpy(q).to(dev)
    gt_ = torch.from_numpy(g).to(dev)
    At, Bt = torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev)
    t0 = time.time()
    index = P.peos_build_tables(xt, gt_, entry, w.L, w.m, At, Bt, w.metric)
    torch.cuda.synchronize()
    log(f"edge records built in {time.time() - t0:.2f}s")
    t0 = time.time()
    gt_ids, gt_d = W.ground_truth(x, q, w.k, w.metric, device=dev)
    log(f"ground truth in {time.time() - t0:.1f}s")

    nq = w.nq
    efs = [int(e) for e in args.efs.split(",")]
    efmax = max(efs + [args.ef or 0])
    ws = torch.empty(P.peos_search_ws_bytes(index, nq, efmax, args.pool), dtype=torch.uint8,
                     device=dev)
    tables = torch.empty((nq, w.L + 1, w.m), dtype=torch.float32, device=dev)
    qnorms = torch.empty(nq, dtype=torch.float32, device=dev)
    ids = torch.empty((nq, w.k), dtype=torch.int64, device=dev)
    dists = torch.empty((nq, w.k), dtype=torch.float32, device=dev)
    stats = torch.empty((nq, P.PEOS_NSTATS), dtype=torch.int32, device=dev)

    def step(ef, mode, ev=None):
        if ev is not None:
            ev[0].record()
        P.peos_query_tables(index, qt, tables, qnorms)
        if ev is not None:
            ev[1].record()
        P.peos_search_tables(index, qt, tables, qnorms, w.k, ef, w.k, args.pool, eps, mode, ids,
                             dists, stats, ws)
        if ev is not None:
            ev[2].record()

    def evaluate(ef, mode):
        step(ef, mode)
        torch.cuda.synchronize()
        r = recall_at_k(x, q, ids.cpu().numpy(), gt_d, w.k, w.metric).mean()
        st = stats.cpu().numpy()
        return r, st

    def timed(ef, mode, steps, warmup):
        for _ in range(warmup):
            step(ef, mode)
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for i in range(steps):
            step(ef, mode, evs[i])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
        step_ms = np.array([e[0].elapsed_time(e[2]) for e in evs])
        table_ms = np.array([e[0].elapsed_time(e[1]) for e in evs])
        search_ms = np.array([e[1].elapsed_time(e[2]) for e in evs])
        return wall, step_ms, table_ms, search_ms

    def sweep(mode):
        pts = []
        for ef in efs:
            r, st = evaluate(ef, mode)
            _, sms, _, _ = timed(ef, mode, 2, 0)
            pts.append((ef, float(r), float(nq / (sms.mean() / 1e3)), st))
            log(f"  mode={'PEOS' if mode == 0 else 'EXH'} ef={ef}: recall@{w.k}={r:.4f} "
                f"qps~{pts[-1][2]:.0f} ndist={st[:, 9].mean():.0f} tests={st[:, 3].mean():.0f} "
                f"spill={(st[:, 11] & 4 != 0).mean():.3f} poolfull={(st[:, 11] & 2 != 0).mean():.3f}")
            if r >= args.target + 0.02:
                break
        return pts

    def pick(pts):
        ok = [p for p in pts if p[1] >= args.target]
        return (ok[0], True) if ok else (max(pts, key=lambda p: p[1]), False)

    if args.profile_only:
        ef = args.ef or w.ef
        wall, sms, tms, srch = timed(ef, 0, args.steps, args.warmup)
        log(f"profile-only ef={ef}: step {sms.mean():.3f} ms search {srch.mean():.3f} ms")
        return

    log("sweep PEOS")
    pe_pts = sweep(P.PEOS_MODE_PEOS)
    log("sweep EXHAUSTIVE")
    ex_pts = sweep(P.PEOS_MODE_EXHAUSTIVE)
    (pe_ef, pe_rec, _, pe_st), pe_ok = pick(pe_pts)
    (ex_ef, ex_rec, _, ex_st), ex_ok = pick(ex_pts)

    log(f"timed PEOS ef={pe_ef} ({args.steps} steps)")
    wall, step_ms, table_ms, search_ms = timed(pe_ef, P.PEOS_MODE_PEOS, args.steps, args.warmup)
    qps = nq * args.steps / wall
    log(f"timed EXHAUSTIVE ef={ex_ef}")
    ex_wall, ex_step_ms, _, ex_search_ms = timed(ex_ef, P.PEOS_MODE_EXHAUSTIVE, args.steps,
                                                 args.warmup)
    ex_qps = nq * args.steps / ex_wall

    # algorithmic bytes of one search launch, from the kernel's own counters
    def alg_bytes(st, mode):
        per_q = (4.0 * w.R * st[:, 0]                        # neighbour ids of each expansion
                 + (w.L + 1 + 16.0) * st[:, 3]               # codes + 4 fp32 scalars per tested edge
                 + 4.0 * w.d * st[:, 9]                      # exact distances
                 + 4.0 * w.d + 4.0 * (w.L + 1) * w.m          # query vector and table
                 + 12.0 * w.k)                               # outputs
        return float(per_q.sum())

    pe_bytes = alg_bytes(pe_st, 0)
    search_s = float(search_ms.mean()) / 1e3
    achieved = pe_bytes / search_s / 1e9
    peak = 8000.0

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(x, g, entry, q, w, pe_ef, eps, args.pool, args.cpu_seconds)

    out = {
        "metric": "QPS at recall@10>=0.95, PEOs vs exhaustive-neighbor search, 1 GPU; p99 ms",
        "value": round(qps, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(float(wall / args.steps * 1e3), 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "nq": nq, "d": w.d, "R": w.R, "L": w.L,
                   "m": w.m, "eps": eps, "k": w.k, "ef": pe_ef, "pool": args.pool,
                   "metric": "l2" if w.metric == 0 else "angular"},
        "recall": round(pe_rec, 4),
        "recall_target_met": bool(pe_ok),
        "p50_ms": round(float(np.percentile(step_ms, 50)), 4),
        "p99_ms": round(float(np.percentile(step_ms, 99)), 4),
        "exhaustive": {"value": round(ex_qps, 1), "ef": ex_ef, "recall": round(ex_rec, 4),
                       "recall_target_met": bool(ex_ok),
                       "p99_ms": round(float(np.percentile(ex_step_ms, 99)), 4),
                       "search_ms": round(float(ex_search_ms.mean()), 4),
                       "ndist_per_query": round(float(ex_st[:, 9].mean()), 1)},
        "speedup_vs_exhaustive": round(qps / ex_qps, 3),
        "per_query": {"ndist": round(float(pe_st[:, 9].mean()), 1),
                      "tests": round(float(pe_st[:, 3].mean()), 1),
                      "expansions": round(float(pe_st[:, 0].mean()), 1),
                      "pass_rate": round(float(pe_st[:, 8].sum() / max(1, pe_st[:, 3].sum())), 4),
                      "alg_bytes": round(pe_bytes / nq, 1)},
        "kernel_ms": {"query_table": round(float(table_ms.mean()), 4),
                      "search": round(float(search_ms.mean()), 4)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": peak, "unit": "GB/s",
                     "frac": round(achieved / peak, 4), "traffic": None},
        "cpu_baseline": cpu,
        "sweep": {"peos": [(p[0], round(p[1], 4), round(p[2], 1)) for p in pe_pts],
                  "exhaustive": [(p[0], round(p[1], 4), round(p[2], 1)) for p in ex_pts]},
    }
    print(json.dumps(out), flush=True)


def cpu_baseline(x, g, entry, q, w, ef, eps, pool, budget_s):
    """The oracle, as it stands, on the host cores: a bounded sample of the
    same queries at the same operating point."""
    import oracle

    threads = min(16, os.cpu_count() or 1)
    n = 16
    t0 = time.perf_counter()
    oracle.search(x, g, entry, q[:n], w.k, ef, w.L, w.m, *w_dirs(w), w.metric, eps, pool=pool,
                  nthreads=threads)
    dt = time.perf_counter() - t0
    n2 = int(min(len(q), max(n, n * budget_s / max(dt, 1e-3))))
    t0 = time.perf_counter()
    oracle.search(x, g, entry, q[:n2], w.k, ef, w.L, w.m, *w_dirs(w), w.metric, eps, pool=pool,
                  nthreads=threads)
    dt = time.perf_counter() - t0
    log(f"cpu baseline: {n2} queries in {dt:.1f}s on {threads} threads")
    return {"value": round(n2 / dt, 2), "unit": "queries/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n2} of the {len(q)} queries, same ef/eps/pool, float64 oracle"}


def w_dirs(w):
    import workloads as W
    return W.directions_for(w)


if __name__ == "__main__":
    main()
