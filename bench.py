"""Benchmark: QPS at recall@10 >= 0.95 of PEOs-routed graph search on one GPU,
against the same search with the routing test off (exhaustive-neighbour).

Workload (default): 1,000,000 x 128 integer-valued vectors (0..255) from a
skewed mixture of 100 exponential clusters (a synthetic stand-in for SIFT),
10,000 queries from the same mixture, pruned 64-NN graph of degree 32,
L = 8 subspaces, m = 16 directions, k = 10, squared l2.

A step = one pass of the whole hot path over the 10,000-query batch: the
projection tables (matrix cores) and the search kernel, inputs resident in
HBM.  Operating points: for each stopping rule (candidate pool = ef, the HNSW
rule; pool = 0, the unbounded queue of the printed Alg. 1) and each eps, the
smallest swept ef whose mean recall@10 reaches 0.95; the reported value is the
fastest PEOs operating point, and "exhaustive" the fastest one with the test
off.  Prints one JSON line.
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

PEAK_HBM_GBS = 8000.0
KERNEL_SOURCES = ("paper_2402_11354_amd/csrc/k_search.hpp",
                  "paper_2402_11354_amd/csrc/peos_device.hpp",
                  "paper_2402_11354_amd/csrc/peos_api.hip")


def kernel_digest():
    """Digest of the search kernel's sources: a memory-counter record applies
    only to the kernel it was taken on."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_record(key):
    """HBM bytes per search launch from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summaries (a 'traffic-record:' JSON line in profiles/*.md), if
    one was taken on this kernel at this operating point; else None."""
    import glob
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(f) as fh:
            for line in fh:
                if not line.startswith("traffic-record:"):
                    continue
                try:
                    rec = json.loads(line.split(":", 1)[1])
                except ValueError:
                    continue
                if all(rec.get(k) == v for k, v in key.items()):
                    return (rec["fetch_kib"] * rec["fetch_scale"]
                            + rec["write_kib"] * rec["write_scale"]) * 1024.0
    return None


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
    ap.add_argument("--pools", default="ef,0",
                    help="candidate-list capacities to sweep: 'ef' = the HNSW stopping rule, "
                         "0 = the unbounded queue of the printed Alg. 1")
    ap.add_argument("--epss", default="0.05,0.1,0.2", help="eps values swept for PEOs")
    ap.add_argument("--target", type=float, default=0.95)
    ap.add_argument("--efs", default="16,24,32,40,48,52,56,60,64,72,80,96,128,192,256")
    ap.add_argument("--sweep-steps", type=int, default=10,
                    help="timed steps per swept operating point")
    ap.add_argument("--no-half", action="store_true",
                    help="skip the sweep of records with 16-bit scalars")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="oracle CPU-baseline budget")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-only", action="store_true",
                    help="skip the sweep; time PEOs at --ef/--pool/--eps (for profiler runs)")
    ap.add_argument("--ef", type=int, default=64)
    ap.add_argument("--pool", default="ef")
    ap.add_argument("--eps", type=float, default=0.1)
    ap.add_argument("--hash-cap", type=int, default=0, help="with --profile-only: visited-hash capacity")
    ap.add_argument("--exhaustive", action="store_true",
                    help="with --profile-only: time the search with the test off")
    ap.add_argument("--slots", type=int, default=0,
                    help="with --profile-only: resident waves of the persistent grid")
    ap.add_argument("--listcap", type=int, default=0,
                    help="with --profile-only: force an LDS list of this capacity")
    ap.add_argument("--waves", type=int, default=0,
                    help="with --profile-only: waves per query (0 = the library's choice)")
    ap.add_argument("--mode", default="headline",
                    choices=("headline", "batched", "serving", "precision", "compact",
                             "descent"),
                    help="headline: the QPS-at-recall comparison (default); batched: one "
                         "captured launch over a batch of uneven k/ef; serving: the request "
                         "loop under Poisson arrivals")
    ap.add_argument("--rates", default="5000,20000,50000,100000,200000",
                    help="serving: arrival rates (queries/s)")
    ap.add_argument("--seconds", type=float, default=1.5, help="serving: duration per rate")
    ap.add_argument("--copy-calibrate", type=int, default=0, metavar="MIB",
                    help="only run one device copy of MIB MiB (a kernel of known traffic for "
                         "calibrating memory counters) and exit")
    ap.add_argument("--compact-L", type=int, default=2,
                    help="compact mode: subspaces of the compact records (1..4)")
    ap.add_argument("--no-long-rows", action="store_true",
                    help="forbid the long-vector search variant (for comparisons)")
    ap.add_argument("--prec-workload", default="gist_like_1m_d960",
                    help="precision mode: the workload (the 960-d one by default)")
    ap.add_argument("--prec-ef", type=int, default=0,
                    help="precision mode: time only k = 10 at this ef (for profiler runs)")
    ap.add_argument("--gather-probe", action="store_true",
                    help="only measure random 512-byte row gathers (the library's calibration "
                         "kernel) over arrays of 64 MB to 4 GB: the practical HBM ceiling of "
                         "the search's access pattern")
    args = ap.parse_args()

    if args.gather_probe:
        return gather_probe()

    if args.copy_calibrate:
        # a plain device copy of known size, for scaling memory counters
        import torch
        dev = torch.device("cuda:0")
        src = torch.ones(args.copy_calibrate << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copied {args.copy_calibrate} MiB")
        return

    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU only; sharding across GPUs is a "
                                   "design note, not a code path", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    if args.mode == "batched":
        return batched(args)
    if args.mode == "serving":
        return serving(args)
    if args.mode == "precision":
        return precision(args)
    if args.mode == "compact":
        return compact(args)
    if args.mode == "descent":
        return descent(args)

    import paper_2402_11354_amd as P
    import workloads as W
    from workloads.graph import recall_at_k

    dev = torch.device("cuda:0")
    w = W.WORKLOADS[args.workload].with_sizes(n=args.n, nq=args.nq)
    t0 = time.time()
    x = W.make_base(w)
    q = W.make_queries(w)
    A, B = W.directions_for(w)
    log(f"data {w.name} n={w.n} nq={w.nq} d={w.d} in {time.time() - t0:.1f}s")
    t0 = time.time()
    g, entry = W.graph_for(w, x, device=dev, log=lambda m: log("graph:", m))
    log(f"graph R={w.R} mean degree {(g >= 0).sum(1).mean():.2f} entry={entry} "
        f"in {time.time() - t0:.1f}s")
    xt, qt, gt_ = (torch.from_numpy(a).to(dev) for a in (x, q, g))
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
    efmax = max(efs + [args.ef])
    ws = torch.empty(P.peos_search_ws_bytes(index, nq, efmax, 0), dtype=torch.uint8, device=dev)
    tables = torch.empty((nq, w.L + 1, w.m), dtype=torch.float32, device=dev)
    qnorms = torch.empty(nq, dtype=torch.float32, device=dev)
    ids = torch.empty((nq, w.k), dtype=torch.int64, device=dev)
    dists = torch.empty((nq, w.k), dtype=torch.float32, device=dev)
    stats = torch.empty((nq, P.PEOS_NSTATS), dtype=torch.int32, device=dev)

    def pool_of(spec, ef):
        return ef if spec == "ef" else int(spec)

    def step(cfg, ev=None, ix=None):
        ef, pool, eps, mode = cfg
        ix = index if ix is None else ix
        if ev is not None:
            ev[0].record()
        P.peos_query_tables(ix, qt, tables, qnorms)
        if ev is not None:
            ev[1].record()
        P.peos_search_tables(ix, qt, tables, qnorms, w.k, ef, w.k, pool, eps, mode, ids, dists,
                             stats, ws)
        if ev is not None:
            ev[2].record()

    def timed(cfg, steps, warmup, ix=None):
        for _ in range(warmup):
            step(cfg, ix=ix)
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for i in range(steps):
            step(cfg, evs[i], ix=ix)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
        step_ms = np.array([e[0].elapsed_time(e[2]) for e in evs])
        table_ms = np.array([e[0].elapsed_time(e[1]) for e in evs])
        search_ms = np.array([e[1].elapsed_time(e[2]) for e in evs])
        return wall, step_ms, table_ms, search_ms

    if args.profile_only:
        P.peos_set_search_tuning(index, args.hash_cap, args.listcap, args.slots, args.waves)
        cfg = (args.ef, pool_of(args.pool, args.ef), args.eps,
               P.PEOS_MODE_EXHAUSTIVE if args.exhaustive else P.PEOS_MODE_PEOS)
        wall, sms, tms, srch = timed(cfg, args.steps, args.warmup)
        log(f"profile-only {cfg}: step {sms.mean():.3f} ms search {srch.mean():.3f} ms "
            f"qps {nq * args.steps / wall:.0f}")
        st = stats.cpu().numpy()
        log(f"per query: expansions {st[:, 0].mean():.1f} tests {st[:, 3].mean():.1f} "
            f"ndist {st[:, 9].mean():.1f} (max {st[:, 9].max()}, p99 "
            f"{np.percentile(st[:, 9], 99):.0f}); visited set spilled to HBM in "
            f"{(st[:, 11] & P.PEOS_STATUS_VISITED_SPILL != 0).mean() * 100:.2f}% of queries")
        log("traffic key " + json.dumps(dict(kernel="k_search", source=kernel_digest(),
                                             workload=w.name, n=w.n, nq=nq, ef=cfg[0],
                                             pool=cfg[1], eps=cfg[2], mode=cfg[3],
                                             hash_cap=args.hash_cap)))
        return

    def sweep(pool_spec, eps, mode, ix=None, tag=""):
        pts = []
        for ef in efs:
            cfg = (ef, pool_of(pool_spec, ef), eps, mode)
            step(cfg, ix=ix)
            torch.cuda.synchronize()
            r = float(recall_at_k(x, q, ids.cpu().numpy(), gt_d, w.k, w.metric).mean())
            st = stats.cpu().numpy()
            wall, _, _, _ = timed(cfg, args.sweep_steps, 2, ix=ix)
            qps = nq * args.sweep_steps / wall
            pts.append(dict(cfg=cfg, recall=r, qps=qps, stats=st))
            log(f"  {'PEOS' if mode == 0 else 'EXH '}{tag} pool={pool_spec} eps={eps} ef={ef}: "
                f"recall={r:.4f} qps~{qps:.0f} exp={st[:, 0].mean():.1f} "
                f"edges/exp={st[:, 1].sum() / max(1, st[:, 0].sum()):.1f} "
                f"ndist={st[:, 9].mean():.0f} tests={st[:, 3].mean():.0f} "
                f"spill={(st[:, 11] & 4 != 0).mean():.2f} full={(st[:, 11] & 2 != 0).mean():.2f}")
            if r >= args.target + 0.015:
                break
        return pts

    def best(pts_lists):
        ok = [p for pts in pts_lists for p in pts if p["recall"] >= args.target]
        if ok:
            return max(ok, key=lambda p: p["qps"]), True
        return max((p for pts in pts_lists for p in pts), key=lambda p: p["recall"]), False

    pools = args.pools.split(",")
    epss = [float(e) for e in args.epss.split(",")]
    pe_sweeps, ex_sweeps = {}, {}
    for ps in pools:
        for eps in epss:
            log(f"sweep PEOS pool={ps} eps={eps}")
            pe_sweeps[(ps, eps)] = sweep(ps, eps, P.PEOS_MODE_PEOS)
        log(f"sweep EXHAUSTIVE pool={ps}")
        ex_sweeps[ps] = sweep(ps, 0.1, P.PEOS_MODE_EXHAUSTIVE)
    pe, pe_ok = best(pe_sweeps.values())
    ex, ex_ok = best(ex_sweeps.values())
    # the same search on records with 16-bit scalars and tables (the paper's
    # default scalar width; arithmetic stays single precision), HNSW rule
    half_sweeps = {}
    half_index = None
    if not args.no_half:
        half_index = P.peos_build_tables(xt, gt_, entry, w.L, w.m, At, Bt, w.metric,
                                         flags=P.PEOS_FLAG_FP16)
        for eps in epss:
            log(f"sweep PEOS half records pool=ef eps={eps}")
            half_sweeps[("ef", eps)] = sweep("ef", eps, P.PEOS_MODE_PEOS, ix=half_index,
                                             tag=" half")

    def interpolated(sweeps):
        """QPS at exactly the target recall, linear in (recall, QPS) between
        the two swept points that bracket it, best over the sweeps."""
        out = None
        for pts in sweeps:
            for a_, b_ in zip(pts, pts[1:]):
                if a_["recall"] < args.target <= b_["recall"]:
                    t = (args.target - a_["recall"]) / (b_["recall"] - a_["recall"])
                    v = a_["qps"] + t * (b_["qps"] - a_["qps"])
                    out = v if out is None else max(out, v)
        return None if out is None else round(out, 1)

    from paper_2402_11354_amd import autotune

    def tuned(cfg):
        ef, pool, eps, mode = cfg
        cap, _ = autotune.tune(index, qt, w.k, ef, pool=pool, eps=eps, mode=mode,
                               use_cache=False, log=log)
        return cap, index.tuned_waves

    pe_cap, pe_waves = tuned(pe["cfg"])
    log(f"timed PEOS {pe['cfg']} hash_cap={pe_cap} ({args.steps} steps)")
    wall, step_ms, table_ms, search_ms = timed(pe["cfg"], args.steps, args.warmup)
    qps = nq * args.steps / wall
    ex_cap, ex_waves = tuned(ex["cfg"])
    log(f"timed EXHAUSTIVE {ex['cfg']} hash_cap={ex_cap}")
    ex_wall, ex_step_ms, _, ex_search_ms = timed(ex["cfg"], args.steps, args.warmup)
    ex_qps = nq * args.steps / ex_wall
    P.peos_set_search_tuning(index)

    # algorithmic bytes of one search launch, from the kernel's own counters
    lay = index.layout()
    code_bytes = lay.code_bytes

    def alg_bytes(st):
        return search_alg_bytes(st, lay, w.k, pe["cfg"][0])

    def sector_bytes(st):
        """The same accesses rounded to whole 64-byte sectors as the kernel
        issues them: a node's id row per expansion, the node's whole record
        (codes and scalars of all R edges) per expansion that ran the test,
        whole vector rows."""
        sec = lambda b: 64.0 * math.ceil(b / 64.0)
        per_q = (sec(4.0 * w.R) * st[:, 0]
                 + (sec(code_bytes * w.R) + sec(16.0 * w.R)) * st[:, 13]
                 + sec(4.0 * w.d) * st[:, 9]
                 + sec(4.0 * w.d) + sec(4.0 * (w.L + 1) * w.m) + sec(12.0 * w.k))
        return float(per_q.sum())

    pe_bytes = alg_bytes(pe["stats"])
    pe_sector = sector_bytes(pe["stats"])
    achieved = pe_bytes / (float(search_ms.mean()) / 1e3) / 1e9
    ef, pool, eps, mode = pe["cfg"]
    traffic = traffic_record(dict(kernel="k_search", source=kernel_digest(), workload=w.name,
                                  n=w.n, nq=nq, ef=ef, pool=pool, eps=eps, mode=mode,
                                  hash_cap=pe_cap))

    # the practical ceiling of the access pattern: the library's calibration
    # gather of random 512-byte rows over an array the size of the search's
    # working set (base vectors + edge records), on the same box, same run
    work_bytes = int(x.nbytes) + int(index.layout().node_stride) * w.n
    ceiling = measure_gather_ceiling(work_bytes)

    cpu, parity = None, None
    if not args.no_cpu_baseline:
        cpu, ref = cpu_baseline(x, g, entry, q, w, pe["cfg"], args.cpu_seconds)
        # the GPU's results at the headline point against the FP64 oracle's
        # on the same queries (the oracle run that the baseline timed)
        step(pe["cfg"])
        torch.cuda.synchronize()
        parity = parity_summary(x, q, w, ids.cpu().numpy(), dists.cpu().numpy(),
                                stats.cpu().numpy(), ref, gt_ids)

    st = pe["stats"]
    ip_pe, ip_ex = interpolated(pe_sweeps.values()), interpolated(ex_sweeps.values())
    half = None
    if half_sweeps:
        hb, hb_ok = best(half_sweeps.values())
        ip_h = interpolated(half_sweeps.values())
        lay_h = half_index.layout()
        half = {"record_bytes": int(lay_h.node_stride),
                "record_bytes_fp32": int(index.layout().node_stride),
                "best": {"ef": hb["cfg"][0], "eps": hb["cfg"][2], "recall": round(hb["recall"], 4),
                         "qps": round(hb["qps"], 1), "recall_target_met": bool(hb_ok)},
                "interpolated_at_target": ip_h,
                "speedup_vs_exhaustive_at_target": (round(ip_h / ip_ex, 3)
                                                    if ip_h and ip_ex else None),
                "speedup_vs_fp32_records_at_target": (round(ip_h / ip_pe, 3)
                                                      if ip_h and ip_pe else None)}

    def pts_json(d):
        out = {}
        for k, v in d.items():
            name = f"pool={k[0]},eps={k[1]}" if isinstance(k, tuple) else f"pool={k}"
            out[name] = [(p["cfg"][0], round(p["recall"], 4), round(p["qps"], 1)) for p in v]
        return out

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
                   "m": w.m, "eps": eps, "k": w.k, "ef": ef, "pool": pool, "hash_cap": pe_cap,
                   "waves_per_query": pe_waves,
                   "stop_rule": "hnsw (pool=ef)" if pool == ef else "unbounded queue (Alg. 1)",
                   "metric": "l2" if w.metric == 0 else "angular"},
        "recall": round(pe["recall"], 4),
        "recall_target_met": bool(pe_ok),
        "p50_ms": round(float(np.percentile(step_ms, 50)), 4),
        "p99_ms": round(float(np.percentile(step_ms, 99)), 4),
        "exhaustive": {"value": round(ex_qps, 1), "ef": ex["cfg"][0], "pool": ex["cfg"][1],
                       "hash_cap": ex_cap, "waves_per_query": ex_waves,
                       "recall": round(ex["recall"], 4), "recall_target_met": bool(ex_ok),
                       "p99_ms": round(float(np.percentile(ex_step_ms, 99)), 4),
                       "search_ms": round(float(ex_search_ms.mean()), 4),
                       "ndist_per_query": round(float(ex["stats"][:, 9].mean()), 1)},
        "speedup_vs_exhaustive": round(qps / ex_qps, 3),
        "interpolated_at_target": {"peos": ip_pe, "exhaustive": ip_ex,
                                   "speedup": (round(ip_pe / ip_ex, 3)
                                               if ip_pe and ip_ex else None),
                                   "note": f"QPS linear in recall between the two swept ef "
                                           f"bracketing recall {args.target}, best over the "
                                           f"sweeps; {args.sweep_steps} timed steps per point; "
                                           f"ef grid {args.efs}, eps {args.epss}"},
        "per_query": {"ndist": round(float(st[:, 9].mean()), 1),
                      "tests": round(float(st[:, 3].mean()), 1),
                      "tests_by_kind": {"a_ge_1_fail": round(float(st[:, 4].mean()), 1),
                                        "a_le_0_pass": round(float(st[:, 5].mean()), 1),
                                        "h_vs_t": round(float(st[:, 6].mean()), 1),
                                        "zero_edge": round(float(st[:, 7].mean()), 1)},
                      "h_vs_t_pass_rate": round(float(
                          (st[:, 8].sum() - st[:, 5].sum())
                          / max(1, st[:, 6].sum())), 4),
                      "edges": round(float(st[:, 1].mean()), 1),
                      "visited_skips": round(float(st[:, 2].mean()), 1),
                      "expansions": round(float(st[:, 0].mean()), 1),
                      "pass_rate": round(float(st[:, 8].sum() / max(1, st[:, 3].sum())), 4),
                      "alg_bytes": round(pe_bytes / nq, 1)},
        "kernel_ms": {"query_table": round(float(table_ms.mean()), 4),
                      "search": round(float(search_ms.mean()), 4)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": None if traffic is None else round(traffic),
                     "alg_bytes": round(pe_bytes),
                     "sector_bytes": round(pe_sector),
                     "sector_frac": round(pe_sector / (float(search_ms.mean()) / 1e3) / 1e9
                                          / PEAK_HBM_GBS, 4),
                     "gather_ceiling": ceiling,
                     "frac_of_gather_ceiling": round(achieved / ceiling, 4) if ceiling else None},
        "cpu_baseline": cpu,
        "parity": parity,
        "half_scalars": half,
        "sweep": {"peos": pts_json(pe_sweeps), "exhaustive": pts_json(ex_sweeps),
                  "peos_half_records": pts_json(half_sweeps)},
    }
    print(json.dumps(out), flush=True)


def search_alg_bytes(st, lay, k, ef):
    """Algorithmic bytes of one search call, summed over its queries, from the
    kernel's own counters and the index layout: the neighbour ids of each
    expansion, the codes and scalars of each tested edge (and the compact
    records' node header per expansion that ran the test), one vector row per
    exact distance (bfloat16 rows with the traversal copy, then the fp32
    re-rank of the final list), the query and its table, the outputs, and an
    id and a row per distance of the upper-layer descent."""
    st = np.asarray(st, np.float64)
    compact = bool(lay.flags & 8)
    bf = bool(lay.flags & 1)
    half = bool(lay.flags & 2)
    e = 2.0 if bf else 4.0
    per_q = (4.0 * lay.R * st[:, 0]
             + float(lay.code_bytes + lay.scalar_bytes) * st[:, 3]
             + (16.0 * st[:, 13] if compact else 0.0)
             + e * lay.d * st[:, 9]
             + 4.0 * lay.d + (2.0 if half else 4.0) * (lay.L + 1) * lay.m
             + 12.0 * k
             + (4.0 * lay.d * ef if bf else 0.0)
             + (e * lay.d + 4.0) * st[:, 12])
    return float(per_q.sum())


def alg_rate(st, lay, k, ef, qps):
    """Bytes per query and the rate they are moved at (TB/s; the peak is 8)."""
    b = search_alg_bytes(st, lay, k, ef) / max(len(st), 1)
    return dict(alg_bytes_per_query=round(b, 1), alg_TBps=round(b * qps / 1e12, 3))


def _setup(name, n, nq, gt_k):
    """Data, graph, edge records and exact top-gt_k of a named workload."""
    import torch

    import paper_2402_11354_amd as P
    import workloads as W

    dev = torch.device("cuda:0")
    w = W.WORKLOADS[name].with_sizes(n=n, nq=nq)
    t0 = time.time()
    x, q = W.make_base(w), W.make_queries(w)
    A, B = W.directions_for(w)
    log(f"data {w.name} n={w.n} nq={w.nq} d={w.d} in {time.time() - t0:.1f}s")
    t0 = time.time()
    g, entry = W.graph_for(w, x, device=dev, log=lambda m: log("graph:", m))
    log(f"graph R={w.R} mean degree {(g >= 0).sum(1).mean():.2f} in {time.time() - t0:.1f}s")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    index = P.peos_build_tables(T(x), T(g), entry, w.L, w.m, T(A), T(B), w.metric)
    t0 = time.time()
    _, gt_d = W.ground_truth(x, q, gt_k, w.metric, device=dev)
    log(f"ground truth in {time.time() - t0:.1f}s")
    return w, x, q, g, entry, index, gt_d


def _interp(pts, target):
    """QPS at exactly the target recall, linear between the two points of the
    (recall, QPS) sweep that bracket it; None if none do."""
    for (r0, q0), (r1, q1) in zip(pts, pts[1:]):
        if r0 < target <= r1:
            return round(q0 + (target - r0) / (r1 - r0) * (q1 - q0), 1)
    return None


def _recall(x, q, ids, gt_d, k, metric):
    from workloads.graph import recall_at_k
    return recall_at_k(x, q, ids, gt_d, k, metric)


def batched(args):
    """One launch over a batch of queries with uneven k and ef (the batched
    persistent form): ef classes tuned per class, tables + split + search
    captured in a HIP graph and replayed."""
    import torch

    import paper_2402_11354_amd as P
    import workloads as W
    from paper_2402_11354_amd import autotune

    name = args.workload if args.workload != "sift_like_1m_d128" else "deep_like_10m_d96"
    w, x, q, g, entry, index, gt_d = _setup(name, args.n, args.nq, 100)
    dev = torch.device("cuda:0")
    nq = w.nq
    k, ef = W.query_params(w, nq)
    kt, eft = torch.from_numpy(k).to(dev), torch.from_numpy(ef).to(dev)
    qt = torch.from_numpy(q).to(dev)
    kmax, efmax = int(k.max()), int(ef.max())
    ids = torch.empty((nq, kmax), dtype=torch.int64, device=dev)
    dists = torch.empty((nq, kmax), dtype=torch.float32, device=dev)
    stats = torch.empty((nq, P.PEOS_NSTATS), dtype=torch.int32, device=dev)
    out = {}
    # stopping rules: the HNSW rule (pool = ef) and a queue of twice each
    # query's ef (the bounded form of the printed Alg. 1)
    for pool, rule in ((1, "hnsw"), (-2, "queue_2ef")):
        ws = torch.empty(P.peos_search_ws_bytes(index, nq, efmax, pool), dtype=torch.uint8,
                         device=dev)
        for mode, label in ((P.PEOS_MODE_PEOS, "peos"), (P.PEOS_MODE_EXHAUSTIVE, "exhaustive")):
            caps = autotune.tune_classes(index, qt, k, ef, pool=pool, eps=w.eps, mode=mode,
                                         log=log)
            gr = P.peos_graph_create(index, qt, kt, eft, kmax, pool, w.eps, mode, ids, dists,
                                     stats, ws, k_all=kmax, ef_all=efmax)
            for _ in range(args.warmup):
                gr.launch()
            torch.cuda.synchronize()
            evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                   for _ in range(args.steps)]
            t0 = time.perf_counter()
            for e0, e1 in evs:
                e0.record()
                gr.launch()
                e1.record()
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            gr.close()
            for c in range(8):
                P.peos_set_class_tuning(index, c)
            ms = np.array([a.elapsed_time(b) for a, b in evs])
            st = stats.cpu().numpy()
            ii = ids.cpu().numpy()
            rec = {}
            for kc in (1, 10, 100):
                sel = np.nonzero(k == kc)[0]
                rec[f"k={kc}"] = round(float(_recall(x, q[sel], ii[sel], gt_d[sel, :kc], kc,
                                                     w.metric).mean()), 4)
            sel = np.nonzero(k >= 10)[0]
            rec["recall@10 (k>=10)"] = round(float(_recall(x, q[sel], ii[sel], gt_d[sel, :10],
                                                           10, w.metric).mean()), 4)
            alg = search_alg_bytes(st, index.layout(), np.asarray(k, np.float64), 0)
            r = dict(qps=round(nq * args.steps / wall, 1), ms=round(float(ms.mean()), 4),
                     p99_ms=round(float(np.percentile(ms, 99)), 4), recall=rec,
                     ndist=round(float(st[:, 9].mean()), 1),
                     expansions=round(float(st[:, 0].mean()), 1),
                     gbs=round(float(alg / (ms.mean() / 1e3) / 1e9), 1),
                     class_hash_caps={str(c): v for c, v in caps.items()},
                     class_waves={str(c): v for c, v in index.tuned_class_waves.items()})
            out[f"{label}_{rule}"] = r
            log(f"batched {label} {rule}: {r}")
    pe, ex = out["peos_queue_2ef"], out["exhaustive_queue_2ef"]
    print(json.dumps({
        "metric": "QPS of one launch over a batch of uneven k/ef (batched persistent form)",
        "value": pe["qps"], "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": pe["ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "nq": nq, "d": w.d, "R": w.R, "L": w.L, "m": w.m,
                   "eps": w.eps, "k": "U{1,10,100}", "ef": "U{32,64,128,256}, max(ef,k)",
                   "stop_rule": "queue of 2 ef per query", "launch": "hip graph, ef classes"},
        "runs": out,
        "speedup_vs_exhaustive": round(pe["qps"] / ex["qps"], 3),
        "roofline": {"bound": "hbm", "achieved": pe["gbs"], "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(pe["gbs"] / PEAK_HBM_GBS, 4), "traffic": None},
    }), flush=True)


def precision(args):
    """The precision form (bfloat16 traversal copy, half scalars and tables,
    single-precision re-rank) against the full-precision path on the same
    graph: QPS at recall >= target for k = 10 and k = 100, recall loss at
    equal ef, and the distance error of every returned result."""
    import torch

    import paper_2402_11354_amd as P
    import workloads as W
    from paper_2402_11354_amd import autotune

    name = args.prec_workload
    w, x, q, g, entry, index, gt_d = _setup(name, args.n, args.nq, 100)
    if args.no_long_rows:
        P.peos_set_long_rows(index, False)
    dev = torch.device("cuda:0")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    A, B = W.directions_for(w)
    lowp = P.peos_build_tables(index._keep[0], index._keep[1], entry, w.L, w.m, T(A), T(B),
                               w.metric, flags=P.PEOS_FLAG_BF16_BASE | P.PEOS_FLAG_FP16)
    qt = T(q)
    nq = w.nq
    xs = torch.from_numpy(x).to(dev).double()
    qs = qt.double()
    result = {}
    plan = ((10, (32, 64, 128, 192, 256, 384, 512)), (100, (128, 192, 256, 384, 512, 768, 1024)))
    if args.prec_ef:
        plan = ((10, (args.prec_ef,)),)
    for k, efs in plan:
        ws = torch.empty(P.peos_search_ws_bytes(index, nq, max(efs), max(efs)),
                         dtype=torch.uint8, device=dev)
        rows = {}
        for label, ix in (("fp32", index), ("precision", lowp)):
            pts = []
            for ef in efs:
                # waves per query for this point (the batch of 1,000 queries
                # leaves the chip room for 2 or 4 waves each)
                autotune.tune(ix, qt, k, ef, pool=ef, eps=w.eps, caps=(0,), waves=(1, 2, 4),
                              reps=2, use_cache=False)
                ids, dd, st = P.search(ix, qt, k, ef, eps=w.eps, pool=ef, ws=ws)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(args.steps):
                    P.search(ix, qt, k, ef, eps=w.eps, pool=ef, ws=ws)
                torch.cuda.synchronize()
                qps = nq * args.steps / (time.perf_counter() - t0)
                ii = ids.cpu().numpy()
                rec = float(_recall(x, q, ii, gt_d[:, :k], k, w.metric).mean())
                if w.metric == W.L2:
                    d64 = ((xs[ids] - qs[:, None, :]) ** 2).sum(-1)
                else:
                    d64 = 1.0 - (xs[ids] * qs[:, None, :]).sum(-1) / qs.norm(dim=1)[:, None]
                err = ((dd.double() - d64).abs() / d64.clamp(min=1e-30)).max().item()
                pts.append(dict(ef=ef, recall=round(rec, 4), qps=round(qps, 1),
                                max_rel_dist_err=err, waves_per_query=ix.tuned_waves,
                                **alg_rate(st.cpu().numpy(), ix.layout(), k, ef, qps)))
                log(f"precision k={k} {label} ef={ef}: recall={rec:.4f} qps={qps:.0f} "
                    f"max rel err={err:.2e} waves/query={ix.tuned_waves}")
            ok = [p_ for p_ in pts if p_["recall"] >= args.target]
            rows[label] = dict(points=pts, at_target=(max(ok, key=lambda p_: p_["qps"])
                                                      if ok else None))
        if k == 10 and not args.prec_ef:
            # the same sweep with the test off (exhaustive-neighbour search)
            pts = []
            for ef in efs:
                autotune.tune(index, qt, k, ef, pool=ef, eps=w.eps, mode=P.PEOS_MODE_EXHAUSTIVE,
                              caps=(0,), waves=(1, 2, 4), reps=2, use_cache=False)
                ids, dd, st = P.search(index, qt, k, ef, mode=P.PEOS_MODE_EXHAUSTIVE, pool=ef,
                                       ws=ws)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(args.steps):
                    P.search(index, qt, k, ef, mode=P.PEOS_MODE_EXHAUSTIVE, pool=ef, ws=ws)
                torch.cuda.synchronize()
                qps = nq * args.steps / (time.perf_counter() - t0)
                rec = float(_recall(x, q, ids.cpu().numpy(), gt_d[:, :k], k, w.metric).mean())
                pts.append(dict(ef=ef, recall=round(rec, 4), qps=round(qps, 1),
                                waves_per_query=index.tuned_waves,
                                **alg_rate(st.cpu().numpy(), index.layout(), k, ef, qps)))
                log(f"precision k={k} exhaustive ef={ef}: recall={rec:.4f} qps={qps:.0f} "
                    f"waves/query={index.tuned_waves}")
            ok = [p_ for p_ in pts if p_["recall"] >= args.target]
            rows["exhaustive_fp32"] = dict(points=pts, at_target=(max(ok, key=lambda p_: p_["qps"])
                                                                  if ok else None))
            rows["interpolated_at_target"] = {
                lab: _interp([(p_["recall"], p_["qps"]) for p_ in rows[lab]["points"]],
                             args.target)
                for lab in ("fp32", "precision", "exhaustive_fp32")}
        loss = [round(a_["recall"] - b_["recall"], 4)
                for a_, b_ in zip(rows["fp32"]["points"], rows["precision"]["points"])]
        rows["recall_loss_at_equal_ef"] = dict(zip([str(e) for e in efs], loss))
        result[f"k={k}"] = rows
    r10 = result["k=10"]
    val = r10["precision"]["at_target"]
    print(json.dumps({
        "metric": "QPS at recall@10>=0.95, precision form vs fp32 path (same graph)",
        "value": val["qps"] if val else None, "unit": "queries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16/f16 storage, f32 arithmetic",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "nq": nq, "d": w.d, "R": w.R, "L": w.L,
                   "m": w.m, "eps": w.eps, "stop_rule": "hnsw (pool=ef)"},
        "results": result,
    }), flush=True)


def compact(args):
    """The compact records (L = --compact-L, default 2; w_reg = 1, w_res = 0, two 8-bit scalars per
    edge, quantile table) against the full records at the workload's L, on the
    same graph, under the HNSW stopping rule: QPS at recall@10 >= target over
    an ef sweep, and the bytes of an edge record."""
    import torch

    import paper_2402_11354_amd as P
    import workloads as W

    w, x, q, g, entry, index, gt_d = _setup(args.workload, args.n, args.nq, 10)
    dev = torch.device("cuda:0")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    Lc = args.compact_L
    Ac, Bc = W.make_directions(Lc, w.m, w.d, w.seed + 2000)
    comp = P.peos_build_tables(index._keep[0], index._keep[1], entry, Lc, w.m, T(Ac), T(Bc),
                               w.metric, flags=P.PEOS_FLAG_COMPACT)
    qt = T(q)
    nq = w.nq
    efs = [int(e) for e in args.efs.split(",")]
    ws = torch.empty(P.peos_search_ws_bytes(index, nq, max(efs), max(efs)), dtype=torch.uint8,
                     device=dev)
    rows = {}
    runs = [("full_L%d" % w.L, index, P.PEOS_MODE_PEOS, e) for e in (0.1, 0.2)]
    runs += [("compact_L%d" % Lc, comp, P.PEOS_MODE_PEOS, e) for e in (0.1, 0.2)]
    runs += [("exhaustive", index, P.PEOS_MODE_EXHAUSTIVE, 0.1)]
    for label, ix, mode, eps in runs:
        key = label if mode == P.PEOS_MODE_EXHAUSTIVE else f"{label}_eps{eps}"
        pts = []
        for ef in efs:
            ids, dd, st = P.search(ix, qt, 10, ef, eps=eps, mode=mode, pool=ef, ws=ws)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                P.search(ix, qt, 10, ef, eps=eps, mode=mode, pool=ef, ws=ws)
            torch.cuda.synchronize()
            qps = nq * args.steps / (time.perf_counter() - t0)
            rec = float(_recall(x, q, ids.cpu().numpy(), gt_d, 10, w.metric).mean())
            s_ = st.cpu().numpy()
            pts.append(dict(ef=ef, recall=round(rec, 4), qps=round(qps, 1),
                            ndist=round(float(s_[:, 9].mean()), 1),
                            tests=round(float(s_[:, 3].mean()), 1),
                            **alg_rate(s_, ix.layout(), 10, ef, qps)))
            log(f"compact {key} ef={ef}: recall={rec:.4f} qps={qps:.0f}")
            if rec >= args.target + 0.02:
                break
        ok = [p_ for p_ in pts if p_["recall"] >= args.target]
        rows[key] = dict(points=pts, at_target=(max(ok, key=lambda p_: p_["qps"]) if ok else None))
    best = lambda pre: max((r["at_target"] for k_, r in rows.items()
                            if k_.startswith(pre) and r["at_target"]),
                           key=lambda p_: p_["qps"], default=None)
    c, f, e = best("compact"), best("full"), best("exhaustive")
    lay_c, lay_f = comp.layout(), index.layout()
    print(json.dumps({
        "metric": "QPS at recall@10>=0.95, compact records vs full records (same graph)",
        "value": c["qps"] if c else None, "unit": "queries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 (8-bit edge scalars)",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "nq": nq, "d": w.d, "R": w.R, "m": w.m,
                   "L_full": w.L, "L_compact": Lc, "stop_rule": "hnsw (pool=ef)"},
        "record_bytes_per_node": {"full": lay_f.node_stride, "compact": lay_c.node_stride},
        "at_target": {"compact": c, "full": f, "exhaustive": e},
        "runs": rows,
    }), flush=True)


def descent(args):
    """Search from the node a greedy descent through HNSW-style upper layers
    reaches, against search from the fixed entry (the medoid), on the same
    base graph, under the HNSW stopping rule: QPS at recall@10 >= target over
    an ef sweep, PEOs and exhaustive, with the descent inside the timed
    region."""
    import torch

    import paper_2402_11354_amd as P
    import workloads as W

    w, x, q, g, entry, index, gt_d = _setup(args.workload, args.n, args.nq, 10)
    dev = torch.device("cuda:0")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    t0 = time.time()
    lay = W.build_upper_layers(x, R_up=16, M=16, seed=w.seed, device=dev,
                               log=lambda m: log("layers:", m))
    log(f"upper layers: {len(lay['layer_start']) - 1} levels, {len(lay['node'])} rows in "
        f"{time.time() - t0:.1f}s")
    A, B = W.directions_for(w)
    hier = P.peos_build_tables(index._keep[0], index._keep[1], entry, w.L, w.m, T(A), T(B),
                               w.metric)
    P.peos_set_upper_layers(hier, dict(node=T(lay["node"]), adj=T(lay["adj"]),
                                       down=T(lay["down"]), top=lay["top"],
                                       layer_start=lay["layer_start"]))
    qt = T(q)
    nq = w.nq
    efs = [int(e) for e in args.efs.split(",")]
    ws = torch.empty(P.peos_search_ws_bytes(index, nq, max(efs), max(efs)), dtype=torch.uint8,
                     device=dev)
    rows = {}
    runs = []
    for label, ix in (("medoid", index), ("descent", hier)):
        runs += [(f"{label}_peos_eps{e}", ix, P.PEOS_MODE_PEOS, e) for e in (0.1, 0.2)]
        runs += [(f"{label}_exhaustive", ix, P.PEOS_MODE_EXHAUSTIVE, 0.1)]
    for key, ix, mode, eps in runs:
        pts = []
        for ef in efs:
            ids, dd, st = P.search(ix, qt, 10, ef, eps=eps, mode=mode, pool=ef, ws=ws)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                P.search(ix, qt, 10, ef, eps=eps, mode=mode, pool=ef, ws=ws)
            torch.cuda.synchronize()
            qps = nq * args.steps / (time.perf_counter() - t0)
            rec = float(_recall(x, q, ids.cpu().numpy(), gt_d, 10, w.metric).mean())
            s_ = st.cpu().numpy()
            pts.append(dict(ef=ef, recall=round(rec, 4), qps=round(qps, 1),
                            expansions=round(float(s_[:, 0].mean()), 1),
                            ndist=round(float(s_[:, 9].mean()), 1),
                            descent_ndist=round(float(s_[:, 12].mean()), 1),
                            **alg_rate(s_, ix.layout(), 10, ef, qps)))
            log(f"descent {key} ef={ef}: recall={rec:.4f} qps={qps:.0f} "
                f"expansions={pts[-1]['expansions']} descent={pts[-1]['descent_ndist']}")
            if rec >= args.target + 0.02:
                break
        ok = [p_ for p_ in pts if p_["recall"] >= args.target]
        rows[key] = dict(points=pts, at_target=(max(ok, key=lambda p_: p_["qps"]) if ok else None))
    best = lambda pre: max((r["at_target"] for k_, r in rows.items()
                            if k_.startswith(pre) and r["at_target"]),
                           key=lambda p_: p_["qps"], default=None)
    res = {k_: best(k_) for k_ in ("medoid_peos", "medoid_exhaustive", "descent_peos",
                                   "descent_exhaustive")}
    v = res["descent_peos"]
    print(json.dumps({
        "metric": "QPS at recall@10>=0.95, search from the upper-layer descent vs from the medoid",
        "value": v["qps"] if v else None, "unit": "queries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "nq": nq, "d": w.d, "R": w.R, "L": w.L,
                   "m": w.m, "upper_R": 16, "upper_M": 16,
                   "levels": len(lay["layer_start"]) - 1, "upper_rows": int(len(lay["node"])),
                   "stop_rule": "hnsw (pool=ef)"},
        "at_target": res,
        "runs": rows,
    }), flush=True)


def serving(args):
    """The request loop under Poisson arrivals: requests of 1..64 queries,
    k in {10, 100}, ef in {32, ..., 512}; p50/p99 latency from arrival to
    completion, completed queries per second, recall@10 of what completed."""
    import paper_2402_11354_amd as P

    name = args.workload if args.workload != "sift_like_1m_d128" else "serving_1m_d256"
    w, x, q, g, entry, index, gt_d = _setup(name, args.n, args.nq, 10)
    rng = np.random.default_rng(w.seed + 11)
    srv = P.Server(index, max_batch=2048, max_k=100, max_ef=512, max_inflight=4,
                   max_pending=1 << 18, pool=1, eps=w.eps, hbm_budget=32 << 30)
    per_rate = []
    hits, total = 0.0, 0
    try:
        for _ in range(16):  # warm-up through every slot
            srv.submit(q[:64], 100, 512)
        while srv.live:
            srv.poll(wait=True)
        for rate in [float(r) for r in args.rates.split(",")]:
            mean_req = 32.5  # queries per request, U{1..64}
            n_req = max(8, int(rate / mean_req * args.seconds))
            arrive = np.cumsum(rng.exponential(mean_req / rate, size=n_req))
            sizes = rng.integers(1, 65, size=n_req)
            ks = rng.choice([10, 100], size=n_req)
            efs = np.maximum(rng.choice([32, 64, 128, 256, 512], size=n_req), ks)
            starts = rng.integers(0, len(q) - 64, size=n_req)
            c0 = srv.counters()
            lat = np.full(n_req, np.nan)
            tick = {}
            rejected = 0
            t0 = time.perf_counter()
            i = 0
            while i < n_req or srv.live:
                now = time.perf_counter() - t0
                while i < n_req and arrive[i] <= now:
                    s = int(starts[i])
                    try:
                        tick[srv.submit(q[s:s + sizes[i]], int(ks[i]), int(efs[i]))] = i
                    except P.PeosError as e:
                        if e.code != P.PEOS_EBUSY:
                            raise
                        rejected += 1
                    i += 1
                for t, ids, _ in srv.poll(wait=False):
                    j = tick.pop(t)
                    lat[j] = time.perf_counter() - t0 - arrive[j]
                    s = int(starts[j])
                    sl = slice(s, s + sizes[j])
                    rc = _recall(x, q[sl], ids[:, :10], gt_d[sl], 10, w.metric)
                    hits += float(rc.sum())
                    total += len(rc)
            elapsed = time.perf_counter() - t0
            c1 = srv.counters()
            done = np.isfinite(lat)
            batches = c1["launches"] - c0["launches"]
            r = dict(rate=rate, requests=n_req, rejected=rejected,
                     qps=round(float(sizes[done].sum()) / elapsed, 1),
                     p50_ms=round(float(np.percentile(lat[done], 50) * 1e3), 3),
                     p99_ms=round(float(np.percentile(lat[done], 99) * 1e3), 3),
                     batches=int(batches),
                     mean_batch=round((c1["queries"] - c0["queries"]) / max(1, batches), 1),
                     seconds=round(elapsed, 3))
            log(f"serving {r}")
            per_rate.append(r)
    finally:
        srv.close()
    top = max(per_rate, key=lambda r: r["qps"])
    print(json.dumps({
        "metric": "serving: completed queries/s under Poisson arrivals, p50/p99 latency",
        "value": top["qps"], "unit": "queries/s", "n_gpus": 1, "steps": len(per_rate),
        "warmup": 16, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "d": w.d, "R": w.R, "L": w.L, "m": w.m,
                   "eps": w.eps, "request_size": "U{1..64}", "k": "{10,100}",
                   "ef": "{32,64,128,256,512}, max(ef,k)", "max_batch": 2048,
                   "launch_slots": 4},
        "p50_ms": top["p50_ms"], "p99_ms": top["p99_ms"],
        "recall@10": round(hits / max(1, total), 4), "rates": per_rate,
    }), flush=True)


def measure_gather_ceiling(array_bytes, waves=4096, iters=64, reps=5):
    """GB/s of the calibration gather (random 512-byte rows, the search's
    pattern) over an array of array_bytes, or None if it cannot run."""
    import torch

    import paper_2402_11354_amd as P

    try:
        dev = torch.device("cuda:0")
        n = max(1, array_bytes // 512)
        x = torch.ones((n, 128), dtype=torch.float32, device=dev)
        sink = torch.empty(waves, dtype=torch.float32, device=dev)
        s = torch.cuda.current_stream()
        for _ in range(2):
            P.peos_probe_gather(x, waves, iters, sink)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            P.peos_probe_gather(x, waves, iters, sink)
        e1.record(s)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        gbs = waves * iters * 16 * 512 / (ms / 1e3) / 1e9
        log(f"gather ceiling over {array_bytes / 2**30:.2f} GiB: {gbs:.0f} GB/s")
        del x
        return round(gbs, 1)
    except (RuntimeError, P.PeosError) as e:
        log(f"gather ceiling not measured: {e}")
        return None


def gather_probe():
    """Random 512-byte row gathers by the library's calibration kernel (8
    lanes per row, 16 rows in flight per wave, the search's pattern) over
    arrays of 64 MB to 4 GB, timed with events on the launch stream: the
    practical HBM ceiling of the search's access pattern."""
    import torch

    import paper_2402_11354_amd as P

    dev = torch.device("cuda:0")
    iters = 64
    res = []
    for mb in (64, 512, 4096):
        n = (mb << 20) // 512
        x = torch.ones((n, 128), dtype=torch.float32, device=dev)
        for waves in (2048, 4096, 16384):
            sink = torch.empty(waves, dtype=torch.float32, device=dev)
            s = torch.cuda.current_stream()
            for _ in range(2):
                P.peos_probe_gather(x, waves, iters, sink)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 5
            e0.record(s)
            for _ in range(reps):
                P.peos_probe_gather(x, waves, iters, sink)
            e1.record(s)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            gbs = waves * iters * 16 * 512 / (ms / 1e3) / 1e9
            res.append({"array_mb": mb, "waves": waves, "ms": round(ms, 4),
                        "gbs": round(gbs, 1)})
            log(f"gather probe {mb} MB, {waves} waves: {ms:.3f} ms, {gbs:.0f} GB/s")
        del x
    print(json.dumps({"gather_probe": res, "row_bytes": 512, "iters": iters}), flush=True)


def cpu_baseline(x, g, entry, q, w, cfg, budget_s):
    """The oracle, as it stands, on the host cores: a bounded sample of the
    same queries at the same operating point, on all threads it is given and
    on one thread."""
    import oracle
    import workloads as W

    ef, pool, eps, mode = cfg
    A, B = W.directions_for(w)
    threads, host_cpus = cpu_share()
    out = {}

    def run(nq, nthreads):
        t0 = time.perf_counter()
        out["ref"] = oracle.search(x, g, entry, q[:nq], w.k, ef, w.L, w.m, A, B, w.metric, eps,
                                   mode=mode, pool=pool, nthreads=nthreads, precision=64)
        return time.perf_counter() - t0

    n = 32
    dt = run(n, threads)
    n2 = int(min(len(q), max(n, n * budget_s / max(dt, 1e-3))))
    dt = run(n2, threads)
    ref = out["ref"]
    log(f"cpu baseline: {n2} queries in {dt:.1f}s on {threads} threads ({host_cpus} visible)")
    n1 = int(min(len(q), max(8, n2 / max(1.0, dt) * 2.0 / threads)))
    dt1 = run(n1, 1)
    log(f"cpu baseline: {n1} queries in {dt1:.1f}s on 1 thread")
    return {"value": round(n2 / dt, 2), "unit": "queries/s", "cores": threads, "kind": "oracle",
            "host_cpus": host_cpus,
            "sample": f"first {n2} of the {len(q)} queries at the same ef/pool/eps "
                      f"(float64 oracle, one query per task on {threads} threads, the host "
                      f"CPU share of this process); single thread: first {n1}",
            "value_1thread": round(n1 / dt1, 2)}, ref


def cpu_share():
    """(threads the oracle runs on, CPUs the host shows).  The threads are
    the CPUs this process may run on, capped by OMP_NUM_THREADS when the
    environment sets the process's CPU share that way."""
    host = os.cpu_count() or 1
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = host
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n), host


def parity_summary(x, q, w, ids, dists, stats, ref, gt_ids):
    """The FP64 parity rule (tests/parity.py: ids equal except within 1e-5
    relative ties on non-fragile queries, distances within 1e-5 relative,
    recall@10 within 0.3 points) on the queries the oracle ran."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from parity import compare64

    nq = ref["ids"].shape[0]
    r = compare64(ids[:nq], dists[:nq], ref, w.k, x, q[:nq], w.metric, gt=gt_ids[:nq],
                  stats=stats[:nq], recall_k=min(10, w.k))
    bad = [b for b in r["bad"] if b[0] >= 0]
    return {"rule": "fp64 oracle: non-fragile ids equal up to 1e-5 ties, counters equal, "
                    "distances within 1e-5 relative, recall@10 within 0.003",
            "queries": nq, "checked": r["checked"], "fragile": r["fragile"],
            "fragile_flags": r["flags"], "mismatched": len(bad),
            "same_ids_all": round(r["same_ids"], 5),
            "max_rel_dist_err": r["max_rel_err"],
            "recall_gpu": round(r["recall_gpu"], 5), "recall_oracle": round(r["recall_oracle"], 5),
            "recall_diff": round(r["recall_gpu"] - r["recall_oracle"], 5),
            "pass": not r["bad"]}


if __name__ == "__main__":
    main()
