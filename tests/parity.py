"""Comparison of GPU search results with the oracle.

Two rules, both applied by the GPU parity tests:

compare64 -- against the oracle run in double precision (precision=64), the
  arbiter: the oracle's distances, list order, delta and routing test are all
  FP64.  A query whose oracle path holds a decision within tau = 1e-5 of its
  boundary (|H - T| relative, A_r within 1e-5 of 1 or of 0 unless the
  numerator's sign is exact in single precision too, two list distances or a
  distance and delta within 1e-5 relative unless both are computed exactly in
  single precision) is *fragile*: counted, reported, judged by recall only.
  Every other query must return the oracle's top-k ids, except at positions
  where the two distances (the GPU's pick and the oracle's, both in FP64) lie
  within 1e-5 relative of each other; every returned distance must lie within
  1e-5 relative (1e-6 absolute near zero) of the FP64 distance of the same
  pair; and mean recall@k against exact k-NN must be within 0.3 points of the
  oracle's.

compare -- against the oracle's precision=32 mode, a second, stricter check:
  that mode takes the distance decisions on the canonical single-precision
  distances (one fixed summation order, the kernel's) while the routing test
  stays FP64, so every query that is not fragile (test decisions only) must
  return exactly the oracle's ids, single-precision distances and per-query
  counters.
"""
import os

import numpy as np

TOL = 1e-5
RECALL_TOL = 0.003

FLAG_NAMES = (("H~T", 1), ("A~1", 2), ("A~0", 4), ("d~delta", 8), ("order", 16))


def _counter_rows(stats, ref, q):
    row = np.asarray(stats)[q]
    # counters 0..10 of the kernel, and its count of expansions that ran the
    # test (stat 13) against the oracle's 12th counter
    if row.shape[0] >= 14:
        return np.concatenate([row[:11], row[13:14]]), ref["counters"][q][:12]
    return row[:11], ref["counters"][q][:11]


def compare(ids, dists, stats, ref, k, check_counters=True):
    """Exact rule against the precision=32 oracle.
    Returns dict(checked, fragile, flags, bad=[(query, reason)])."""
    ids = np.asarray(ids)[:, :k]
    dists = np.asarray(dists)[:, :k]
    rids = ref["ids"][:, :k]
    rd = ref["dist"][:, :k]
    rd64 = ref["dist64"][:, :k]
    frag = ref["fragile"] != 0
    bad = []
    checked = 0
    for q in range(len(ids)):
        if frag[q]:
            continue
        checked += 1
        if not np.array_equal(ids[q], rids[q]):
            bad.append((q, f"ids {ids[q].tolist()} vs {rids[q].tolist()}"))
            continue
        if not np.array_equal(dists[q].astype(np.float64), rd[q]):
            bad.append((q, f"dists {dists[q].tolist()} vs {rd[q].tolist()}"))
            continue
        if check_counters and stats is not None:
            g, r = _counter_rows(stats, ref, q)
            if not np.array_equal(g, r):
                bad.append((q, f"counters {g.tolist()} vs {r.tolist()}"))
    # precision of every returned distance against float64
    valid = ids >= 0
    d32 = dists.astype(np.float64)
    same = (ids == rids) & valid
    err = np.abs(d32[same] - rd64[same])
    lim = TOL * np.abs(rd64[same]) + 1e-6
    if np.any(err > lim):
        bad.append((-1, f"{int((err > lim).sum())} distances beyond 1e-5 relative of float64"))
    flags = {name: int(((ref["fragile"] & bit) != 0).sum()) for name, bit in FLAG_NAMES}
    return dict(checked=checked, fragile=int(frag.sum()), flags=flags, bad=bad)


def pair_dist64(base, queries, ids, metric):
    """FP64 distance of every (query, id) pair (ids < 0 give +inf): squared
    l2, 1 - x.q/|q| or -x.q."""
    ids = np.asarray(ids)
    out = np.full(ids.shape, np.inf)
    qs = np.asarray(queries, np.float64)
    for qi in range(ids.shape[0]):
        sel = ids[qi] >= 0
        if not sel.any():
            continue
        xb = np.asarray(base[ids[qi][sel]], np.float64)
        q = qs[qi]
        if metric == 0:
            out[qi, sel] = ((xb - q) ** 2).sum(1)
        elif metric == 2:
            out[qi, sel] = -(xb @ q)
        else:
            out[qi, sel] = 1.0 - xb @ q / np.linalg.norm(q)
    return out


def recall_of(ids, gt, k):
    """Mean |top-k ids ∩ exact top-k| / k."""
    ids = np.asarray(ids)[:, :k]
    gt = np.asarray(gt)[:, :k]
    return float(np.mean([len(set(a[a >= 0].tolist()) & set(b.tolist())) / k
                          for a, b in zip(ids, gt)]))


def compare64(ids, dists, ref64, k, base, queries, metric, gt=None, stats=None,
              check_counters=True, recall_k=10, recall_min_queries=50):
    """The rule against the FP64 oracle (see the module docstring).

    ref64: oracle.search(..., precision=64).  gt: exact top-k ids (FP64 brute
    force) for the recall rule, or None to skip it; the rule is applied
    when the batch has at least recall_min_queries queries (below that, one
    fragile query taking another path moves the mean by more than the
    tolerance) and reported always.  stats: the kernel's
    per-query counters; on a non-fragile query the path is the oracle's, so
    they must equal its counters (a stricter check than the ids).
    Returns dict(checked, fragile, flags, bad, same_ids (fraction of all
    queries with identical top-k ids), max_rel_err (largest relative error
    of a returned distance against FP64), recall_gpu, recall_oracle)."""
    ids = np.asarray(ids)[:, :k]
    dists = np.asarray(dists)[:, :k].astype(np.float64)
    rids = ref64["ids"][:, :k]
    rd = ref64["dist"][:, :k]
    frag = ref64["fragile"] != 0
    g64 = pair_dist64(base, queries, ids, metric)
    bad = []
    checked = 0
    for q in range(len(ids)):
        if frag[q]:
            continue
        checked += 1
        if np.array_equal(ids[q], rids[q]):
            pass
        else:
            vg, vr = ids[q] >= 0, rids[q] >= 0
            diff = np.nonzero(ids[q] != rids[q])[0]
            a, b = g64[q, diff], rd[q, diff]
            tie = (vg[diff] & vr[diff]
                   & (np.abs(a - b) <= TOL * np.maximum(np.abs(a), np.abs(b))))
            valid = ids[q][vg]
            if not tie.all() or len(np.unique(valid)) != len(valid):
                bad.append((q, f"ids {ids[q].tolist()} vs {rids[q].tolist()}"))
                continue
        if check_counters and stats is not None:
            gc, rc = _counter_rows(stats, ref64, q)
            if not np.array_equal(gc, rc):
                bad.append((q, f"counters {gc.tolist()} vs {rc.tolist()}"))
    valid = ids >= 0
    err = np.abs(dists[valid] - g64[valid])
    lim = TOL * np.abs(g64[valid]) + 1e-6
    if np.any(err > lim):
        bad.append((-1, f"{int((err > lim).sum())} distances beyond 1e-5 relative of float64"))
    rel = err / np.maximum(np.abs(g64[valid]), 1e-30)
    out = dict(checked=checked, fragile=int(frag.sum()),
               flags={name: int(((ref64["fragile"] & bit) != 0).sum())
                      for name, bit in FLAG_NAMES},
               bad=bad, same_ids=float(np.mean(np.all(ids == rids, axis=1))) if len(ids) else 1.0,
               max_rel_err=float(rel.max()) if rel.size else 0.0,
               recall_gpu=None, recall_oracle=None)
    if gt is not None and len(ids):
        kk = min(recall_k, k)
        out["recall_gpu"] = recall_of(ids, gt, kk)
        out["recall_oracle"] = recall_of(rids, gt, kk)
        if (len(ids) >= recall_min_queries
                and abs(out["recall_gpu"] - out["recall_oracle"]) > RECALL_TOL + 1e-12):
            bad.append((-2, f"recall@{kk} {out['recall_gpu']:.4f} vs oracle "
                            f"{out['recall_oracle']:.4f}"))
    return out


def check_both(gpu, x, g, entry, q, k, ef, L, m, A, B, metric, eps, min_checked=0.8,
               counters=True, label="", extra_fragile=None, gt=None, min_same=0.95, **kw):
    """Run the oracle in both precisions on the GPU's inputs and apply both
    rules.  gpu = (ids, dists, stats) as numpy arrays; kw goes to
    oracle.search (mode, pool, kstride, perm, simhash, entries ...); with
    entries, kw may hold entries64 (the FP64 descent's entries) for the FP64
    run; extra_fragile (nq bools) marks queries fragile before the search
    (a fragile descent).  min_checked: least fraction of the queries that
    must be non-fragile under the FP64 rule; min_same: least fraction of all
    the queries, fragile ones included, whose top-k ids equal the FP64
    oracle's (a fragile decision may go either way, but rarely does).  gt:
    exact top-10 ids of q (FP64
    brute force), computed here when None.  Returns (res32, res64)."""
    import oracle as O

    ids, dists, stats = gpu
    kw64 = dict(kw)
    if "entries64" in kw:
        kw64["entries"] = kw64.pop("entries64")
        kw.pop("entries64")
    ref32 = O.search(x, g, entry, q, k, ef, L, m, A, B, metric, eps, precision=32, **kw)
    ref64 = O.search(x, g, entry, q, k, ef, L, m, A, B, metric, eps, precision=64, **kw64)
    if extra_fragile is not None:
        add = np.where(np.asarray(extra_fragile, bool), 16, 0).astype(np.int32)
        ref32["fragile"] = ref32["fragile"] | add
        ref64["fragile"] = ref64["fragile"] | add
    ks = ids.shape[1] if np.ndim(k) else int(k)
    kr = min(10, ks)
    if gt is None:
        gt, _ = O.brute_force(x, q, kr, metric)
    st = stats if counters else None
    r32 = compare(ids, dists, st, ref32, ks, check_counters=counters)
    r64 = compare64(ids, dists, ref64, ks, x, q, metric, gt=gt, stats=st, check_counters=counters,
                    recall_k=kr)
    print(f"[gpu] {label}: fp64 rule checked={r64['checked']}/{len(ids)} fragile={r64['fragile']} "
          f"{r64['flags']} same_ids={r64['same_ids']:.3f} max_rel_err={r64['max_rel_err']:.2e} "
          f"recall gpu={r64['recall_gpu']:.4f} oracle={r64['recall_oracle']:.4f}; "
          f"fp32 rule checked={r32['checked']}", flush=True)
    assert not r64["bad"], r64["bad"][:5]
    assert not r32["bad"], r32["bad"][:5]
    assert r64["same_ids"] >= min_same, r64["same_ids"]
    if not os.environ.get("PEOS_PARITY_SURVEY"):
        assert r64["checked"] >= min_checked * len(ids), (r64["checked"], len(ids))
    else:
        print(f"[survey] {label}: checked {r64['checked']}/{len(ids)} min {min_checked}",
              flush=True)
    return r32, r64
