"""Comparison of GPU search results with the oracle.

The oracle runs with its distance decisions in single precision (the kernel's
precision, one fixed summation order), so the order of the candidate list,
delta and every insertion are decided on identical values on both sides.  The
routing test itself is evaluated in double precision by the oracle, so:
  * a query whose oracle path holds a fragile test decision (|H - T| within
    1e-5 relative, or A_r within 1e-5 of 1 or of 0) may legitimately take
    another path on the GPU: it is counted and judged by recall only;
  * every other query must return exactly the oracle's ids and single
    precision distances and identical per-query counters;
  * every returned distance must lie within 1e-5 relative (1e-6 absolute near
    zero) of the double-precision distance of the same pair.
"""
import numpy as np

TOL = 1e-5

FLAG_NAMES = (("H~T", 1), ("A~1", 2), ("A~0", 4), ("d~delta", 8), ("order", 16))


def compare(ids, dists, stats, ref, k, check_counters=True):
    """Returns dict(checked, fragile, flags, bad=[(query, reason)])."""
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
            row = np.asarray(stats)[q]
            # counters 0..10 of the kernel, and its count of expansions that
            # ran the test (stat 13) against the oracle's 12th counter
            if row.shape[0] >= 14:
                g = np.concatenate([row[:11], row[13:14]])
                r = ref["counters"][q][:12]
            else:
                g = row[:11]
                r = ref["counters"][q][:11]
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
