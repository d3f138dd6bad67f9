"""Comparison of GPU search results with the oracle.

Rules (the FP32 GPU path against the float64 oracle):
  * a query whose oracle path has a fragile decision (a test with |H - T|,
    |A_r - 1| or |A_r| within 1e-5 relative, a distance within 1e-5 relative
    of delta, or two list entries within 1e-5 relative) may legitimately take
    another path in single precision: it is counted and judged by recall only;
  * every other query must return the oracle's ids, except that two results
    whose oracle distances lie within 1e-5 relative may swap, with distances
    within 1e-5 relative (plus 1e-6 absolute for angular distances near 0),
    and identical per-query counters.
"""
import numpy as np

TOL = 1e-5


def _near(a, b, tol=TOL, atol=1e-6):
    return abs(a - b) <= tol * max(abs(a), abs(b)) + atol


def compare(ids, dists, stats, ref, k, check_counters=True):
    """Returns dict(checked, fragile, bad=[(query, reason)])."""
    ids = np.asarray(ids)[:, :k]
    dists = np.asarray(dists, np.float64)[:, :k]
    rids = ref["ids"][:, :k]
    rd = ref["dist"][:, :k]
    frag = ref["fragile"] != 0
    bad = []
    checked = 0
    for q in range(len(ids)):
        if frag[q]:
            continue
        checked += 1
        for i in range(k):
            a, b = ids[q, i], rids[q, i]
            if b < 0 or a < 0:
                if a != b:
                    bad.append((q, f"padding differs at {i}: {a} vs {b}"))
                    break
                continue
            if not _near(dists[q, i], rd[q, i]):
                bad.append((q, f"distance {i}: {dists[q, i]!r} vs {rd[q, i]!r}"))
                break
            if a != b:
                # allowed only between results with near-equal oracle distances
                where = np.nonzero(rids[q] == a)[0]
                j = where[0] if len(where) else None
                if j is None:
                    ok = i == k - 1 or _near(rd[q, i], rd[q, -1])
                else:
                    ok = _near(rd[q, i], rd[q, j])
                if not ok:
                    bad.append((q, f"id {i}: {a} vs {b}"))
                    break
        if check_counters and stats is not None:
            g = np.asarray(stats)[q, :11]
            r = ref["counters"][q]
            if not np.array_equal(g, r):
                bad.append((q, f"counters {g.tolist()} vs {r.tolist()}"))
    return dict(checked=checked, fragile=int(frag.sum()), bad=bad)
