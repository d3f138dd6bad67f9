"""The parity rules themselves (tests/parity.py), on the CPU: the oracle's
single-precision mode stands in for a GPU result.  It must pass the FP64
rule, and each planted mistake (a wrong id, a distance off by 2e-5, a lost
neighbour in many queries, a changed counter) must fail it."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from parity import compare64, pair_dist64, recall_of


@pytest.fixture(scope="module")
def tiny():
    w = W.TINY
    x, q = W.make_base(w), W.make_queries(w)
    g, entry = W.build_graph(x, w.R, w.cand)
    A, B = W.directions_for(w)
    args = (x, g, entry, q, w.k, w.ef, w.L, w.m, A, B, w.metric, w.eps)
    r32 = O.search(*args, pool=w.ef, precision=32)
    r64 = O.search(*args, pool=w.ef, precision=64)
    gt, _ = O.brute_force(x, q, w.k, w.metric)
    return w, x, q, r32, r64, gt


def fake_stats(ref):
    """Counters laid out as the kernel's 14 statistics."""
    c = ref["counters"]
    st = np.zeros((len(c), 14), np.int64)
    st[:, :11] = c[:, :11]
    st[:, 13] = c[:, 11]
    return st


def test_single_precision_oracle_passes_the_fp64_rule(tiny):
    w, x, q, r32, r64, gt = tiny
    res = compare64(r32["ids"], r32["dist"], r64, w.k, x, q, w.metric, gt=gt,
                    stats=fake_stats(r32))
    assert not res["bad"], res["bad"][:3]
    assert res["checked"] >= 0.75 * len(q)
    assert res["max_rel_err"] < 1e-5
    assert res["recall_gpu"] == pytest.approx(res["recall_oracle"], abs=0.003)


def test_wrong_id_fails(tiny):
    w, x, q, r32, r64, gt = tiny
    ids = r32["ids"].copy()
    qi = int(np.nonzero(r64["fragile"] == 0)[0][0])
    ids[qi, 3] = (ids[qi, 3] + 1) % x.shape[0]
    dists = r32["dist"].copy()
    dists[qi] = pair_dist64(x, q[qi:qi + 1], ids[qi:qi + 1], w.metric)[0]
    res = compare64(ids, dists, r64, w.k, x, q, w.metric)
    assert any(b[0] == qi for b in res["bad"])


def test_distance_off_by_2e5_fails(tiny):
    w, x, q, r32, r64, gt = tiny
    dists = r32["dist"].copy()
    dists[5, 2] *= 1 + 2e-5
    res = compare64(r32["ids"], dists, r64, w.k, x, q, w.metric)
    assert any(b[0] == -1 for b in res["bad"])


def test_recall_loss_fails(tiny):
    """Every query loses its own best neighbour (replaced by a far node):
    recall drops by 1 point, beyond the 0.3-point tolerance."""
    w, x, q, r32, r64, gt = tiny
    ids = r32["ids"].copy()
    far = np.argmax(pair_dist64(x, q, np.tile(np.arange(x.shape[0]), (len(q), 1)), w.metric), 1)
    ids[:, 0] = far
    res = compare64(ids, pair_dist64(x, q, ids, w.metric), r64, w.k, x, q, w.metric, gt=gt)
    assert any(b[0] == -2 for b in res["bad"])
    assert recall_of(ids, gt, 10) < recall_of(r64["ids"], gt, 10) - 0.003


def test_changed_counter_fails(tiny):
    w, x, q, r32, r64, gt = tiny
    st = fake_stats(r32)
    qi = int(np.nonzero(r64["fragile"] == 0)[0][0])
    st[qi, 9] += 1
    res = compare64(r32["ids"], r32["dist"], r64, w.k, x, q, w.metric, stats=st)
    assert any(b[0] == qi and "counters" in b[1] for b in res["bad"])


def test_tie_exemption_allows_swapped_equal_distances(tiny):
    """Two results at positions of equal FP64 distance may come in either
    order: planted as a duplicated base row."""
    w, x, q, r32, r64, gt = tiny
    x2 = x.copy()
    qi = 0
    a, b = int(r64["ids"][qi, 3]), int(r64["ids"][qi, 4])
    x2[b] = x2[a]
    ids = r64["ids"].copy()
    ids[qi, 3], ids[qi, 4] = b, a
    ref = dict(r64)
    ref["ids"] = r64["ids"].copy()
    ref["dist"] = pair_dist64(x2, q, ref["ids"], w.metric)
    ref["fragile"] = r64["fragile"].copy()
    ref["fragile"][qi] = 0
    res = compare64(ids, pair_dist64(x2, q, ids, w.metric), ref, w.k, x2, q, w.metric,
                    check_counters=False)
    assert not [bb for bb in res["bad"] if bb[0] == qi]
