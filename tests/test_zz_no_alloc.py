"""peos_search_static (no workspace: the library's device scratch array),
through the C ABI, against peos_search on the same inputs: identical ids,
distances and counters on two calls in a row, the second with a smaller
batch of per-query k and ef (so the class split also runs in the scratch),
and the FP64 parity rule on the first; a batch whose per-query part does
not fit the scratch is refused before any work."""
import ctypes

import numpy as np
import pytest

import workloads as W
from parity import check_both

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2402_11354_amd")

pytestmark = pytest.mark.gpu


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda:0"))


def ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def static_call(index, q, k, ef, k_all, ef_all, kstride, pool, eps):
    nq = q.shape[0]
    ids = torch.full((nq, kstride), -7, dtype=torch.int64, device=q.device)
    dists = torch.full((nq, kstride), -7.0, dtype=torch.float32, device=q.device)
    stats = torch.full((nq, P.PEOS_NSTATS), -7, dtype=torch.int32, device=q.device)
    kt = k if torch.is_tensor(k) else None
    et = ef if torch.is_tensor(ef) else None
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = P.lib().peos_search_static(index.handle, ptr(q), nq, ptr(kt), ptr(et), k_all, ef_all,
                                    kstride, pool, ctypes.c_float(eps), P.PEOS_MODE_PEOS,
                                    ptr(ids), ptr(dists), ptr(stats), stream)
    torch.cuda.synchronize()
    return rc, ids, dists, stats


@pytest.fixture(scope="module")
def case():
    w = W.TINY
    x, q = W.make_base(w), W.make_queries(w)
    g, entry = W.build_graph(x, w.R, w.cand)
    A, B = W.directions_for(w)
    index = P.peos_build_tables(T(x), T(g), entry, w.L, w.m, T(A), T(B), w.metric)
    return w, x, q, g, entry, A, B, index


def test_static_search_equals_workspace_search(case):
    w, x, q, g, entry, A, B, index = case
    qt = T(q)
    # call 1: the whole batch, one k and ef
    print("[gpu] static search: call 1, 100 queries", flush=True)
    rc, ids, dists, stats = static_call(index, qt, None, None, w.k, w.ef, w.k, w.ef, w.eps)
    assert rc == P.PEOS_OK, P.lib().peos_last_error()
    ref = P.search(index, qt, w.k, w.ef, eps=w.eps, pool=w.ef)
    torch.cuda.synchronize()
    assert torch.equal(ids, ref[0]) and torch.equal(dists, ref[1]) and torch.equal(stats, ref[2])
    check_both((ids.cpu().numpy(), dists.cpu().numpy(), stats.cpu().numpy()), x, g, entry, q,
               w.k, w.ef, w.L, w.m, A, B, w.metric, w.eps, pool=w.ef, min_checked=0.65,
               label="static search")
    # call 2: a smaller batch with per-query k and ef (class split)
    print("[gpu] static search: call 2, 37 queries, per-query k and ef", flush=True)
    rng = np.random.default_rng(5)
    k = rng.choice([1, 5, 10, 20], size=37).astype(np.int32)
    ef = rng.choice([16, 32, 64, 128], size=37).astype(np.int32)
    q2 = qt[20:57].contiguous()
    rc, ids2, dists2, stats2 = static_call(index, q2, T(k), T(ef), 20, 128, 20, 1, w.eps)
    assert rc == P.PEOS_OK, P.lib().peos_last_error()
    ref2 = P.search(index, q2, T(k), T(ef), eps=w.eps, pool=1, kstride=20)
    torch.cuda.synchronize()
    assert torch.equal(ids2, ref2[0]) and torch.equal(dists2, ref2[1])
    assert torch.equal(stats2, ref2[2])


def test_static_search_refuses_what_does_not_fit(case):
    w, x, q, g, entry, A, B, index = case
    # (L+1) m 4 + 12 bytes per query: 140,000 queries need about 46 MB of
    # tables alone; 240,000 about 79 MB, beyond the 64 MiB scratch
    nq = 240_000
    qt = torch.ones((nq, w.d), dtype=torch.float32, device="cuda:0")
    ids = torch.empty((nq, w.k), dtype=torch.int64, device="cuda:0")
    dists = torch.empty((nq, w.k), dtype=torch.float32, device="cuda:0")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = P.lib().peos_search_static(index.handle, ptr(qt), nq, None, None, w.k, w.ef, w.k, w.ef,
                                    ctypes.c_float(w.eps), P.PEOS_MODE_PEOS, ptr(ids), ptr(dists),
                                    None, stream)
    assert rc == P.PEOS_ENOSPACE
    assert b"scratch" in P.lib().peos_last_error()
