"""Proximity graph and ground truth for the synthetic workloads.

The graph is an input of the search, not part of PEOs: the paper plugs its
test into existing indexes (HNSW, NSSG; Sec. "Problem Definition" and the
experimental setup).  Here it is a pruned exact-kNN graph:

  1. candidates: the `cand` exact nearest neighbours of every node, ordered
     by (squared l2 distance, id), self excluded;
  2. relative-neighbourhood pruning: walk the candidates in order and keep c
     when dist(c, v) < dist(c, k) for every already-kept k, up to R kept;
  3. reverse edges: every kept edge v->u offers v as a candidate of u; when
     the union of u's kept list and its offers (closest `cand`, duplicates
     dropped) has at most R members u keeps all of them, otherwise the union
     is pruned again with rule 2 (the reverse-link rule of HNSW).

  4. connectivity: nodes not reachable from the entry are linked in, NSG
     style: an unreached node u whose candidate list holds a reached node with
     a free slot gets an edge from the first such node; when no unreached node
     has one, the unreached node of smallest id is linked from its nearest
     reached node that has a free slot.  Repeat until every node is reached.

The entry node is the medoid (exact for small n, nearest-to-mean otherwise).
Rows hold neighbour ids padded with -1 (pruned lists in ascending distance,
connectivity links appended).

Everything runs on torch, on the CPU in float64 for small inputs or on a GPU
in float32 (exact for integer-valued data, whose squared distances stay below
2**24).  The same code builds the graph for every consumer, so the search and
the oracle always walk the same graph.
"""
from __future__ import annotations

import math

import numpy as np
import torch

L2 = 0
ANGULAR = 1
IP = 2


def _dev_dtype(device):
    device = torch.device(device)
    return device, (torch.float64 if device.type == "cpu" else torch.float32)


def _sqnorm(x):
    return (x * x).sum(-1)


def knn(base: torch.Tensor, queries: torch.Tensor, k: int, exclude_self: bool = False,
        row_chunk: int = 2048, col_chunk: int = 1 << 20, log=None):
    """Exact k nearest base rows of every query row by squared l2, ordered by
    (distance, id).  With exclude_self, query i is base row i and is skipped."""
    nq, n = queries.shape[0], base.shape[0]
    k_eff = min(k, n - (1 if exclude_self else 0))
    out_i = torch.full((nq, k), -1, dtype=torch.int64, device=base.device)
    out_d = torch.full((nq, k), math.inf, dtype=base.dtype, device=base.device)
    if k_eff <= 0 or nq == 0:
        return out_i, out_d
    bn = _sqnorm(base)
    for r0 in range(0, nq, row_chunk):
        if log and r0 and (r0 // row_chunk) % 64 == 0:
            log(f"knn rows {r0}/{nq}")
        q = queries[r0:r0 + row_chunk]
        qn = _sqnorm(q)
        best_d = None
        best_i = None
        for c0 in range(0, n, col_chunk):
            b = base[c0:c0 + col_chunk]
            dd = qn[:, None] + bn[None, c0:c0 + b.shape[0]] - 2.0 * (q @ b.T.contiguous())
            dd.clamp_(min=0)
            if exclude_self:
                rows = torch.arange(q.shape[0], device=base.device)
                cols = rows + r0 - c0
                ok = (cols >= 0) & (cols < b.shape[0])
                dd[rows[ok], cols[ok]] = math.inf
            kk = min(k_eff + 8, b.shape[0])  # slack so ties at the cut sort by id
            vd, vi = torch.topk(dd, kk, dim=1, largest=False, sorted=False)
            vi = vi + c0
            if best_d is None:
                best_d, best_i = vd, vi
            else:
                best_d = torch.cat([best_d, vd], 1)
                best_i = torch.cat([best_i, vi], 1)
                best_d, sel = torch.topk(best_d, min(k_eff + 8, best_d.shape[1]), dim=1,
                                         largest=False, sorted=False)
                best_i = torch.gather(best_i, 1, sel)
        # order by (distance, id)
        o = torch.argsort(best_i, dim=1, stable=True)
        best_i = torch.gather(best_i, 1, o)
        best_d = torch.gather(best_d, 1, o)
        o = torch.argsort(best_d, dim=1, stable=True)
        best_i = torch.gather(best_i, 1, o)[:, :k_eff]
        best_d = torch.gather(best_d, 1, o)[:, :k_eff]
        out_i[r0:r0 + q.shape[0], :k_eff] = best_i
        out_d[r0:r0 + q.shape[0], :k_eff] = best_d
    return out_i, out_d


def knn_ivf(x: torch.Tensor, k: int, nlist: int = 1024, nprobe: int = 16, iters: int = 8,
            seed: int = 0, log=None):
    """Approximate k nearest neighbours of every row of x among the rows of x
    (self excluded), for bases too large for the exact product: k-means
    centroids from a sample; every row scans the primary lists of its
    `nprobe` nearest centroids, one probe rank at a time, merging into a
    running top-k ordered by (distance, id).  Returns (ids, dists) like knn."""
    n, d = x.shape
    g = torch.Generator(device="cpu").manual_seed(seed)
    sample = x[torch.randperm(n, generator=g)[:min(n, 64 * nlist)].to(x.device)]
    cent = sample[:nlist].clone()
    # the centroid sums on the host: index_add_ on the GPU adds with atomics,
    # in an order that changes from run to run, and so would the centroids,
    # the lists and the graph; on the host the order is fixed
    sample_h = sample.cpu()
    for _ in range(iters):
        a, _ = knn(cent, sample, 1)
        a = a[:, 0].cpu()
        nc = cent.shape[0]  # nlist, or fewer for a sample smaller than that
        sums = torch.zeros((nc, d), dtype=sample_h.dtype).index_add_(0, a, sample_h)
        cnt = torch.bincount(a, minlength=nc).to(sample_h.dtype)
        ok = cnt > 0
        cent_h = cent.cpu()
        cent_h[ok] = sums[ok] / cnt[ok, None]
        cent = cent_h.to(x.device)
    probes, _ = knn(cent, x, nprobe, row_chunk=16384)        # n x nprobe, nearest first
    primary = probes[:, 0]
    order = torch.argsort(primary, stable=True)
    counts = torch.bincount(primary, minlength=nlist)
    starts = (torch.cumsum(counts, 0) - counts).tolist()
    counts = counts.tolist()
    kk = k + 1
    best_i = torch.full((n, kk), -1, dtype=torch.int64, device=x.device)
    best_d = torch.full((n, kk), math.inf, dtype=x.dtype, device=x.device)
    for j in range(nprobe):
        if log:
            log(f"ivf probe {j + 1}/{nprobe}")
        pj = probes[:, j]
        qord = torch.argsort(pj, stable=True)
        qcnt = torch.bincount(pj, minlength=nlist)
        qst = (torch.cumsum(qcnt, 0) - qcnt).tolist()
        qcnt = qcnt.tolist()
        cur_i = torch.full((n, kk), -1, dtype=torch.int64, device=x.device)
        cur_d = torch.full((n, kk), math.inf, dtype=x.dtype, device=x.device)
        for c in range(nlist):
            if qcnt[c] == 0 or counts[c] == 0:
                continue
            members = order[starts[c]:starts[c] + counts[c]]
            b = x[members]
            bn = _sqnorm(b)
            qs = qord[qst[c]:qst[c] + qcnt[c]]
            for q0 in range(0, qs.shape[0], 8192):
                qi = qs[q0:q0 + 8192]
                q = x[qi]
                dd = _sqnorm(q)[:, None] + bn[None, :] - 2.0 * (q @ b.T.contiguous())
                dd.clamp_(min=0)
                dd[members[None, :] == qi[:, None]] = math.inf
                t = min(kk, members.shape[0])
                vd, vi = torch.topk(dd, t, dim=1, largest=False, sorted=False)
                cur_i[qi, :t] = members[vi]
                cur_d[qi, :t] = vd
        # merge (the lists of different probes are disjoint)
        ci = torch.cat([best_i, cur_i], 1)
        cd = torch.cat([best_d, cur_d], 1)
        cd = torch.where(ci >= 0, cd, torch.full_like(cd, math.inf))
        big = torch.iinfo(torch.int64).max
        key = torch.where(ci >= 0, ci, torch.full_like(ci, big))
        o = torch.argsort(key, dim=1, stable=True)
        ci, cd = torch.gather(ci, 1, o), torch.gather(cd, 1, o)
        o = torch.argsort(cd, dim=1, stable=True)
        best_i, best_d = torch.gather(ci, 1, o)[:, :kk], torch.gather(cd, 1, o)[:, :kk]
        del ci, cd, cur_i, cur_d, key, o
    best_i, best_d = best_i[:, :k], best_d[:, :k]
    best_i = torch.where(torch.isfinite(best_d), best_i, torch.full_like(best_i, -1))
    return best_i, best_d


def _prune(x: torch.Tensor, cand_i: torch.Tensor, cand_d: torch.Tensor, R: int,
           chunk: int = 16384):
    """Relative-neighbourhood pruning of ordered candidate lists (see module
    docstring, rule 2).  Returns (ids, dists), n x R, padded with (-1, inf)."""
    n, C = cand_i.shape
    out_i = torch.full((n, R), -1, dtype=torch.int64, device=x.device)
    out_d = torch.full((n, R), math.inf, dtype=x.dtype, device=x.device)
    for s in range(0, n, chunk):
        ci = cand_i[s:s + chunk]
        cd = cand_d[s:s + chunk]
        B = ci.shape[0]
        valid = ci >= 0
        xv = x[ci.clamp(min=0)]                      # B x C x d
        nv = _sqnorm(xv)
        pw = nv[:, :, None] + nv[:, None, :] - 2.0 * torch.bmm(xv, xv.transpose(1, 2).contiguous())
        pw.clamp_(min=0)
        kept = torch.zeros(B, C, dtype=torch.bool, device=x.device)
        cnt = torch.zeros(B, dtype=torch.int64, device=x.device)
        for j in range(C):
            ok = valid[:, j] & (cnt < R)
            if j:
                blocked = (kept[:, :j] & (pw[:, j, :j] <= cd[:, j:j + 1])).any(1)
                ok &= ~blocked
            kept[:, j] = ok
            cnt += ok.to(torch.int64)
        pos = torch.cumsum(kept.to(torch.int64), 1) - 1
        rows = torch.arange(B, device=x.device)[:, None].expand(B, C)
        m = kept & (pos < R)
        oi = out_i[s:s + B]
        od = out_d[s:s + B]
        oi[rows[m], pos[m]] = ci[m]
        od[rows[m], pos[m]] = cd[m]
    return out_i, out_d


def _reverse_merge(x, fwd_i, fwd_d, cand, chunk=16384):
    """Offer every kept edge v->u to u and rebuild u's ordered candidate list
    (kept list + offers, duplicates dropped, closest `cand`)."""
    n, R = fwd_i.shape
    src = torch.arange(n, device=x.device).repeat_interleave(R)
    dst = fwd_i.reshape(-1)
    dd = fwd_d.reshape(-1)
    ok = dst >= 0
    src, dst, dd = src[ok], dst[ok], dd[ok]
    # order offers by (dst, dist, src)
    o = torch.argsort(dd, stable=True)
    src, dst, dd = src[o], dst[o], dd[o]
    o = torch.argsort(dst, stable=True)
    src, dst, dd = src[o], dst[o], dd[o]
    counts = torch.bincount(dst, minlength=n)
    starts = torch.cumsum(counts, 0) - counts
    pos = torch.arange(dst.shape[0], device=x.device) - starts[dst]
    keep = pos < cand
    rev_i = torch.full((n, cand), -1, dtype=torch.int64, device=x.device)
    rev_d = torch.full((n, cand), math.inf, dtype=x.dtype, device=x.device)
    rev_i[dst[keep], pos[keep]] = src[keep]
    rev_d[dst[keep], pos[keep]] = dd[keep]
    ci = torch.cat([fwd_i, rev_i], 1)
    cd = torch.cat([fwd_d, rev_d], 1)
    # drop duplicates: sort by id, invalidate repeats
    big = torch.iinfo(torch.int64).max
    key = torch.where(ci >= 0, ci, torch.full_like(ci, big))
    o = torch.argsort(key, dim=1, stable=True)
    ci = torch.gather(ci, 1, o)
    cd = torch.gather(cd, 1, o)
    dup = torch.zeros_like(ci, dtype=torch.bool)
    dup[:, 1:] = (ci[:, 1:] == ci[:, :-1]) & (ci[:, 1:] >= 0)
    ci = torch.where(dup, torch.full_like(ci, -1), ci)
    cd = torch.where(dup | (ci < 0), torch.full_like(cd, math.inf), cd)
    # order by (dist, id); invalid entries (inf) go last
    key = torch.where(ci >= 0, ci, torch.full_like(ci, big))
    o = torch.argsort(key, dim=1, stable=True)
    ci, cd = torch.gather(ci, 1, o), torch.gather(cd, 1, o)
    o = torch.argsort(cd, dim=1, stable=True)
    ci, cd = torch.gather(ci, 1, o)[:, :cand], torch.gather(cd, 1, o)[:, :cand]
    return ci, cd


def reachable(g: torch.Tensor, entry: int) -> torch.Tensor:
    """Boolean mask of the nodes reachable from `entry` along graph rows."""
    n = g.shape[0]
    reached = torch.zeros(n, dtype=torch.bool, device=g.device)
    reached[entry] = True
    frontier = torch.tensor([entry], device=g.device)
    while frontier.numel():
        nb = g[frontier].reshape(-1)
        nb = nb[nb >= 0]
        new = torch.zeros(n, dtype=torch.bool, device=g.device)
        new[nb] = True
        new &= ~reached
        reached |= new
        frontier = torch.nonzero(new).reshape(-1)
    return reached


def _connect(x, g, cand_i, entry, max_rounds=100000):
    """Rule 4 of the module docstring.  Mutates and returns g (int64)."""
    n, R = g.shape
    for _ in range(max_rounds):
        reached = reachable(g, entry)
        un = torch.nonzero(~reached).reshape(-1)
        if un.numel() == 0:
            return g
        free = R - (g >= 0).sum(1)
        ci = cand_i[un]
        okc = (ci >= 0) & reached[ci.clamp(min=0)] & (free[ci.clamp(min=0)] > 0)
        has = okc.any(1)
        if has.any():
            first = torch.argmax(okc.to(torch.int8), dim=1)
            u = un[has]
            r = ci[has, first[has]]
        else:
            u = un[:1]
            w = (reached & (free > 0)).nonzero().reshape(-1)
            if w.numel() == 0:
                raise RuntimeError("graph has no free slot to connect unreached nodes")
            dd = _sqnorm(x[w] - x[u])
            r = w[torch.argmin(dd)].reshape(1)
        # at most free[r] new links into each r per round, lowest u first
        o = torch.argsort(r, stable=True)
        u, r = u[o], r[o]
        cnt = torch.bincount(r, minlength=n)
        start = torch.cumsum(cnt, 0) - cnt
        rank = torch.arange(r.numel(), device=g.device) - start[r]
        ok = rank < free[r]
        u, r, rank = u[ok], r[ok], rank[ok]
        slot = (R - free[r]) + rank
        g[r, slot] = u
    raise RuntimeError("graph connectivity did not converge")


def medoid(x: torch.Tensor, exact_limit: int = 20000) -> int:
    """Entry node: argmin of summed Euclidean distance (n <= exact_limit),
    else the node nearest to the mean."""
    n = x.shape[0]
    if n <= exact_limit:
        best, best_v = 0, math.inf
        xn = _sqnorm(x)
        for s in range(0, n, 2048):
            q = x[s:s + 2048]
            dd = (_sqnorm(q)[:, None] + xn[None, :] - 2.0 * q @ x.T.contiguous()).clamp(min=0).sqrt()
            tot = dd.sum(1)
            v, i = torch.min(tot, 0)
            if float(v) < best_v:
                best_v, best = float(v), s + int(i)
        return best
    mu = x.mean(0, keepdim=True)
    return int(torch.argmin(_sqnorm(x - mu)))


EXACT_KNN_LIMIT = 2_000_000


def _random_edges(g: torch.Tensor, count: int, seed: int):
    """Fill up to `count` free slots of every row with distinct random ids
    (not the row itself, not already in the row): long-range shortcuts that
    keep a pruned kNN graph navigable when its clusters are tight."""
    n, R = g.shape
    gen = torch.Generator(device="cpu").manual_seed(seed)
    for _ in range(count):
        free = (g < 0).any(1)
        pos = torch.argmax((g < 0).to(torch.int8), dim=1)  # first free slot
        r = torch.randint(0, n, (n,), generator=gen).to(g.device)
        rows = torch.arange(n, device=g.device)
        ok = free & (r != rows) & ~(g == r[:, None]).any(1)
        g[rows[ok], pos[ok]] = r[ok]
    return g


def build_graph(base: np.ndarray, R: int, cand: int, device="cpu", reverse: bool = True,
                log=None, rand_edges: int = 0, seed: int = 0):
    """Pruned exact-kNN graph (module docstring).  Returns (graph int32 n x R
    padded with -1, entry id).  `log` receives progress lines.  Above
    EXACT_KNN_LIMIT rows the candidates come from knn_ivf (approximate).
    rand_edges > 0 adds that many random long-range edges per node (in free
    slots) before the connectivity repair."""
    device, dt = _dev_dtype(device)
    x = torch.as_tensor(base).to(device=device, dtype=dt)
    if x.shape[0] > EXACT_KNN_LIMIT:
        ci, cd = knn_ivf(x, cand, log=log)
        if log:
            log("ivf knn done")
    else:
        ci, cd = knn(x, x, cand, exclude_self=True, log=log)
    if log:
        log("knn done, pruning")
    gi, gd = _prune(x, ci, cd, R)
    if reverse:
        if log:
            log("reverse edges")
        ci, cd = _reverse_merge(x, gi, gd, cand)
        small = (ci >= 0).sum(1) <= R
        pi, pd = _prune(x, ci, cd, R)
        gi = torch.where(small[:, None], ci[:, :R], pi)
        gd = torch.where(small[:, None], cd[:, :R], pd)
    entry = medoid(x)
    if rand_edges > 0:
        gi = _random_edges(gi, rand_edges, seed)
    kc, _ = knn(x, x, cand, exclude_self=True) if not reverse else (ci, cd)
    if log:
        log("connectivity")
    gi = _connect(x, gi, kc, entry)
    return gi.to(torch.int32).cpu().numpy(), entry


def ground_truth(base: np.ndarray, queries: np.ndarray, k: int, metric: int, device="cpu"):
    """Exact top-k ids and distances (squared l2, 1 - x.q/|q| for angular,
    -x.q for the inner product), ordered by (distance, id), in float64 on
    any device (the recall reference: no single-precision cancellation in
    |q|^2 + |x|^2 - 2 q.x)."""
    device = torch.device(device)
    dt = torch.float64
    x = torch.as_tensor(base).to(device=device, dtype=dt)
    q = torch.as_tensor(queries).to(device=device, dtype=dt)
    if metric == L2:
        # 256 query rows x 1M columns of float64 per block (2 GB)
        ids, dd = knn(x, q, k, row_chunk=256)
        return ids.cpu().numpy(), dd.cpu().numpy()
    qn = q if metric == IP else q / torch.linalg.norm(q, dim=1, keepdim=True)
    ids_all = []
    d_all = []
    xt = x.T.contiguous()
    rows = max(1, (1 << 31) // (8 * x.shape[0]))  # about 2 GB of float64 per block
    for s in range(0, q.shape[0], rows):
        sim = qn[s:s + rows] @ xt
        kk = min(k + 8, x.shape[0])
        v, i = torch.topk(sim, kk, dim=1)
        dd = -v if metric == IP else 1.0 - v
        o = torch.argsort(i, dim=1, stable=True)
        i, dd = torch.gather(i, 1, o), torch.gather(dd, 1, o)
        o = torch.argsort(dd, dim=1, stable=True)
        ids_all.append(torch.gather(i, 1, o)[:, :k])
        d_all.append(torch.gather(dd, 1, o)[:, :k])
    return torch.cat(ids_all).cpu().numpy(), torch.cat(d_all).cpu().numpy()


def exact_distances(base: np.ndarray, queries: np.ndarray, ids: np.ndarray, metric: int):
    """float64 distances of (query, id) pairs; -1 ids give +inf."""
    ids = np.asarray(ids)
    safe = np.where(ids >= 0, ids, 0)
    xb = base[safe].astype(np.float64)
    q = queries.astype(np.float64)[:, None, :]
    if metric == L2:
        dd = ((xb - q) ** 2).sum(-1)
    elif metric == IP:
        dd = -(xb * q).sum(-1)
    else:
        dd = 1.0 - (xb * q).sum(-1) / np.linalg.norm(q, axis=-1)
    return np.where(ids >= 0, dd, np.inf)


def recall_at_k(base, queries, ids, gt_dist, k: int, metric: int, rel_tol: float = 1e-6):
    """Tie-aware recall@k: a returned id counts when its exact distance is no
    larger than the exact k-th distance (so equal-distance neighbours, common
    with integer data, are interchangeable).  Returns the per-query recall."""
    ids = np.asarray(ids)[:, :k]
    dd = exact_distances(base, queries, ids, metric)
    kth = np.asarray(gt_dist, dtype=np.float64)[:, k - 1:k]
    hit = dd <= kth + rel_tol * np.abs(kth) + 1e-12
    # a repeated id may not count twice
    for i in range(ids.shape[0]):
        row = ids[i]
        _, first = np.unique(row, return_index=True)
        mask = np.zeros(k, dtype=bool)
        mask[first] = True
        hit[i] &= mask & (row >= 0)
    return hit.sum(1) / float(k)


def build_upper_layers(base: np.ndarray, R_up: int = 16, M: int = 16, seed: int = 0,
                       device="cpu", log=None):
    """HNSW-style upper layers for the entry descent.  Node i reaches level
    floor(-ln(U_i) / ln M) with U_i uniform in (0, 1] (seeded); layer l >= 1
    holds the nodes of level >= l, linked by a pruned k-NN graph of degree
    R_up built like the base graph (a complete graph when the layer has at
    most R_up + 1 nodes).  Rows of layer 1 come first.  Returns dict(node
    (rows,) base ids, adj (rows, R_up) rows of the neighbours in the same
    layer or -1, down (rows,) row of the same node one layer below or -1 in
    layer 1, top (the starting row: the top layer's medoid), layer_start
    (levels + 1,))."""
    n = base.shape[0]
    rng = np.random.default_rng([seed, 11])
    u = 1.0 - rng.random(n)
    level = np.floor(-np.log(u) / math.log(M)).astype(np.int64)
    top_level = max(1, int(level.max()))
    if level.max() < 1:
        level[int(np.argmin(u))] = 1
    layers = [np.nonzero(level >= lv)[0] for lv in range(1, top_level + 1)]
    starts = np.concatenate([[0], np.cumsum([len(ids) for ids in layers])]).astype(np.int64)
    rows = int(starts[-1])
    node = np.concatenate(layers).astype(np.int32)
    adj = np.full((rows, R_up), -1, np.int32)
    down = np.full(rows, -1, np.int32)
    top = 0
    for lv, ids in enumerate(layers, 1):
        off, k = int(starts[lv - 1]), len(ids)
        if k <= R_up + 1:
            for i in range(k):
                others = [off + j for j in range(k) if j != i]
                adj[off + i, :len(others)] = others
            ent = 0
        else:
            g, ent = build_graph(base[ids], R_up, 2 * R_up, device=device)
            adj[off:off + k] = np.where(g >= 0, g + off, -1)
        if lv >= 2:
            prev = layers[lv - 2]
            down[off:off + k] = starts[lv - 2] + np.searchsorted(prev, ids)
        if lv == top_level:
            top = off + int(ent)
        if log:
            log(f"upper layer {lv}: {k} nodes")
    return dict(node=node, adj=adj, down=down, top=top, layer_start=starts)
