"""Launch-plan autotuner for peos_search.

The search kernel keeps each query's visited set in an LDS hash.  A larger hash
avoids moving busy queries' visited sets to HBM but costs LDS, hence resident
waves per CU; the best capacity depends on the graph, ef and the stopping rule.
`tune` times peos_search on the caller's batch with 1, 2 or 4 waves per query
(more waves gather each query's rows together; they pay when the batch is too
small to fill the chip with one wave per query) and then with a few
capacities, and sets the fastest with peos_set_search_tuning on that index
(the plan belongs to the index and touches no other).  Results never depend on the choice
(only speed does).  Choices are cached per device and problem shape in a JSON
file (PEOS_TUNE_CACHE, default ~/.cache/peos_tune.json).
"""
from __future__ import annotations

import json
import os

import torch

from . import peos_search_ws_bytes, peos_set_search_tuning, search

CACHE = os.environ.get("PEOS_TUNE_CACHE", os.path.expanduser("~/.cache/peos_tune.json"))
HASH_CAPS = (0, 1024, 1536, 1792, 2048, 3072, 4096, 8192)  # 0 = the library's default plan
WAVES = (0, 1, 2, 4)  # waves per query; 0 = the library's automatic choice
KEEP_DEFAULT = 0.03  # another plan must be this much faster to replace the default


def _key(index, nq, k, ef, pool, mode):
    lay = index.layout()
    dev = torch.cuda.get_device_name(0)
    return f"{dev}|n={lay.n}|d={lay.d}|R={lay.R}|L={lay.L}|m={lay.m}|nq={nq}|k={k}|ef={ef}|pool={pool}|mode={mode}"


def _load():
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(cache):
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        tmp = CACHE + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, CACHE)
    except OSError:
        pass


def _time(index, queries, k, ef, pool, eps, mode, ws, reps):
    """Average ms of one search call, or None when the plan does not fit."""
    try:
        search(index, queries, k, ef, eps=eps, mode=mode, pool=pool, ws=ws)  # warm-up
    except RuntimeError:
        return None  # LDS plan too large for this capacity
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        search(index, queries, k, ef, eps=eps, mode=mode, pool=pool, ws=ws)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _pick(times):
    """Fastest key; the default (first key) stays unless another is at least
    KEEP_DEFAULT faster, so that the choice is stable from run to run."""
    keys = list(times)
    best = min(keys, key=times.get)
    if times[best] > (1.0 - KEEP_DEFAULT) * times[keys[0]]:
        best = keys[0]
    return best


def tune(index, queries, k, ef, pool=0, eps=0.1, mode=0, caps=HASH_CAPS, waves=WAVES, reps=3,
         use_cache=True, log=None):
    """Pick and set the launch plan of this operating point on this index:
    first the waves per query (the library's automatic choice, or 1, 2, 4),
    then the visited-hash capacity at that choice.  Returns (hash_cap,
    {cap: ms}); the chosen waves per query are in index.tuned_waves."""
    nq = queries.shape[0]
    key = _key(index, nq, k, ef, pool, mode)
    cache = _load() if use_cache else {}
    if key in cache:
        cap = int(cache[key]["hash_cap"])
        nw = int(cache[key].get("waves", 0))
        peos_set_search_tuning(index, cap, waves=nw)
        index.tuned_waves = nw
        return cap, cache[key].get("ms", {})
    efmax = max(ef, k)
    ws = torch.empty(peos_search_ws_bytes(index, nq, efmax, pool), dtype=torch.uint8,
                     device=queries.device)
    wtimes = {}
    for nw in waves:
        peos_set_search_tuning(index, 0, waves=nw)
        t = _time(index, queries, k, ef, pool, eps, mode, ws, reps)
        if t is not None:
            wtimes[nw] = t
            if log:
                log(f"autotune ef={ef} pool={pool} mode={mode} waves={nw}: {t:.3f} ms")
    nw = _pick(wtimes) if wtimes else 0
    times = {}
    for cap in caps:
        peos_set_search_tuning(index, cap, waves=nw)
        t = _time(index, queries, k, ef, pool, eps, mode, ws, reps)
        if t is None:
            continue
        times[cap] = t
        if log:
            log(f"autotune ef={ef} pool={pool} mode={mode} waves={nw} hash_cap={cap}: {t:.3f} ms")
    best = _pick(times)
    peos_set_search_tuning(index, best, waves=nw)
    index.tuned_waves = nw
    cache[key] = {"hash_cap": best, "waves": nw,
                  "ms": {str(c): round(t, 4) for c, t in times.items()},
                  "waves_ms": {str(c): round(t, 4) for c, t in wtimes.items()}}
    if use_cache:
        _store(cache)
    return best, times


def ef_classes(k, ef):
    """Host copy of the device's ef-class split: class c holds effective list
    sizes max(min(ef, max ef), k) in (32 << (c-1), 32 << c]."""
    import numpy as np
    k = np.asarray(k)
    ef = np.asarray(ef)
    eff = np.maximum(np.minimum(ef, ef.max()), k)
    efmax = int(max(ef.max(), k.max()))
    nclass = 1
    while nclass < 8 and efmax > (32 << (nclass - 1)):
        nclass += 1
    cls = np.zeros(len(eff), np.int64)
    for c in range(nclass - 1):
        cls += eff > (32 << c)
    return cls


def tune_classes(index, queries, k, ef, pool=1, eps=0.1, mode=0, caps=HASH_CAPS, waves=WAVES,
                 reps=2, log=None):
    """Pick the launch plan of every ef class of a batch with per-query k and
    ef (host arrays), timing each class on its own queries: first the waves
    per query (the library's automatic choice, or 1, 2, 4: a class whose
    lists and visited hash take much LDS runs few workgroups per CU, and more
    waves per workgroup keep more rows in flight), then the visited-hash
    capacity at that choice; set with peos_set_class_tuning.  Returns
    {class: hash_cap}; the chosen waves are in index.tuned_class_waves."""
    import numpy as np
    from . import peos_set_class_tuning
    cls = ef_classes(k, ef)
    chosen = {}
    index.tuned_class_waves = {}
    dev = queries.device
    for c in np.unique(cls).tolist():
        sel = np.nonzero(cls == c)[0]
        qs = queries[torch.from_numpy(sel).to(dev)]
        kt = torch.from_numpy(np.ascontiguousarray(k[sel], dtype=np.int32)).to(dev)
        et = torch.from_numpy(np.ascontiguousarray(ef[sel], dtype=np.int32)).to(dev)
        efmax = int(max(ef[sel].max(), k[sel].max()))
        ws = torch.empty(peos_search_ws_bytes(index, len(sel), efmax, pool), dtype=torch.uint8,
                         device=dev)

        def timed(cap, nw):
            peos_set_class_tuning(index, c, cap, 0, nw)
            try:
                search(index, qs, kt, et, eps=eps, mode=mode, pool=pool, ws=ws)
            except RuntimeError:
                return None
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                search(index, qs, kt, et, eps=eps, mode=mode, pool=pool, ws=ws)
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / reps

        wtimes = {}
        for nw in waves:
            t = timed(0, nw)
            if t is not None:
                wtimes[nw] = t
        nw = _pick(wtimes) if wtimes else 0
        times = {}
        for cap in caps:
            t = timed(cap, nw)
            if t is not None:
                times[cap] = t
        best = _pick(times)
        peos_set_class_tuning(index, c, best, 0, nw)
        chosen[c] = best
        index.tuned_class_waves[c] = nw
        if log:
            log(f"autotune class {c} ({len(sel)} queries, ef <= {efmax}): waves "
                + " ".join(f"{x}:{t:.3f}ms" for x, t in wtimes.items()) + f" -> {nw}; hash "
                + " ".join(f"{cp}:{t:.3f}ms" for cp, t in times.items()) + f" -> {best}")
    return chosen
