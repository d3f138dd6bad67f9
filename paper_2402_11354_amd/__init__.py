"""Python binding of libpeos (include/peos.h): argument marshalling only.

Every function here has the name of the C entry point it calls and takes
torch CUDA tensors (device memory and streams come from PyTorch); all the work
runs in the HIP kernels of libpeos.so.  There is no fallback: if the library
is missing or the device is not gfx950 the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpeos.so")

PEOS_OK = 0
PEOS_EINVAL = -1
PEOS_ENOSPACE = -2
PEOS_EHIP = -3
PEOS_EGRAPH = -4
PEOS_EDEVICE = -5
PEOS_EBUSY = -6
PEOS_METRIC_L2 = 0
PEOS_METRIC_ANGULAR = 1
PEOS_METRIC_IP = 2
PEOS_MODE_PEOS = 0
PEOS_MODE_EXHAUSTIVE = 1
PEOS_MODE_SIMHASH = 2
PEOS_FLAG_BF16_BASE = 1
PEOS_FLAG_FP16 = 2
PEOS_FLAG_SIMHASH = 4
PEOS_FLAG_COMPACT = 8
PEOS_STAT_STATUS = 11
PEOS_STAT_DESCENT = 12
PEOS_STAT_TEST_EXPANSIONS = 13
PEOS_NSTATS = 14
STATS = ("expansions", "edges", "visited_skips", "tests", "test_ge1", "test_le0", "test_h",
         "test_zero", "passes", "ndist", "inserted", "status")
PEOS_STATUS_ZERO_QUERY = 1
PEOS_STATUS_POOL_FULL = 2
PEOS_STATUS_VISITED_SPILL = 4


class PeosError(RuntimeError):
    def __init__(self, fn, code, msg):
        super().__init__(f"{fn} failed ({code}): {msg}")
        self.code = code


class peos_layout(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("d", ctypes.c_int32), ("R", ctypes.c_int32),
                ("L", ctypes.c_int32), ("m", ctypes.c_int32), ("metric", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("entry", ctypes.c_int32),
                ("node_stride", ctypes.c_int64), ("codes_offset", ctypes.c_int64),
                ("scalars_offset", ctypes.c_int64), ("code_bytes", ctypes.c_int64),
                ("scalar_bytes", ctypes.c_int64), ("bf16_offset", ctypes.c_int64),
                ("simhash_offset", ctypes.c_int64)]


class peos_build_options(ctypes.Structure):
    _fields_ = [("perm", ctypes.c_void_p), ("simhash_dirs", ctypes.c_void_p)]


class peos_upper_layers(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("R", ctypes.c_int32), ("rows", ctypes.c_int64),
                ("top", ctypes.c_int64), ("layer_start", ctypes.c_void_p),
                ("node", ctypes.c_void_p), ("adj", ctypes.c_void_p), ("down", ctypes.c_void_p)]


class peos_serve_config(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_int32), ("max_k", ctypes.c_int32),
                ("max_ef", ctypes.c_int32), ("max_inflight", ctypes.c_int32),
                ("max_pending", ctypes.c_int32), ("pool", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("launch_waves", ctypes.c_int32),
                ("eps", ctypes.c_float), ("reserved", ctypes.c_float),
                ("hbm_budget", ctypes.c_size_t), ("lds_budget", ctypes.c_size_t)]


_lib = None


def lib():
    """The loaded libpeos.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "python -m paper_2402_11354_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        P, i64, i32, sz, f32 = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t,
                                ctypes.c_float)
        Psz = ctypes.POINTER(ctypes.c_size_t)
        L.peos_index_bytes.argtypes = [i64, i32, i32, i32, i32, i32, Psz, Psz]
        L.peos_build_tables.argtypes = [P, i64, i32, P, i32, i32, i32, i32, P, P, i32, i32, P, sz,
                                        P, sz, P, ctypes.POINTER(P)]
        L.peos_index_layout.argtypes = [P, ctypes.POINTER(peos_layout)]
        L.peos_build_tables_ex.argtypes = [P, i64, i32, P, i32, i32, i32, i32, P, P, i32, i32,
                                           ctypes.POINTER(peos_build_options), P, sz, P, sz, P,
                                           ctypes.POINTER(P)]
        L.peos_dimension_permutation_ws_bytes.argtypes = [i32, Psz]
        L.peos_dimension_permutation.argtypes = [P, i64, i32, P, i32, i32, P, P, sz, P]
        L.peos_set_upper_layers.argtypes = [P, ctypes.POINTER(peos_upper_layers)]
        L.peos_probe_gather.argtypes = [P, i64, i32, i32, P, P]
        L.peos_free.argtypes = [P]
        L.peos_free.restype = None
        L.peos_query_tables.argtypes = [P, P, i64, P, P, P]
        L.peos_search_ws_bytes.argtypes = [P, i64, i32, i32, Psz]
        L.peos_search_tables.argtypes = [P, P, P, P, i64, P, P, i32, i32, i32, i32, f32, i32, P, P,
                                         P, P, sz, P]
        L.peos_search.argtypes = [P, P, i64, P, P, i32, i32, i32, i32, f32, i32, P, P, P, P, sz, P]
        L.peos_search_static.argtypes = [P, P, i64, P, P, i32, i32, i32, i32, f32, i32, P, P, P,
                                         P]
        L.peos_set_search_tuning.argtypes = [P, i32, i32, i32, i32]
        L.peos_set_long_rows.argtypes = [P, i32]
        L.peos_set_class_tuning.argtypes = [P, i32, i32, i32, i32]
        L.peos_serve_open.argtypes = [P, ctypes.POINTER(peos_serve_config), ctypes.POINTER(P)]
        L.peos_serve_submit.argtypes = [P, P, i32, i32, i32, P, P, ctypes.POINTER(ctypes.c_uint64)]
        L.peos_serve_poll.argtypes = [P, i32, P, i32, ctypes.POINTER(i32)]
        L.peos_serve_counters.argtypes = [P, P]
        L.peos_serve_close.argtypes = [P]
        L.peos_serve_close.restype = None
        L.peos_graph_create.argtypes = [P, P, i64, P, P, i32, i32, i32, i32, f32, i32, P, P, P, P,
                                        sz, ctypes.POINTER(P)]
        L.peos_graph_launch.argtypes = [P, P]
        L.peos_graph_destroy.argtypes = [P]
        L.peos_graph_destroy.restype = None
        L.peos_strerror.argtypes = [i32]
        L.peos_strerror.restype = ctypes.c_char_p
        L.peos_last_error.restype = ctypes.c_char_p
        for name in ("peos_index_bytes", "peos_build_tables", "peos_index_layout",
                     "peos_build_tables_ex", "peos_dimension_permutation_ws_bytes",
                     "peos_dimension_permutation",
                     "peos_query_tables", "peos_search_ws_bytes", "peos_search_tables",
                     "peos_search", "peos_search_static", "peos_set_search_tuning",
                     "peos_set_long_rows",
                     "peos_set_class_tuning",
                     "peos_graph_create", "peos_graph_launch", "peos_serve_open",
                     "peos_serve_submit", "peos_serve_poll", "peos_serve_counters",
                     "peos_set_upper_layers", "peos_probe_gather"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(fn, rc):
    if rc != PEOS_OK:
        raise PeosError(fn, rc, lib().peos_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def peos_index_bytes(n, d, R, L, m, flags=0):
    """(index_bytes, build_ws_bytes)."""
    ib, wb = ctypes.c_size_t(), ctypes.c_size_t()
    _check("peos_index_bytes", lib().peos_index_bytes(n, d, R, L, m, flags, ctypes.byref(ib),
                                                      ctypes.byref(wb)))
    return ib.value, wb.value


class PeosIndex:
    """A built index: the C handle plus the device tensors it points into
    (kept alive here)."""

    def __init__(self, handle, keep):
        self.handle = handle
        self._keep = keep
        self.tuned_waves = 0  # waves per query the autotuner chose (0 = automatic)
        self.tuned_class_waves = {}  # the same per ef class (autotune.tune_classes)

    def layout(self):
        return peos_index_layout(self)

    def close(self):
        if self.handle:
            lib().peos_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def peos_build_tables(base, graph, entry, L, m, dirs_a, dirs_b, metric, flags=0, stream=None,
                      perm=None, simhash_dirs=None):
    """Build the edge records.  base (n, d) float32, graph (n, R) int32,
    dirs_a (L, m, d/L) float32, dirs_b (m, d) float32, all on the device.
    perm: optional int32 device tensor (d), the test's dimension permutation;
    simhash_dirs: (64, d) float32 device tensor, with PEOS_FLAG_SIMHASH
    (peos_build_tables_ex)."""
    n, d = base.shape
    R = graph.shape[1]
    ib, wb = peos_index_bytes(n, d, R, L, m, flags)
    mem = torch.empty(ib, dtype=torch.uint8, device=base.device)
    ws = torch.empty(wb, dtype=torch.uint8, device=base.device)
    h = ctypes.c_void_p()
    opt = peos_build_options(None if perm is None else perm.data_ptr(),
                             None if simhash_dirs is None else simhash_dirs.data_ptr())
    _check("peos_build_tables_ex",
           lib().peos_build_tables_ex(_ptr(base), n, d, _ptr(graph), R, int(entry), L, m,
                                      _ptr(dirs_a), _ptr(dirs_b), metric, flags,
                                      ctypes.byref(opt), _ptr(mem), ib, _ptr(ws), wb,
                                      _stream(stream), ctypes.byref(h)))
    return PeosIndex(h, (base, graph, dirs_a, dirs_b, perm, simhash_dirs, mem))


def peos_set_upper_layers(index, layers):
    """Upper layers for the entry descent (peos_set_upper_layers).  layers:
    dict with node (rows,), adj (rows, R), down (rows,) int32 device tensors,
    top (int) and layer_start (levels + 1 ints, host); None removes them.
    The tensors are kept alive with the index."""
    if layers is None:
        _check("peos_set_upper_layers", lib().peos_set_upper_layers(index.handle, None))
        index._upper = None
        return
    ls = np.ascontiguousarray(layers["layer_start"], dtype=np.int64)
    node, adj, down = layers["node"], layers["adj"], layers["down"]
    up = peos_upper_layers(len(ls) - 1, adj.shape[1], node.shape[0], int(layers["top"]),
                           ls.ctypes.data, node.data_ptr(), adj.data_ptr(), down.data_ptr())
    _check("peos_set_upper_layers", lib().peos_set_upper_layers(index.handle, ctypes.byref(up)))
    index._upper = (node, adj, down)


def peos_probe_gather(rows, waves, iters, sink, stream=None):
    """Calibration gather of random 512-byte rows (peos_probe_gather).
    rows: (n, 128) float32 device tensor; sink: (waves,) float32."""
    _check("peos_probe_gather", lib().peos_probe_gather(_ptr(rows), rows.shape[0], int(waves),
                                                        int(iters), _ptr(sink), _stream(stream)))


def peos_dimension_permutation(base, graph, L, stream=None):
    """The dimension permutation (host int32 numpy array of d entries)."""
    n, d = base.shape
    wb = ctypes.c_size_t()
    _check("peos_dimension_permutation_ws_bytes",
           lib().peos_dimension_permutation_ws_bytes(d, ctypes.byref(wb)))
    ws = torch.empty(wb.value, dtype=torch.uint8, device=base.device)
    perm = np.zeros(d, np.int32)
    _check("peos_dimension_permutation",
           lib().peos_dimension_permutation(_ptr(base), n, d, _ptr(graph), graph.shape[1], L,
                                            perm.ctypes.data, _ptr(ws), wb.value,
                                            _stream(stream)))
    return perm


def peos_index_layout(index):
    out = peos_layout()
    _check("peos_index_layout", lib().peos_index_layout(index.handle, ctypes.byref(out)))
    return out


def peos_query_tables(index, queries, tables, qnorms, stream=None):
    _check("peos_query_tables",
           lib().peos_query_tables(index.handle, _ptr(queries), queries.shape[0], _ptr(tables),
                                   _ptr(qnorms), _stream(stream)))


def peos_search_ws_bytes(index, nq, efmax, pool=0):
    out = ctypes.c_size_t()
    _check("peos_search_ws_bytes",
           lib().peos_search_ws_bytes(index.handle, nq, efmax, pool, ctypes.byref(out)))
    return out.value


def peos_search_tables(index, queries, tables, qnorms, k, ef, kstride, pool, eps, mode, ids,
                       dists, stats, ws, k_all=None, ef_all=None, stream=None):
    """k, ef: int or per-query int32 device tensors (then k_all / ef_all are
    their upper bounds)."""
    kt = k if torch.is_tensor(k) else None
    et = ef if torch.is_tensor(ef) else None
    ka = int(k_all if k_all is not None else (k if kt is None else int(kt.max())))
    ea = int(ef_all if ef_all is not None else (ef if et is None else int(et.max())))
    _check("peos_search_tables",
           lib().peos_search_tables(index.handle, _ptr(queries), _ptr(tables), _ptr(qnorms),
                                    queries.shape[0], _ptr(kt), _ptr(et), ka, ea, kstride, pool,
                                    float(eps), mode, _ptr(ids), _ptr(dists), _ptr(stats),
                                    _ptr(ws), ws.numel(), _stream(stream)))


def peos_search(index, queries, k, ef, kstride, pool, eps, mode, ids, dists, stats, ws,
                k_all=None, ef_all=None, stream=None):
    kt = k if torch.is_tensor(k) else None
    et = ef if torch.is_tensor(ef) else None
    ka = int(k_all if k_all is not None else (k if kt is None else int(kt.max())))
    ea = int(ef_all if ef_all is not None else (ef if et is None else int(et.max())))
    _check("peos_search",
           lib().peos_search(index.handle, _ptr(queries), queries.shape[0], _ptr(kt), _ptr(et),
                             ka, ea, kstride, pool, float(eps), mode, _ptr(ids), _ptr(dists),
                             _ptr(stats), _ptr(ws), ws.numel(), _stream(stream)))


def peos_search_static(index, queries, k, ef, kstride, pool, eps, mode, ids, dists, stats,
                       k_all=None, ef_all=None, stream=None):
    """peos_search with the library's own device scratch (no workspace)."""
    kt = k if torch.is_tensor(k) else None
    et = ef if torch.is_tensor(ef) else None
    ka = int(k_all if k_all is not None else (k if kt is None else int(kt.max())))
    ea = int(ef_all if ef_all is not None else (ef if et is None else int(et.max())))
    _check("peos_search_static",
           lib().peos_search_static(index.handle, _ptr(queries), queries.shape[0], _ptr(kt),
                                    _ptr(et), ka, ea, kstride, pool, float(eps), mode, _ptr(ids),
                                    _ptr(dists), _ptr(stats), _stream(stream)))


def peos_set_search_tuning(index, hash_cap=0, listcap=0, slots=0, waves=0):
    """Override the index's search launch plan (0 = automatic); see include/peos.h."""
    _check("peos_set_search_tuning",
           lib().peos_set_search_tuning(index.handle, hash_cap, listcap, slots, waves))


def peos_set_long_rows(index, enable=True):
    """Allow or forbid the long-vector search variant on this index."""
    _check("peos_set_long_rows", lib().peos_set_long_rows(index.handle, 1 if enable else 0))


def peos_set_class_tuning(index, cls, hash_cap=0, slots=0, waves=0):
    """Launch plan of ef class cls (lists <= 32 << cls) of a split batch on this index."""
    _check("peos_set_class_tuning",
           lib().peos_set_class_tuning(index.handle, cls, hash_cap, slots, waves))


class PeosGraph:
    """A captured peos_search (HIP graph) and the tensors baked into it."""

    def __init__(self, handle, keep):
        self.handle = handle
        self._keep = keep

    def launch(self, stream=None):
        _check("peos_graph_launch", lib().peos_graph_launch(self.handle, _stream(stream)))

    def close(self):
        if self.handle:
            lib().peos_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def peos_graph_create(index, queries, k, ef, kstride, pool, eps, mode, ids, dists, stats, ws,
                      k_all=None, ef_all=None):
    """Capture peos_search over these buffers into a graph (see include/peos.h)."""
    kt = k if torch.is_tensor(k) else None
    et = ef if torch.is_tensor(ef) else None
    ka = int(k_all if k_all is not None else (k if kt is None else int(kt.max())))
    ea = int(ef_all if ef_all is not None else (ef if et is None else int(et.max())))
    h = ctypes.c_void_p()
    _check("peos_graph_create",
           lib().peos_graph_create(index.handle, _ptr(queries), queries.shape[0], _ptr(kt),
                                   _ptr(et), ka, ea, kstride, pool, float(eps), mode, _ptr(ids),
                                   _ptr(dists), _ptr(stats), _ptr(ws), ws.numel(),
                                   ctypes.byref(h)))
    return PeosGraph(h, (index, queries, kt, et, ids, dists, stats, ws))


def search(index, queries, k, ef, eps=0.1, mode=PEOS_MODE_PEOS, pool=0, kstride=None,
           ws=None, stream=None):
    """Allocate outputs (and workspace if not given) and run peos_search.
    Returns (ids int64 (nq, kstride), dists float32, stats int32 (nq, PEOS_NSTATS))."""
    nq = queries.shape[0]
    kmax = int(k if not torch.is_tensor(k) else k.max())
    efmax = max(int(ef if not torch.is_tensor(ef) else ef.max()), kmax)
    ks = kstride or kmax
    dev = queries.device
    ids = torch.empty((nq, ks), dtype=torch.int64, device=dev)
    dists = torch.empty((nq, ks), dtype=torch.float32, device=dev)
    stats = torch.empty((nq, PEOS_NSTATS), dtype=torch.int32, device=dev)
    if ws is None:
        ws = torch.empty(peos_search_ws_bytes(index, nq, efmax, pool), dtype=torch.uint8,
                         device=dev)
    if nq:
        peos_search(index, queries, k, ef, ks, pool, eps, mode, ids, dists, stats, ws,
                    k_all=kmax, ef_all=efmax, stream=stream)
    return ids, dists, stats


SERVE_COUNTERS = ("launches", "requests", "queries", "max_batch", "inflight", "pending", "slots",
                  "lds_inflight")


class Server:
    """The serving loop (peos_serve_*): submit requests of host queries, poll
    for completed ones.  Keeps each request's host buffers alive until it
    completes."""

    def __init__(self, index, max_batch=64, max_k=100, max_ef=512, max_inflight=4,
                 max_pending=1 << 16, pool=1, mode=PEOS_MODE_PEOS, eps=0.1, launch_waves=0,
                 hbm_budget=0, lds_budget=0):
        cfg = peos_serve_config(max_batch, max_k, max_ef, max_inflight, max_pending, pool, mode,
                                launch_waves, eps, 0.0, hbm_budget, lds_budget)
        h = ctypes.c_void_p()
        _check("peos_serve_open", lib().peos_serve_open(index.handle, ctypes.byref(cfg),
                                                        ctypes.byref(h)))
        self.handle = h
        self.index = index
        self.live = {}
        self._done = np.zeros(4096, np.uint64)

    def submit(self, queries, k, ef):
        """queries: host (nq, d) float32.  Returns the ticket; raises
        PeosError (code PEOS_EBUSY) when the queue is full."""
        q = np.ascontiguousarray(queries, dtype=np.float32)
        nq = q.shape[0]
        ids = np.empty((nq, k), np.int64)
        dists = np.empty((nq, k), np.float32)
        t = ctypes.c_uint64()
        # the buffers are held before the call: the library writes to them
        # until the request completes
        self._held = (q, ids, dists)
        try:
            _check("peos_serve_submit",
                   lib().peos_serve_submit(self.handle, q.ctypes.data, nq, int(k), int(ef),
                                           ids.ctypes.data, dists.ctypes.data, ctypes.byref(t)))
            self.live[t.value] = (q, ids, dists)
        finally:
            self._held = None
        return t.value

    def poll(self, wait=False):
        """[(ticket, ids, dists)] of the requests completed since the last poll."""
        out = []
        n = ctypes.c_int32()
        while True:
            _check("peos_serve_poll", lib().peos_serve_poll(self.handle, 1 if wait else 0,
                                                            self._done.ctypes.data,
                                                            len(self._done), ctypes.byref(n)))
            for t in self._done[:n.value].tolist():
                _, ids, dists = self.live.pop(t)
                out.append((t, ids, dists))
            if n.value < len(self._done):
                return out
            wait = False

    def counters(self):
        c = np.zeros(8, np.int64)
        _check("peos_serve_counters", lib().peos_serve_counters(self.handle, c.ctypes.data))
        return dict(zip(SERVE_COUNTERS, c.tolist()))

    def close(self):
        if self.handle:
            lib().peos_serve_close(self.handle)
            self.handle = None
            self.live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
