"""PEOs oracle -- TEST INFRASTRUCTURE ONLY.

A plain CPU implementation of what the PEOs-routed graph search computes,
written from the paper (Lu, Xiao, Ishikawa, ICML 2024) to check the HIP
library.  It shares no code with that library and never imports it.  Only the
test suite, the smoke entry and the CPU-baseline leg of the benchmark may use
it; the product path never does.

Parts:
  * ``peos_oracle.c`` (loaded here through ctypes): edge records of PEOs steps
    (1)-(3), the projection table of step (5), the routing test of steps (4)
    and (6) / Alg. 2, and the search loop of Alg. 1 -- double precision, with
    the edge codes decided in single precision (see that file's header).
  * this module: exact brute-force k-NN in float64 (the recall reference) and
    the closed forms of the analysis section used as pins.

Every function below is pinned by a test in tests/test_oracle_*.py.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

L2 = 0
ANGULAR = 1
IP = 2  # maximum inner product, distance -x.q (appendix, Extension to MIPS)
MODE_PEOS = 0
MODE_EXHAUSTIVE = 1
MODE_SIMHASH = 2

COUNTERS = ("expansions", "edges", "visited_skips", "tests", "test_ge1", "test_le0",
            "test_h", "test_zero", "passes", "ndist", "inserted", "test_expansions")
F_HT, F_A1, F_A0, F_DELTA, F_ORDER = 1, 2, 4, 8, 16
LP_BF16_BASE, LP_FP16 = 1, 2
LP_COMPACT = 8  # compact records: L <= 4, w_reg = 1, w_res = 0, 8-bit scalars, quantile table
COMPACT_LUT_BINS = 256

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "peos_oracle.c")
# PEOS_ORACLE_LIB: another build of the same source (the sanitizer test's)
_LIB = os.environ.get("PEOS_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C part with gcc (no fp contraction, so the single-precision
    code decisions follow the stated fmaf order exactly)."""
    stale = (not os.path.exists(_LIB)
             or os.path.getmtime(_LIB) < os.path.getmtime(_SRC))
    if force or stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-pthread", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32, f64 = ctypes.c_int64, ctypes.c_int, ctypes.c_double
        lib.oracle_norm_ppf.argtypes = [f64]
        lib.oracle_norm_ppf.restype = f64
        lib.oracle_threshold.argtypes = [f64, f64, f64, i32, f64, f64]
        lib.oracle_threshold.restype = f64
        lib.oracle_edge_record.argtypes = [P, P, i32, i32, i32, P, P, P, P, P]
        lib.oracle_edge_record.restype = i32
        lib.oracle_build_tables.argtypes = [P, i64, i32, P, i32, i32, i32, P, P, P, P, P, i32]
        lib.oracle_build_tables.restype = i32
        lib.oracle_query_table.argtypes = [P, i32, i32, i32, P, P, P]
        lib.oracle_query_table.restype = None
        lib.oracle_test_edge.argtypes = [P, P, P, P, i32, i32, i32, P, P, i32, f64, i32, P, i32, P]
        lib.oracle_test_edge.restype = i32
        lib.oracle_search.argtypes = [P, i64, i32, P, i32, i32, i32, i32, P, P, i32, P, i64, P, P,
                                      i32, i32, f64, i32, f64, i32, i32, P, P, i32, P, i32, P, P, P,
                                      P, P, P]
        lib.oracle_descend.argtypes = [P, i64, i32, i32, P, P, P, i64, i32, i32, P, i64, i32, i32,
                                       f64, P, P, P]
        lib.oracle_descend.restype = i32
        lib.oracle_search.restype = i32
        lib.oracle_dimension_permutation.argtypes = [P, i64, i32, P, i32, i32, P, P]
        lib.oracle_simhash_bits.argtypes = [P, i32, P, i32, P]
        lib.oracle_simhash_bits.restype = None
        lib.oracle_dimension_permutation.restype = i32
        lib.oracle_compact_lut.argtypes = [i32, i32, f64, P]
        lib.oracle_compact_lut.restype = None
        lib.oracle_compact_tables.argtypes = [P, i64, i32, P, i32, i32, i32, P, P, P, P]
        lib.oracle_compact_tables.restype = i32
        lib.oracle_compact_test.argtypes = [P, i32, i32, P, P, i32, i32, i32, P, P, i32, f64, f64,
                                            f64, P]
        lib.oracle_compact_test.restype = i32
        lib.oracle_round_half.argtypes = [f64]
        lib.oracle_round_half.restype = f64
        lib.oracle_round_bf16.argtypes = [ctypes.c_float]
        lib.oracle_round_bf16.restype = ctypes.c_float
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


# ---------------------------------------------------------------------------
# constants
# ---------------------------------------------------------------------------
def round_half(x: float) -> float:
    """Nearest binary16 value (ties to even), as a float."""
    return _load().oracle_round_half(float(x))


def round_bf16(x: float) -> float:
    """Nearest bfloat16 value of a float32 (ties to even)."""
    return _load().oracle_round_bf16(float(x))


def norm_ppf(p: float) -> float:
    """Standard normal quantile (bisection on the erfc form of the CDF)."""
    return _load().oracle_norm_ppf(float(p))


def eta(L: int, m: int) -> float:
    """sqrt(2 L ln m): the mean scale of N_min^{e,x} in step (4)."""
    return math.sqrt(2.0 * L * math.log(m))


def threshold(A: float, w_reg: float, w_res: float, L: int, m: int, eps: float) -> float:
    """T_r of step (6): eps-quantile of N(A eta, w_reg^2 + L w_res^2 - L A^2/(L+1))."""
    return _load().oracle_threshold(float(A), float(w_reg), float(w_res), int(L), eta(L, m),
                                    norm_ppf(eps))


# ---------------------------------------------------------------------------
# steps (1)-(3), (5), (6)
# ---------------------------------------------------------------------------
def edge_record(xv, xu, L, m, A, B):
    """Codes (L+1 bytes; [0] residual, [1..L] blocks), scalars
    {|e|, w_reg, w_res, g_e=(|u|^2-|v|^2)/2} and the smallest top-2 margin."""
    xv, xu, A, B = _f32(xv), _f32(xu), _f32(A), _f32(B)
    d = xv.shape[0]
    codes = np.zeros(L + 1, np.uint8)
    scal = np.zeros(4, np.float64)
    margin = np.zeros(1, np.float64)
    rc = _load().oracle_edge_record(_p(xv), _p(xu), d, L, m, _p(A), _p(B), _p(codes), _p(scal),
                                    _p(margin))
    if rc:
        raise ValueError("bad edge-record arguments")
    return codes, scal, float(margin[0])


def build_tables(base, graph, L, m, A, B, nthreads=None):
    """Records of every edge: codes (n, R, L+1) uint8, scal (n, R, 4) float64,
    margin (n, R) float64.  Padding edges are zero."""
    base, A, B = _f32(base), _f32(A), _f32(B)
    graph = np.ascontiguousarray(graph, dtype=np.int32)
    n, d = base.shape
    R = graph.shape[1]
    codes = np.zeros((n, R, L + 1), np.uint8)
    scal = np.zeros((n, R, 4), np.float64)
    margin = np.zeros((n, R), np.float64)
    nt = nthreads or min(16, os.cpu_count() or 1)
    rc = _load().oracle_build_tables(_p(base), n, d, _p(graph), R, L, m, _p(A), _p(B), _p(codes),
                                     _p(scal), _p(margin), nt)
    if rc:
        raise ValueError("bad build arguments")
    return codes, scal, margin


def query_table(q, L, m, A, B):
    """(L+1) x m projection table of step (5) in float64: row 0 = q'.b_j,
    row i = q'_i . a^i_j."""
    q, A, B = _f32(q), _f32(A), _f32(B)
    out = np.zeros((L + 1, m), np.float64)
    _load().oracle_query_table(_p(q), q.shape[0], L, m, _p(A), _p(B), _p(out))
    return out


def test_edge(xv, xu, xp, q, L, m, A, B, metric, eps, lowp=0, simhash=None):
    """One routing test of edge (v, u) against furthest result p.
    Returns (pass, A_r, H, T, kind) with kind 0 zero edge / 1 A>=1 / 2 A<=0 / 3 H-vs-T.
    lowp = LP_FP16: the precision-form test (half-rounded scalars and table).
    simhash (nb, d): the SimHash test; H is then the collision count."""
    xv, xu, xp, q, A, B = map(_f32, (xv, xu, xp, q, A, B))
    out = np.zeros(4, np.float64)
    sh = None if simhash is None else _f32(simhash)
    ok = _load().oracle_test_edge(_p(xv), _p(xu), _p(xp), _p(q), q.shape[0], L, m, _p(A), _p(B),
                                  metric, float(eps), int(lowp), _p(sh),
                                  0 if sh is None else sh.shape[0], _p(out))
    return bool(ok), out[0], out[1], out[2], int(out[3])


# ---------------------------------------------------------------------------
# Alg. 1
# ---------------------------------------------------------------------------
def search(base, graph, entry, queries, k, ef, L, m, A, B, metric, eps, mode=MODE_PEOS,
           tau=1e-5, nthreads=None, kstride=None, pool=0, precision=64, lowp=0, perm=None,
           simhash=None, entries=None):
    """Batched search.  k, ef: scalars or per-query arrays (ef := max(ef, k)).
    pool: capacity of the candidate list; 0 = unbounded (Alg. 1 as printed),
    0 < pool <= ef = the HNSW stopping rule, pool < 0 = |pool| x each
    query's ef.  precision: 64 = distances in float64;
    32 = the distance decisions taken on the canonical single-precision
    distances (the GPU kernel's precision; see dist32 in peos_oracle.c).
    lowp: precision form (LP_FP16 and LP_BF16_BASE imply precision 32):
    LP_FP16 = routing test on half-rounded edge scalars and tables;
    LP_BF16_BASE = traversal on the bfloat16-rounded base, result list
    re-ranked in single precision on the full base (see routing_test_lowp and
    oracle_search in peos_oracle.c); LP_COMPACT = the compact records' test
    (its scalar codes and quantile table are single-precision decisions in
    either precision; the search distances follow `precision`).
    perm: optional dimension permutation (d ints) of the test: edge records
    and tables on permuted coordinates, distances on the original ones.
    simhash: (nb, d) sign-projection vectors, required by MODE_SIMHASH.
    entries: optional per-query entry nodes (from descend) instead of entry.
    Returns dict(ids (nq, kstride) int64, dist (as decided), dist64 float64,
    counters (nq, 11) int64, fragile (nq,) int32 flag words, status (nq,) int32)."""
    if precision not in (32, 64):
        raise ValueError("precision must be 32 or 64")
    base, queries = _f32(base), _f32(queries)
    A = _f32(A) if A is not None else np.zeros(1, np.float32)
    B = _f32(B) if B is not None else np.zeros(1, np.float32)
    graph = np.ascontiguousarray(graph, dtype=np.int32)
    n, d = base.shape
    nq = queries.shape[0]
    karr = np.ascontiguousarray(np.broadcast_to(np.asarray(k, np.int32), (nq,)))
    efarr = np.ascontiguousarray(np.broadcast_to(np.asarray(ef, np.int32), (nq,)))
    ks = int(kstride or (karr.max() if nq else 1))
    ids = np.zeros((nq, ks), np.int64)
    dist = np.zeros((nq, ks), np.float64)
    dist64 = np.zeros((nq, ks), np.float64)
    cnt = np.zeros((nq, len(COUNTERS)), np.int64)
    frag = np.zeros(nq, np.int32)
    status = np.zeros(nq, np.int32)
    nt = nthreads or min(16, os.cpu_count() or 1)
    perm_arr = None if perm is None else np.ascontiguousarray(perm, dtype=np.int32)
    if perm_arr is not None and sorted(perm_arr.tolist()) != list(range(d)):
        raise ValueError("perm must be a permutation of range(d)")
    sh = None if simhash is None else _f32(simhash)
    nb = 0 if sh is None else sh.shape[0]
    ent = None if entries is None else np.ascontiguousarray(entries, dtype=np.int32)
    if ent is not None and (ent.shape != (nq,) or ent.min(initial=0) < 0 or ent.max(initial=0) >= n):
        raise ValueError("entries must hold one base id per query")
    rc = _load().oracle_search(_p(base), n, d, _p(graph), graph.shape[1], int(entry), L, m, _p(A),
                               _p(B), metric, _p(queries), nq, _p(karr), _p(efarr), ks,
                               int(pool), float(eps), mode, float(tau), 1 if precision == 32 else 0,
                               int(lowp), _p(perm_arr), _p(sh), nb, _p(ent), nt, _p(ids),
                               _p(dist),
                               _p(dist64), _p(cnt), _p(frag), _p(status))
    if rc:
        raise ValueError("bad search arguments")
    return dict(ids=ids, dist=dist, dist64=dist64, counters=cnt, fragile=frag, status=status)


def descend(base, layers, queries, metric, precision=32, lowp=0, tau=1e-5):
    """Greedy descent through upper layers to each query's entry node (see
    oracle_descend in peos_oracle.c).  layers: dict with node (rows,), adj
    (rows, Ru), down (rows,), top.  Returns (entries (nq,) int32, ndist (nq,)
    int64, fragile (nq,) int32)."""
    base, queries = _f32(base), _f32(queries)
    node = np.ascontiguousarray(layers["node"], dtype=np.int32)
    adj = np.ascontiguousarray(layers["adj"], dtype=np.int32)
    down = np.ascontiguousarray(layers["down"], dtype=np.int32)
    n, d = base.shape
    nq = queries.shape[0]
    ent = np.zeros(nq, np.int32)
    nd = np.zeros(nq, np.int64)
    frag = np.zeros(nq, np.int32)
    rc = _load().oracle_descend(_p(base), n, d, int(metric), _p(node), _p(adj), _p(down),
                                node.shape[0], adj.shape[1], int(layers["top"]), _p(queries), nq,
                                1 if precision == 32 else 0, int(lowp), float(tau), _p(ent),
                                _p(nd), _p(frag))
    if rc:
        raise ValueError("bad descent arguments")
    return ent, nd, frag


def simhash_bits(v, C):
    """Sign bits [v . c_i >= 0] of the rows of C, as a uint64 word array."""
    v, C = _f32(v), _f32(C)
    nb = C.shape[0]
    bits = np.zeros((nb + 63) // 64, np.uint64)
    _load().oracle_simhash_bits(_p(v), v.shape[0], _p(C), nb, _p(bits))
    return bits


def compact_lut(L, m, eps):
    """Quantile table of the compact form: entry b = T(b/256) of step (6) with
    w_reg = 1, w_res = 0, rounded down to float32 (see peos_oracle.c)."""
    out = np.zeros(COMPACT_LUT_BINS, np.float32)
    _load().oracle_compact_lut(int(L), int(m), float(eps), _p(out))
    return out


def compact_tables(base, graph, L, metric, perm=None):
    """Compact records: hdr (n, 4) float32 {g_lo, g_step, i_lo, i_step} per
    node; cg, ci (n, R) uint8 codes of g_e/|e| (floor) and 1/|e| (nearest;
    255 = zero-length edge)."""
    base = _f32(base)
    graph = np.ascontiguousarray(graph, dtype=np.int32)
    n, d = base.shape
    R = graph.shape[1]
    hdr = np.zeros((n, 4), np.float32)
    cg = np.zeros((n, R), np.uint8)
    ci = np.zeros((n, R), np.uint8)
    pa = None if perm is None else np.ascontiguousarray(perm, dtype=np.int32)
    rc = _load().oracle_compact_tables(_p(base), n, d, _p(graph), R, int(L), int(metric), _p(pa),
                                       _p(hdr), _p(cg), _p(ci))
    if rc:
        raise ValueError("bad compact-table arguments")
    return hdr, cg, ci


def compact_test(hdr, cg, ci, codes, q, L, m, A, B, metric, eps, dv, delta):
    """One compact-form test on decoded codes and traversal distances.
    Returns (pass, A_r, H, T, kind)."""
    hdr, q, A, B = _f32(hdr), _f32(q), _f32(A), _f32(B)
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    out = np.zeros(4, np.float64)
    ok = _load().oracle_compact_test(_p(hdr), int(cg), int(ci), _p(codes), _p(q), q.shape[0],
                                     int(L), int(m), _p(A), _p(B), int(metric), float(eps),
                                     float(dv), float(delta), _p(out))
    if ok < 0:
        raise ValueError("bad compact-test arguments")
    return bool(ok), out[0], out[1], out[2], int(out[3])


def dimension_permutation(base, graph, L):
    """The optional dimension permutation (appendix "Dimension Permutation"):
    returns (perm, avg) with perm[i*d/L + t] the original dimension placed at
    coordinate t of sub-vector i, avg[j] = mean squared j-th edge coordinate."""
    base = _f32(base)
    graph = np.ascontiguousarray(graph, dtype=np.int32)
    n, d = base.shape
    perm = np.zeros(d, np.int32)
    avg = np.zeros(d, np.float64)
    rc = _load().oracle_dimension_permutation(_p(base), n, d, _p(graph), graph.shape[1], L,
                                              _p(perm), _p(avg))
    if rc:
        raise ValueError("bad arguments")
    return perm, avg


# ---------------------------------------------------------------------------
# exact k-NN (recall reference)
# ---------------------------------------------------------------------------
def brute_force(base, queries, k, metric):
    """Exact top-k in float64 by (distance, id): squared l2, 1 - x.q/|q|, or
    -x.q (inner product)."""
    xb = np.asarray(base, np.float64)
    ids_out = np.full((len(queries), k), -1, np.int64)
    d_out = np.full((len(queries), k), np.inf)
    for i, q in enumerate(np.asarray(queries, np.float64)):
        if metric == L2:
            dd = ((xb - q) ** 2).sum(1)
        elif metric == IP:
            dd = -(xb @ q)
        else:
            dd = 1.0 - xb @ q / np.linalg.norm(q)
        order = np.lexsort((np.arange(len(dd)), dd))[:k]
        ids_out[i, :len(order)] = order
        d_out[i, :len(order)] = dd[order]
    return ids_out, d_out


# ---------------------------------------------------------------------------
# closed forms of the analysis section (pins)
# ---------------------------------------------------------------------------
def ewreg_exact(L: int, d: int) -> float:
    """E[w_reg] for e uniform on the sphere: sqrt(L) E[sqrt(X)] with
    X ~ Beta(d'/2, (d-d')/2), written with Gamma functions (proof of the
    lemma bounding w_reg)."""
    dp = d // L
    lg = math.lgamma
    return math.sqrt(L) * (dp - 1) / (d - 1) * math.exp(
        lg((dp - 1) / 2) + lg(d / 2) - lg(dp / 2) - lg((d - 1) / 2))


def ewreg_bound(L: int, d: int) -> float:
    """The lemma's lower bound (d'-1) sqrt(2Ld-3L) / ((d-1) sqrt(2d'+2 sqrt3-6))."""
    dp = d / L
    return (dp - 1) * math.sqrt(2 * L * d - 3 * L) / ((d - 1) * math.sqrt(2 * dp + 2 * math.sqrt(3) - 6))


def rceos_min_m(n_hash: int, theta: float) -> float:
    """RCEOs beats SimHash with n hash functions when m > exp(n / (2 theta (pi - theta)))."""
    return math.exp(n_hash / (2 * theta * (math.pi - theta)))


def peos_opt_min_L(n_hash: int, theta: float, m: int) -> float:
    """PEOs(opt): L ln m > n / (2 theta (pi - theta))."""
    return n_hash / (2 * theta * (math.pi - theta)) / math.log(m)


def peos_crossing_L(n_hash: int, theta: float, m: int, d: int) -> float:
    """Smallest real L with L ln m > (w_reg^2 + L w_res^2) n / (2 theta (pi-theta)),
    w_res^2 taken as E[w_res^2] = 1 - E[w_reg^2] under the isotropic law, with
    E[w_reg^2] = L E[X], X ~ Beta(d'/2, (d-d')/2) = L (d'/d) = 1 for integer d';
    for real L the expectation is evaluated with d' = d/L through
    E[w_reg]^2 + Var, approximated here by E[w_reg]^2 (Table 5 setting)."""
    c = n_hash / (2 * theta * (math.pi - theta))

    def f(L):
        dp = d / L
        lg = math.lgamma
        ew = math.sqrt(L) * (dp - 1) / (d - 1) * math.exp(
            lg((dp - 1) / 2) + lg(d / 2) - lg(dp / 2) - lg((d - 1) / 2))
        wres2 = max(0.0, 1.0 - ew * ew)
        return L * math.log(m) - (ew * ew + L * wres2) * c

    lo, hi = 1.01, 50.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(mid) > 0:
            hi = mid
        else:
            lo = mid
    return hi


def max_abs_normal_moments(m: int):
    """Mean and variance of M_m = max of m iid |N(0,1)| (numerical integration
    of its CDF (2 Phi(x) - 1)^m)."""
    from scipy import integrate, stats

    cdf = lambda x: (2 * stats.norm.cdf(x) - 1) ** m
    mean = integrate.quad(lambda x: 1 - cdf(x), 0, np.inf, epsabs=1e-13)[0]
    ex2 = integrate.quad(lambda x: 2 * x * (1 - cdf(x)), 0, np.inf, epsabs=1e-13)[0]
    return mean, ex2 - mean * mean
