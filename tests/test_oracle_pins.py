"""Pins of the oracle against what the paper and mathematics fix.

Each test ties one oracle function to something other than itself: values
printed in the paper (tests/golden/), closed forms of the analysis section,
special inputs that reduce a step to its textbook definition, brute force on
tiny inputs, and invariants of the search (disabling the test reproduces
exhaustive-neighbour search; the single sorted list equals the two-heap
formulation).
"""
import heapq
import math
import os

import numpy as np
import pytest
from scipy import stats
from scipy.spatial.distance import cdist

import oracle as O
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_printed_values.txt")


def golden():
    out = {}
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        key, val = line.split()[:2]
        out[key] = float(val)
    return out


@pytest.fixture(scope="module", autouse=True)
def _lib(oracle_lib):
    return oracle_lib


# ---------------------------------------------------------------------------
# P8: threshold closed form, quantile constants, eta
# ---------------------------------------------------------------------------
def test_norm_ppf_matches_scipy():
    for p in [1e-12, 1e-4, 0.05, 0.1, 0.2, 0.3, 0.5]:
        assert O.norm_ppf(p) == pytest.approx(stats.norm.ppf(p), rel=1e-12, abs=1e-13)
    # textbook values
    assert O.norm_ppf(0.05) == pytest.approx(-1.644853626951473, abs=1e-12)
    assert O.norm_ppf(0.1) == pytest.approx(-1.281551565544601, abs=1e-12)
    assert O.norm_ppf(0.2) == pytest.approx(-0.841621233572914, abs=1e-12)


def test_eta_values():
    assert O.eta(4, 16) == pytest.approx(4.709640, abs=1e-6)
    assert O.eta(8, 16) == pytest.approx(6.660437, abs=1e-6)
    assert O.eta(16, 16) == pytest.approx(9.419280, abs=1e-6)


@pytest.mark.parametrize("L,m,eps", [(4, 16, 0.1), (8, 16, 0.05), (16, 16, 0.2), (8, 128, 0.2), (1, 128, 0.5)])
def test_threshold_is_normal_quantile(L, m, eps):
    rng = np.random.default_rng(5)
    for _ in range(50):
        A = rng.uniform(0.001, 0.999)
        wreg = rng.uniform(0.5, 1.0)
        wres = math.sqrt(1 - wreg * wreg)
        var = wreg ** 2 + L * wres ** 2 - L * A * A / (L + 1)
        ref = stats.norm.ppf(eps, loc=A * math.sqrt(2 * L * math.log(m)), scale=math.sqrt(var))
        assert O.threshold(A, wreg, wres, L, m, eps) == pytest.approx(ref, rel=1e-11, abs=1e-11)


def test_threshold_monotone_in_A():
    for eps in (0.05, 0.2, 0.5):
        A = np.linspace(0.001, 0.999, 400)
        T = [O.threshold(a, 0.97, math.sqrt(1 - 0.97 ** 2), 8, 16, eps) for a in A]
        assert np.all(np.diff(T) > 0)


# ---------------------------------------------------------------------------
# P9: closed forms of the analysis section vs the printed values
# ---------------------------------------------------------------------------
def test_wreg_bound_and_exact_mean_vs_printed():
    g = golden()
    bound = O.ewreg_bound(8, 128)
    assert bound == pytest.approx(0.97892, abs=5e-6)
    assert math.floor(bound * 1000) / 1000 == g["wreg_bound_d128_L8"]
    assert O.ewreg_exact(8, 128) == pytest.approx(0.98643, abs=5e-6)
    assert O.ewreg_exact(8, 128) >= bound


def test_table5_values():
    g = golden()
    assert math.ceil(O.rceos_min_m(64, math.pi / 2)) == g["table5_rceos_min_m"]
    assert round(O.peos_opt_min_L(64, math.pi / 2, 128), 2) == g["table5_peos_opt_min_L"]
    crossing = O.peos_crossing_L(64, math.pi / 2, 128, 384)
    assert crossing > O.peos_opt_min_L(64, math.pi / 2, 128)
    assert abs(crossing - g["table5_peos_min_L"]) < 0.01


def test_max_abs_normal_moments():
    mean, var = O.max_abs_normal_moments(16)
    assert mean == pytest.approx(2.0772, abs=1e-4) and var == pytest.approx(0.2347, abs=1e-4)
    # Monte Carlo cross-check
    z = np.abs(np.random.default_rng(0).standard_normal((400000, 16))).max(1)
    assert z.mean() == pytest.approx(mean, abs=4e-3)
    mean128, _ = O.max_abs_normal_moments(128)
    assert mean128 == pytest.approx(2.8276, abs=1e-4)


# ---------------------------------------------------------------------------
# P6: edge records (steps (1)-(3))
# ---------------------------------------------------------------------------
def _blocks(e, L):
    return e.reshape(L, -1)


def test_edge_scalars_closed_forms():
    rng = np.random.default_rng(11)
    L, m, d = 8, 16, 128
    A, B = W.make_directions(L, m, d, 3)
    for _ in range(200):
        xv = rng.standard_normal(d).astype(np.float32)
        xu = (xv + rng.standard_normal(d) * rng.uniform(0.1, 3)).astype(np.float32)
        codes, scal, _ = O.edge_record(xv, xu, L, m, A, B)
        e = xu.astype(np.float64) - xv.astype(np.float64)
        s = np.linalg.norm(_blocks(e, L), axis=1)
        assert scal[0] == pytest.approx(np.linalg.norm(e), rel=1e-12)
        assert scal[1] ** 2 + scal[2] ** 2 == pytest.approx(1.0, abs=1e-12)
        assert scal[1] == pytest.approx(s.sum() / (math.sqrt(L) * np.linalg.norm(e)), rel=1e-12)
        g_e = 0.5 * (xu.astype(np.float64) @ xu - xv.astype(np.float64) @ xv)
        assert scal[3] == pytest.approx(g_e, rel=1e-12, abs=1e-9)


def test_equal_block_norms_give_wreg_one():
    L, m, d = 4, 16, 32
    A, B = W.make_directions(L, m, d, 4)
    rng = np.random.default_rng(2)
    blocks = rng.standard_normal((L, d // L))
    blocks /= np.linalg.norm(blocks, axis=1, keepdims=True)
    xu = blocks.reshape(-1).astype(np.float32)
    _, scal, _ = O.edge_record(np.zeros(d, np.float32), xu, L, m, A, B)
    assert scal[1] == pytest.approx(1.0, abs=1e-7) and scal[2] == pytest.approx(0.0, abs=1e-3)


def test_codes_are_argmax_of_projections():
    """Codes equal the float64 argmax of |e_i . a^i_j| (and of |e_res . b_j|
    with e_res = e - (sum_k s_k / L)[e_i / s_i]) wherever the top two are not
    within 1e-5 relative."""
    rng = np.random.default_rng(12)
    L, m, d = 8, 16, 128
    A, B = W.make_directions(L, m, d, 5)
    checked = 0
    for _ in range(300):
        xv = rng.standard_normal(d).astype(np.float32)
        xu = (xv + rng.standard_normal(d)).astype(np.float32)
        codes, _, margin = O.edge_record(xv, xu, L, m, A, B)
        if margin < 1e-5:
            continue
        e = xu.astype(np.float64) - xv.astype(np.float64)
        eb = _blocks(e, L)
        for i in range(L):
            p = A[i].astype(np.float64) @ eb[i]
            j = int(np.argmax(np.abs(p)))
            assert codes[1 + i] == j + (m if p[j] < 0 else 0)
        s = np.linalg.norm(eb, axis=1)
        eres = (eb - (s.sum() / L) * eb / s[:, None]).reshape(-1)
        p = B.astype(np.float64) @ eres
        j = int(np.argmax(np.abs(p)))
        assert codes[0] == j + (m if p[j] < 0 else 0)
        checked += 1
    assert checked > 250


def test_basis_edge_code_reduces_to_direction_entry():
    """e = +/- basis vector t of block i: |e_i . a^i_j| = |a^i_j[t]|."""
    L, m, d = 4, 16, 32
    A, B = W.make_directions(L, m, d, 6)
    dp = d // L
    for i in range(L):
        for t in range(dp):
            for sgn in (1.0, -1.0):
                xu = np.zeros(d, np.float32)
                xu[i * dp + t] = sgn
                codes, scal, _ = O.edge_record(np.zeros(d, np.float32), xu, L, m, A, B)
                col = sgn * A[i, :, t].astype(np.float64)
                j = int(np.argmax(np.abs(col)))
                assert codes[1 + i] == j + (m if col[j] < 0 else 0)
                # blocks other than i are zero: code (+, first direction)
                for i2 in range(L):
                    if i2 != i:
                        assert codes[1 + i2] == 0
                # one nonzero block: e is its own regular part
                assert scal[1] == pytest.approx(1.0) and scal[2] == pytest.approx(0.0, abs=1e-12)
                assert codes[0] == 0


def test_zero_edge_record():
    L, m, d = 4, 16, 32
    A, B = W.make_directions(L, m, d, 7)
    x = np.random.default_rng(1).standard_normal(d).astype(np.float32)
    codes, scal, _ = O.edge_record(x, x, L, m, A, B)
    assert np.all(codes == 0) and scal[0] == 0 and scal[1] == 1 and scal[2] == 0


def test_single_subspace_is_rceos():
    """L = 1: w_reg = 1, w_res = 0, and the code is the RCEOs argmax over the
    full-space directions."""
    rng = np.random.default_rng(3)
    m, d = 16, 32
    A, B = W.make_directions(1, m, d, 8)
    for _ in range(50):
        xv = rng.standard_normal(d).astype(np.float32)
        xu = rng.standard_normal(d).astype(np.float32)
        codes, scal, margin = O.edge_record(xv, xu, 1, m, A, B)
        assert scal[1] == pytest.approx(1.0, abs=1e-12) and scal[2] == pytest.approx(0.0, abs=1e-7)
        if margin < 1e-5:
            continue
        p = A[0].astype(np.float64) @ (xu.astype(np.float64) - xv)
        j = int(np.argmax(np.abs(p)))
        assert codes[1] == j + (m if p[j] < 0 else 0)


def test_isotropic_wreg_mean_matches_gamma_form():
    rng = np.random.default_rng(21)
    L, m, d = 8, 16, 128
    A, B = W.make_directions(L, m, d, 9)
    N = 6000
    w = np.empty(N)
    z = np.zeros(d, np.float32)
    for t in range(N):
        _, scal, _ = O.edge_record(z, rng.standard_normal(d).astype(np.float32), L, m, A, B)
        w[t] = scal[1]
    se = w.std() / math.sqrt(N)
    assert abs(w.mean() - O.ewreg_exact(L, d)) < 4 * se
    assert w.mean() >= golden()["wreg_bound_d128_L8"]


def test_zero_block_projection_reading():
    """A zero block: e_reg is the projection on the line of
    g = [e_i/(sqrt(L)|e_i|)] with a zero component there, so
    w_reg = sum_i |e_i| / (sqrt(L') |e|), L' = nonzero blocks."""
    L, m, d = 4, 16, 32
    A, B = W.make_directions(L, m, d, 10)
    rng = np.random.default_rng(4)
    xu = rng.standard_normal(d).astype(np.float32)
    xu[8:16] = 0.0
    codes, scal, _ = O.edge_record(np.zeros(d, np.float32), xu, L, m, A, B)
    e = xu.astype(np.float64)
    s = np.linalg.norm(e.reshape(L, -1), axis=1)
    assert scal[1] == pytest.approx(s.sum() / (math.sqrt(3) * np.linalg.norm(e)), rel=1e-12)
    assert scal[1] ** 2 + scal[2] ** 2 == pytest.approx(1.0, abs=1e-12)
    assert codes[2] == 0


# ---------------------------------------------------------------------------
# step (5): projection table
# ---------------------------------------------------------------------------
def test_table_of_basis_query_is_direction_entry():
    L, m, d = 4, 16, 32
    A, B = W.make_directions(L, m, d, 11)
    dp = d // L
    for k in range(d):
        q = np.zeros(d, np.float32)
        q[k] = 3.0  # normalization removes the 3
        T = O.query_table(q, L, m, A, B)
        np.testing.assert_allclose(T[0], B[:, k], rtol=0, atol=1e-12)
        i, t = divmod(k, dp)
        np.testing.assert_allclose(T[1 + i], A[i, :, t], rtol=0, atol=1e-12)
        for i2 in range(L):
            if i2 != i:
                assert np.all(T[1 + i2] == 0)


# ---------------------------------------------------------------------------
# P7: the projection estimate has the closed-form mean and variance
# ---------------------------------------------------------------------------
def _H_moments(e, q, L, m, wreg, wres):
    Mm, Mv = O.max_abs_normal_moments(m)
    qn = q / np.linalg.norm(q)
    eb, qb = e.reshape(L, -1), qn.reshape(L, -1)
    mu1 = var1 = 0.0
    for i in range(L):
        nq = np.linalg.norm(qb[i])
        c = eb[i] @ qb[i] / (np.linalg.norm(eb[i]) * nq)
        mu1 += nq * c * Mm
        var1 += nq * nq * (c * c * Mv + 1 - c * c)
    s = np.linalg.norm(eb, axis=1)
    eres = (eb - (s.sum() / L) * eb / s[:, None]).reshape(-1)
    c0 = eres @ qn / np.linalg.norm(eres)
    mu = wreg * mu1 + math.sqrt(L) * wres * c0 * Mm
    var = wreg ** 2 * var1 + L * wres ** 2 * (c0 * c0 * Mv + 1 - c0 * c0)
    return mu, var


@pytest.mark.parametrize("metric", [W.L2, W.ANGULAR])
def test_projection_estimate_moments(metric):
    """Over random direction draws, H of the test has the mean and variance
    the extreme-value argument gives (per block: |q'_i| cos(theta_i) M_m plus
    an independent N(0, |q'_i|^2 sin^2) term; M_m = max of m |N(0,1)|)."""
    rng = np.random.default_rng(31)
    L, m, d = 4, 16, 32
    xv = rng.standard_normal(d).astype(np.float32)
    xu = (xv + rng.standard_normal(d) * np.repeat([0.6, 1.0, 1.4, 0.8], d // L)).astype(np.float32)
    q = (xv + 0.8 * (xu - xv) + 0.9 * rng.standard_normal(d)).astype(np.float32)
    # choose p so that 0 < A < 1 for this edge: p at the distance that puts A mid-range
    N = 5000
    Hs = []
    wreg = wres = None
    for t in range(N):
        A, B = W.make_directions(L, m, d, 10_000 + t)
        codes, scal, _ = O.edge_record(xv, xu, L, m, A, B)
        T = O.query_table(q, L, m, A, B)
        lk = lambda i, c: (-1.0 if c >= m else 1.0) * T[i, c % m]
        H1 = sum(lk(i, codes[i]) for i in range(1, L + 1))
        H2 = lk(0, codes[0])
        wreg, wres = scal[1], scal[2]
        Hs.append(wreg * H1 + math.sqrt(L) * wres * H2)
    Hs = np.array(Hs)
    e = xu.astype(np.float64) - xv
    mu, var = _H_moments(e, q.astype(np.float64), L, m, wreg, wres)
    assert abs(Hs.mean() - mu) < 4 * math.sqrt(var / N)
    assert Hs.var() == pytest.approx(var, rel=0.08)


def test_routing_test_H_matches_table_sum():
    """The H reported by the routing test is w_reg H1 + sqrt(L) w_res H2 built
    from the same codes and table (ties test_edge to the P7 pin)."""
    rng = np.random.default_rng(8)
    L, m, d = 4, 16, 32
    A, B = W.make_directions(L, m, d, 12)
    n_h = 0
    for _ in range(300):
        xv, q = rng.standard_normal((2, d)).astype(np.float32)
        xu = (xv + 0.5 * rng.standard_normal(d)).astype(np.float32)
        xp = (q + rng.standard_normal(d) * rng.uniform(0.5, 2)).astype(np.float32)
        ok, Ar, H, T, kind = O.test_edge(xv, xu, xp, q, L, m, A, B, W.L2, 0.1)
        if kind != 3:
            continue
        codes, scal, _ = O.edge_record(xv, xu, L, m, A, B)
        tab = O.query_table(q, L, m, A, B)
        lk = lambda i, c: (-1.0 if c >= m else 1.0) * tab[i, c % m]
        H_ref = scal[1] * sum(lk(i, codes[i]) for i in range(1, L + 1)) + math.sqrt(L) * scal[2] * lk(0, codes[0])
        assert H == pytest.approx(H_ref, rel=1e-12, abs=1e-12)
        assert T == pytest.approx(O.threshold(Ar, scal[1], scal[2], L, m, 0.1), rel=1e-12)
        assert ok == (H >= T)
        n_h += 1
    assert n_h > 50


# ---------------------------------------------------------------------------
# P5: A_r algebra
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("metric", [W.L2, W.ANGULAR, W.IP])
def test_A_r_literal_equals_distance_form_and_is_exact_cosine_threshold(metric):
    rng = np.random.default_rng(13 + metric)
    L, m, d = 4, 16, 32
    A, B = W.make_directions(L, m, d, 13)
    n_checked = 0
    for _ in range(2000):
        xv, xu, xp, q = rng.standard_normal((4, d)) * rng.uniform(0.3, 3, size=(4, 1))
        if metric == W.ANGULAR:
            xv, xu, xp = [x / np.linalg.norm(x) for x in (xv, xu, xp)]
        xv, xu, xp, q = [x.astype(np.float32).astype(np.float64) for x in (xv, xu, xp, q)]
        ok, Ar, H, T, kind = O.test_edge(xv, xu, xp, q, L, m, A, B, metric, 0.1)
        e = xu - xv
        if metric == W.L2:
            dist = lambda x: ((x - q) ** 2).sum()
            num = 0.5 * (xu @ xu - xv @ xv) + 0.5 * (dist(xv) - dist(xp))
            Aref = num / (np.linalg.norm(q) * np.linalg.norm(e))
        elif metric == W.IP:
            # appendix (Extension to MIPS): (p.q - v.q) / (|q| |e|), p the
            # result of smallest inner product
            dist = lambda x: -(x @ q)
            Aref = (xp @ q - xv @ q) / (np.linalg.norm(q) * np.linalg.norm(e))
        else:
            dist = lambda x: 1 - x @ q / np.linalg.norm(q)
            Aref = (dist(xv) - dist(xp)) / np.linalg.norm(e)
        assert Ar == pytest.approx(Aref, rel=1e-10, abs=1e-12)
        cos = e @ q / (np.linalg.norm(e) * np.linalg.norm(q))
        du, delta = dist(xu), dist(xp)
        if abs(du - delta) > 1e-9 * abs(delta) and abs(cos - Ar) > 1e-9:
            assert (du < delta) == (cos > Ar)
            if Ar >= 1:
                assert du >= delta and not ok and kind == 1
            if Ar <= 0:
                assert ok and kind == 2
            n_checked += 1
    assert n_checked > 1500


def test_zero_length_edge_decided_by_sign():
    L, m, d = 4, 16, 32
    A, B = W.make_directions(L, m, d, 14)
    rng = np.random.default_rng(0)
    for _ in range(50):
        xv, xp, q = rng.standard_normal((3, d)).astype(np.float32)
        ok, Ar, H, T, kind = O.test_edge(xv, xv, xp, q, L, m, A, B, W.L2, 0.1)
        dv = ((xv.astype(np.float64) - q) ** 2).sum()
        dp = ((xp.astype(np.float64) - q) ** 2).sum()
        assert kind == 0 and ok == (dv < dp)


# ---------------------------------------------------------------------------
# P1 / P2 / P3 / P4: search
# ---------------------------------------------------------------------------
def _tiny(n=300, d=16, R=8, seed=0, metric=W.L2):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, d)).astype(np.float32)
    q = rng.standard_normal((20, d)).astype(np.float32)
    if metric == W.ANGULAR:
        x /= np.linalg.norm(x, axis=1, keepdims=True)
    g, entry = W.build_graph(x, R, 2 * R)
    return x, q, g, entry


@pytest.mark.parametrize("metric", [W.L2, W.ANGULAR, W.IP])
def test_brute_force_matches_cdist(metric):
    rng = np.random.default_rng(1)
    x = rng.standard_normal((500, 12))
    q = rng.standard_normal((30, 12))
    if metric == W.ANGULAR:
        x /= np.linalg.norm(x, axis=1, keepdims=True)  # the angular metric takes unit base vectors
    ids, dd = O.brute_force(x, q, 7, metric)
    if metric == W.L2:
        full = cdist(q, x, "sqeuclidean")
    elif metric == W.IP:
        # -x.q = (cosine distance - 1) |q| |x|
        full = ((cdist(q, x, "cosine") - 1.0) * np.linalg.norm(q, axis=1)[:, None]
                * np.linalg.norm(x, axis=1)[None, :])
    else:
        full = cdist(q, x, "cosine")  # 1 - cos
    for i in range(len(q)):
        order = sorted(range(len(x)), key=lambda j: (full[i, j], j))[:7]
        assert list(ids[i]) == order
        np.testing.assert_allclose(dd[i], full[i, order], rtol=1e-12, atol=1e-11)


@pytest.mark.parametrize("metric", [W.L2, W.ANGULAR, W.IP])
@pytest.mark.parametrize("mode", [O.MODE_EXHAUSTIVE, O.MODE_PEOS])
def test_search_with_list_larger_than_n_is_exact_knn(metric, mode):
    """With ef >= n the list never fills, no test runs, every reachable node
    is visited: the search returns exact k-NN (the graph is connected)."""
    x, q, g, entry = _tiny(metric=metric)
    L, m = 4, 16
    A, B = W.make_directions(L, m, x.shape[1], 15)
    out = O.search(x, g, entry, q, 10, x.shape[0], L, m, A, B, metric, 0.1, mode=mode)
    ids, dd = O.brute_force(x, q, 10, metric)
    assert np.array_equal(out["ids"], ids)
    np.testing.assert_allclose(out["dist"], dd, rtol=1e-12, atol=1e-12)
    c = out["counters"]
    assert np.all(c[:, O.COUNTERS.index("ndist")] == x.shape[0])
    assert np.all(c[:, O.COUNTERS.index("expansions")] == x.shape[0])
    assert np.all(c[:, O.COUNTERS.index("edges")] == (g >= 0).sum())
    assert np.all(c[:, O.COUNTERS.index("tests")] == 0)


@pytest.mark.parametrize("metric", [W.L2, W.ANGULAR, W.IP])
def test_vanishing_eps_reproduces_exhaustive_search(metric):
    """eps -> 0+ leaves only the exact prune A_r >= 1 (which implies
    dist(u) >= delta): same ids and distances as exhaustive search, fewer
    distance computations."""
    w = W.TINY.with_sizes(n=1000, nq=40)
    x, q = W.make_base(w), W.make_queries(w)
    if metric == W.ANGULAR:
        x /= np.linalg.norm(x, axis=1, keepdims=True)
    else:
        # put the origin next to the first query: the l2 form of A_r divides
        # by |q|, so a short query makes the exact prune A_r >= 1 fire
        o = q[0] - 0.01
        x, q = (x - o).astype(np.float32), (q - o).astype(np.float32)
    g, entry = W.build_graph(x, w.R, w.cand)
    A, B = W.directions_for(w)
    ex = O.search(x, g, entry, q, 10, 16, w.L, w.m, A, B, metric, 0.1, mode=O.MODE_EXHAUSTIVE)
    pe = O.search(x, g, entry, q, 10, 16, w.L, w.m, A, B, metric, 1e-300, mode=O.MODE_PEOS)
    assert np.array_equal(ex["ids"], pe["ids"])
    np.testing.assert_array_equal(ex["dist"], pe["dist"])
    ci = O.COUNTERS.index
    assert np.all(pe["counters"][:, ci("ndist")] <= ex["counters"][:, ci("ndist")])
    assert pe["counters"][:, ci("test_ge1")].sum() > 0
    # every H-vs-T test passes when the quantile goes to -infinity (no
    # zero-length edges occur in this continuous data)
    c = pe["counters"]
    assert np.all(c[:, ci("test_zero")] == 0)
    assert np.all(c[:, ci("passes")] == c[:, ci("test_h")] + c[:, ci("test_le0")])


@pytest.mark.parametrize("precision", [64, 32])
@pytest.mark.parametrize("pool_mul", [0, 1])
def test_inner_product_search_scales_with_the_query(precision, pool_mul):
    """Inner product (appendix, Extension to MIPS): multiplying q by 8 (exact
    in binary floating point) multiplies every distance p.q, v.q by 8 and |q|
    by 8, so A_r = (p.q - v.q)/(|q||e|) and q/|q| are unchanged: the same
    path, counters and ids, distances times 8.  A test without |q| in the
    denominator of A_r would see 8 times larger A_r and prune differently."""
    w = W.TINY.with_sizes(n=1500, nq=40)
    x, q = W.make_base(w), W.make_queries(w)
    g, entry = W.build_graph(x, w.R, w.cand)
    A, B = W.directions_for(w)
    kw = dict(pool=pool_mul * 32, precision=precision)
    a = O.search(x, g, entry, q, 10, 32, w.L, w.m, A, B, W.IP, 0.1, **kw)
    b = O.search(x, g, entry, (8.0 * q).astype(np.float32), 10, 32, w.L, w.m, A, B, W.IP, 0.1,
                 **kw)
    assert np.array_equal(a["ids"], b["ids"])
    assert np.array_equal(a["counters"], b["counters"])
    np.testing.assert_array_equal(8.0 * a["dist"], b["dist"])
    ci = O.COUNTERS.index
    if pool_mul == 0:
        # the unbounded queue expands nodes outside the list: real tests run
        assert a["counters"][:, ci("test_h")].sum() > 0


def test_inner_product_on_unit_vectors_is_angular():
    """On unit-norm base vectors and queries, -x.q = (1 - x.q/|q|) - 1: the
    inner-product search takes the angular search's path (same ids and
    counters away from near ties) with distances shifted by one."""
    w = W.TINY.with_sizes(n=1500, nq=40)
    x, q = W.make_base(w), W.make_queries(w)
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    q = (q / np.linalg.norm(q, axis=1, keepdims=True)).astype(np.float32)
    g, entry = W.build_graph(x, w.R, w.cand)
    A, B = W.directions_for(w)
    ang = O.search(x, g, entry, q, 10, 32, w.L, w.m, A, B, W.ANGULAR, 0.1)
    ip = O.search(x, g, entry, q, 10, 32, w.L, w.m, A, B, W.IP, 0.1)
    clean = (ang["fragile"] == 0) & (ip["fragile"] == 0)
    assert clean.sum() >= 0.5 * len(q)
    assert np.array_equal(ang["ids"][clean], ip["ids"][clean])
    assert np.array_equal(ang["counters"][clean], ip["counters"][clean])
    # |q| is one only to single precision (the stored query is float32)
    np.testing.assert_allclose(ip["dist"][clean], ang["dist"][clean] - 1.0, rtol=0, atol=1e-6)


def _two_heap_search(x, g, entry, q, k, ef, L, m, A, B, metric, eps, mode):
    """HNSW-style formulation: candidate min-heap C, result max-heap W; same
    delta snapshot per expansion and the same insertion rule."""
    x64 = x.astype(np.float64)
    q64 = q.astype(np.float64)

    def dist(i):
        if metric == W.L2:
            return float(((x64[i] - q64) ** 2).sum())
        return float(1 - x64[i] @ q64 / np.linalg.norm(q64))

    ef = max(ef, k)
    d0 = dist(entry)
    C = [(d0, entry)]
    Wh = [(-d0, -entry)]  # max-heap on (dist, id)
    visited = {entry}
    expansions, ndist = 0, 1
    while C:
        c = heapq.heappop(C)
        worst = (-Wh[0][0], -Wh[0][1])
        if len(Wh) >= ef and c > worst:
            break
        expansions += 1
        full = len(Wh) == ef
        delta = worst[0] if full else math.inf
        p = worst[1]
        S = []
        for u in g[c[1]]:
            if u < 0 or u in visited:
                continue
            ok = True
            if full and mode == O.MODE_PEOS:
                ok = O.test_edge(x[c[1]], x[u], x[p], q, L, m, A, B, metric, eps)[0]
            if not ok:
                continue
            visited.add(u)
            ndist += 1
            du = dist(u)
            if not full or du < delta:
                S.append((du, int(u)))
        for s in S:
            heapq.heappush(C, s)
            heapq.heappush(Wh, (-s[0], -s[1]))
            if len(Wh) > ef:
                heapq.heappop(Wh)
    res = sorted((-a, -b) for a, b in Wh)[:k]
    return [r[1] for r in res], [r[0] for r in res], expansions, ndist


@pytest.mark.parametrize("mode", [O.MODE_EXHAUSTIVE, O.MODE_PEOS])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_single_list_with_pool_ef_equals_two_heap(mode, seed):
    x, q, g, entry = _tiny(n=250, d=8, R=6, seed=seed)
    L, m = 2, 8
    A, B = W.make_directions(L, m, 8, 16 + seed)
    ef = [6, 10, 20][seed]
    out = O.search(x, g, entry, q, 5, ef, L, m, A, B, W.L2, 0.2, mode=mode, pool=ef)
    for i in range(len(q)):
        ids, dd, nexp, nd = _two_heap_search(x, g, entry, q[i], 5, ef, L, m, A, B, W.L2, 0.2, mode)
        assert list(out["ids"][i][:len(ids)]) == ids
        np.testing.assert_allclose(out["dist"][i][:len(ids)], dd, rtol=1e-12)
        assert out["counters"][i, O.COUNTERS.index("expansions")] == nexp
        assert out["counters"][i, O.COUNTERS.index("ndist")] == nd


def test_padding_and_k_above_ef():
    """k > ef uses ef := k; fewer reachable nodes than k pads with (-1, inf)."""
    x = np.random.default_rng(0).standard_normal((6, 8)).astype(np.float32)
    g = np.full((6, 4), -1, np.int32)
    g[0, :2] = [1, 2]
    g[1, 0] = 0
    q = np.ones((1, 8), np.float32)
    out = O.search(x, g, 0, q, 5, 2, 2, 8, np.zeros((2, 8, 4), np.float32),
                   np.zeros((8, 8), np.float32), W.L2, 0.1, mode=O.MODE_EXHAUSTIVE)
    assert sorted(out["ids"][0][:3]) == [0, 1, 2]
    assert list(out["ids"][0][3:]) == [-1, -1] and np.all(np.isinf(out["dist"][0][3:]))


def test_zero_query_status():
    x = np.random.default_rng(0).standard_normal((10, 8)).astype(np.float32)
    g = np.zeros((10, 2), np.int32) - 1
    out = O.search(x, g, 0, np.zeros((1, 8), np.float32), 1, 4, 2, 8, None, None, W.L2, 0.1)
    assert out["status"][0] == -1 and out["ids"][0, 0] == -1


def _literal_alg1(x, g, entry, q, k, ef, L, m, A, B, metric, eps, mode, pool=None):
    """Alg. 1 as printed: result list R (best ef so far) and priority queue P
    holding every pushed node until it is popped; the loop runs until P is
    empty.  With `pool`, P keeps at most pool - |R| entries that are not in R
    (the worst are dropped).  Same delta snapshot per expansion."""
    x64, q64 = x.astype(np.float64), q.astype(np.float64)

    def dist(i):
        if metric == W.L2:
            return float(((x64[i] - q64) ** 2).sum())
        return float(1 - x64[i] @ q64 / np.linalg.norm(q64))

    ef = max(ef, k)
    Rl = [(dist(entry), entry)]
    P = [(dist(entry), entry)]
    visited = {entry}
    expansions, ndist = 0, 1
    while P:
        c = heapq.heappop(P)
        expansions += 1
        full = len(Rl) == ef
        delta, p = (Rl[-1] if full else (math.inf, -1))
        S = []
        for u in g[c[1]]:
            if u < 0 or u in visited:
                continue
            ok = True
            if full and mode == O.MODE_PEOS:
                ok = O.test_edge(x[c[1]], x[u], x[p], q, L, m, A, B, metric, eps)[0]
            if not ok:
                continue
            visited.add(u)
            ndist += 1
            du = dist(u)
            if not full or du < delta:
                S.append((du, int(u)))
        for s_ in S:
            heapq.heappush(P, s_)
        Rl = sorted(Rl + S)[:ef]
        if pool is not None:
            rs = set(Rl)
            outside = sorted(e for e in P if e not in rs)
            keep_out = max(0, pool - len(Rl))
            P = [e for e in P if e in rs] + outside[:keep_out]
            heapq.heapify(P)
    return [r[1] for r in Rl[:k]], [r[0] for r in Rl[:k]], expansions, ndist


@pytest.mark.parametrize("mode", [O.MODE_EXHAUSTIVE, O.MODE_PEOS])
@pytest.mark.parametrize("pool_mul", [0, 2, 3])
@pytest.mark.parametrize("seed", [0, 1])
def test_single_list_equals_literal_alg1(mode, pool_mul, seed):
    """The one-list form with an unbounded pool is Alg. 1 as printed (R plus
    a priority queue emptied to the end); a bounded pool matches Alg. 1 whose
    queue keeps only the best pool - |R| nodes outside R."""
    x, q, g, entry = _tiny(n=250, d=8, R=6, seed=10 + seed)
    L, m = 2, 8
    A, B = W.make_directions(L, m, 8, 40 + seed)
    ef = [6, 12][seed]
    pool = pool_mul * ef
    out = O.search(x, g, entry, q, 5, ef, L, m, A, B, W.L2, 0.2, mode=mode, pool=pool)
    for i in range(len(q)):
        ids, dd, nexp, nd = _literal_alg1(x, g, entry, q[i], 5, ef, L, m, A, B, W.L2, 0.2, mode,
                                          pool=pool if pool else None)
        assert list(out["ids"][i][:len(ids)]) == ids
        np.testing.assert_allclose(out["dist"][i][:len(ids)], dd, rtol=1e-12)
        assert out["counters"][i, O.COUNTERS.index("expansions")] == nexp
        assert out["counters"][i, O.COUNTERS.index("ndist")] == nd


@pytest.mark.parametrize("mode", [O.MODE_EXHAUSTIVE, O.MODE_PEOS])
@pytest.mark.parametrize("pool_mul", [0, 1])
def test_integer_data_ties_follow_strict_insertion(mode, pool_mul):
    """Small-integer data makes equal distances common: ties are broken by
    id, and a neighbour at exactly delta is not inserted (strict <)."""
    rng = np.random.default_rng(77)
    x = rng.integers(0, 4, size=(300, 8)).astype(np.float32)
    q = rng.integers(0, 4, size=(25, 8)).astype(np.float32)
    g, entry = W.build_graph(x, 6, 12)
    L, m = 2, 8
    A, B = W.make_directions(L, m, 8, 99)
    ef = 8
    out = O.search(x, g, entry, q, 5, ef, L, m, A, B, W.L2, 0.2, mode=mode, pool=pool_mul * ef)
    ties = 0
    for i in range(len(q)):
        ids, dd, nexp, nd = _literal_alg1(x, g, entry, q[i], 5, ef, L, m, A, B, W.L2, 0.2, mode,
                                          pool=pool_mul * ef if pool_mul else None)
        assert list(out["ids"][i][:len(ids)]) == ids
        assert out["counters"][i, O.COUNTERS.index("expansions")] == nexp
        assert out["counters"][i, O.COUNTERS.index("ndist")] == nd
        ties += len(dd) - len(set(dd))
    assert ties > 0


# ---------------------------------------------------------------------------
# the single-precision distance decisions (the GPU kernel's precision)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("metric", [W.L2, W.ANGULAR, W.IP])
def test_fp32_distances_within_rounding_bound(metric):
    w = W.TINY.with_sizes(n=1500, nq=40)
    x, q = W.make_base(w), W.make_queries(w)
    if metric == W.ANGULAR:
        x /= np.linalg.norm(x, axis=1, keepdims=True)
    g, entry = W.build_graph(x, w.R, w.cand)
    A, B = W.directions_for(w)
    out = O.search(x, g, entry, q, 10, 32, w.L, w.m, A, B, metric, 0.1, precision=32)
    d32, d64 = out["dist"], out["dist64"]
    assert np.all(d32 == d32.astype(np.float32))   # values are single precision
    u = 2.0 ** -24
    if metric == W.L2:
        assert np.all(np.abs(d32 - d64) <= (w.d + 2) * u * d64)
    elif metric == W.IP:
        # a dot product of d terms: (d + 2) u sum |x_k q_k| <= (d + 2) u |x||q|
        scale = (np.linalg.norm(x.astype(np.float64), axis=1)[out["ids"]]
                 * np.linalg.norm(q.astype(np.float64), axis=1)[:, None])
        assert np.all(np.abs(d32 - d64) <= (w.d + 2) * u * scale)
        return
    else:
        assert np.all(np.abs(d32 - d64) <= (w.d + 4) * u)
    # and far inside the 1e-5 relative tolerance of the GPU parity
    assert np.all(np.abs(d32 - d64) <= 1e-5 * np.abs(d64) + 1e-6)


@pytest.mark.parametrize("metric", [W.L2, W.ANGULAR, W.IP])
@pytest.mark.parametrize("pool_mul", [0, 1])
def test_fp32_decisions_equal_fp64_away_from_near_ties(metric, pool_mul):
    """Single-precision distance decisions change nothing unless two
    distances (or a distance and delta) are within 1e-5 relative."""
    w = W.TINY.with_sizes(n=2000, nq=100)
    x, q = W.make_base(w), W.make_queries(w)
    if metric == W.ANGULAR:
        x /= np.linalg.norm(x, axis=1, keepdims=True)
    g, entry = W.build_graph(x, w.R, w.cand)
    A, B = W.directions_for(w)
    kw = dict(pool=pool_mul * 32)
    o64 = O.search(x, g, entry, q, 10, 32, w.L, w.m, A, B, metric, 0.1, precision=64, **kw)
    o32 = O.search(x, g, entry, q, 10, 32, w.L, w.m, A, B, metric, 0.1, precision=32, **kw)
    clean = (o64["fragile"] & (O.F_DELTA | O.F_ORDER)) == 0
    # observed: 69-82% of the queries clean on these workloads, and the two
    # precisions agree on every query (clean or not)
    assert clean.sum() >= 0.65 * len(q)
    assert np.array_equal(o64["ids"][clean], o32["ids"][clean])
    assert np.array_equal(o64["counters"][clean], o32["counters"][clean])
    np.testing.assert_allclose(o32["dist64"][clean], o64["dist"][clean], rtol=0, atol=0)
    assert np.mean(np.all(o64["ids"] == o32["ids"], axis=1)) >= 0.97


@pytest.mark.parametrize("metric", [W.L2, W.IP])
@pytest.mark.parametrize("pool_mul", [0, 1])
def test_integer_data_decisions_do_not_depend_on_precision(metric, pool_mul):
    """On integer-valued vectors with squared norms and distances below 2^22
    every distance, delta and A_r numerator is an integer (or half-integer)
    that single precision computes exactly in any order, so the search's
    distance decisions and the sign of A_r cannot depend on the precision:
    none of them is flagged, and the single- and double-precision searches are
    identical on every query (ids, distances, counters)."""
    w = W.SIFT_LIKE.with_sizes(n=6000, nq=60)
    x, q = W.make_base(w), W.make_queries(w)
    assert np.all(x == np.floor(x)) and (x.astype(np.float64) ** 2).sum(1).max() < 2 ** 22
    g, entry = W.build_graph(x, w.R, w.cand)
    A, B = W.directions_for(w)
    kw = dict(pool=pool_mul * 48)
    o64 = O.search(x, g, entry, q, 10, 48, w.L, w.m, A, B, metric, 0.2, precision=64, **kw)
    o32 = O.search(x, g, entry, q, 10, 48, w.L, w.m, A, B, metric, 0.2, precision=32, **kw)
    assert np.all(o64["fragile"] & (O.F_DELTA | O.F_ORDER | O.F_A0) == 0)
    assert np.array_equal(o64["ids"], o32["ids"])
    assert np.array_equal(o64["counters"], o32["counters"])
    assert np.array_equal(o64["dist"], o32["dist"])
    # the same data shifted by 1/3 is not integer-valued: near ties are flagged again
    xs, qs = x + np.float32(1 / 3), q + np.float32(1 / 3)
    o64s = O.search(xs, g, entry, qs, 10, 48, w.L, w.m, A, B, metric, 0.2, precision=64, **kw)
    if metric == W.L2:
        assert np.any(o64s["fragile"] & (O.F_DELTA | O.F_ORDER))


# ---------------------------------------------------------------------------
# the precision form: storage roundings, bfloat16 traversal + re-rank, half
# tables and scalars
# ---------------------------------------------------------------------------
def test_round_half_matches_ieee_binary16():
    """Against numpy's conversion of doubles to IEEE half (round to nearest
    even), over normal, subnormal, tie and overflow values."""
    rng = np.random.default_rng(0)
    xs = np.concatenate([
        rng.normal(size=2000) * 10.0 ** rng.uniform(-9, 5, size=2000),
        [0.0, -0.0, 1.0, 65504.0, 65519.99, 65520.0, 1e6, 2.0 ** -24, 2.0 ** -25,
         3 * 2.0 ** -26, 2.0 ** -14, (1 + 2.0 ** -11), (1 + 3 * 2.0 ** -11), -(1 + 2.0 ** -11)],
    ])
    for x in xs:
        with np.errstate(over="ignore"):
            ref = float(np.float16(np.float64(x)))
        got = O.round_half(x)
        assert got == ref or (math.isinf(got) and math.isinf(ref) and got == ref), x


def test_round_bf16_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    xs = (rng.normal(size=3000) * 10.0 ** rng.uniform(-30, 30, size=3000)).astype(np.float32)
    xs = np.concatenate([xs, np.float32([1.00390625, 1.01171875, -1.00390625, 3.0, 0.0])])
    ref = torch.from_numpy(xs).to(torch.bfloat16).to(torch.float32).numpy()
    got = np.array([O.round_bf16(v) for v in xs], np.float32)
    assert np.array_equal(got, ref)


def _tiny_case(metric, n=1500, nq=50):
    w = W.TINY.with_sizes(n=n, nq=nq)
    x, q = W.make_base(w), W.make_queries(w)
    if metric == W.ANGULAR:
        x /= np.linalg.norm(x, axis=1, keepdims=True)
    g, entry = W.build_graph(x, w.R, w.cand)
    A, B = W.directions_for(w)
    return w, x, q, g, entry, A, B


@pytest.mark.parametrize("mode", [O.MODE_PEOS, O.MODE_EXHAUSTIVE])
def test_bf16_traversal_on_bf16_exact_data_equals_fp32(mode):
    """Integer data in 0..255 is exact in bfloat16: the bfloat16 traversal
    and its re-rank change nothing."""
    w = W.SIFT_LIKE.with_sizes(n=3000, nq=40)
    x, q = W.make_base(w), W.make_queries(w)
    g, entry = W.build_graph(x, w.R, w.cand)
    A, B = W.directions_for(w)
    a = O.search(x, g, entry, q, 10, 32, w.L, w.m, A, B, w.metric, 0.1, mode=mode, precision=32)
    b = O.search(x, g, entry, q, 10, 32, w.L, w.m, A, B, w.metric, 0.1, mode=mode,
                 lowp=O.LP_BF16_BASE)
    assert np.array_equal(a["ids"], b["ids"]) and np.array_equal(a["dist"], b["dist"])
    assert np.array_equal(a["counters"], b["counters"])


@pytest.mark.parametrize("metric", [W.L2, W.ANGULAR, W.IP])
def test_bf16_rerank_returns_full_precision_order(metric):
    """The bfloat16 traversal's output is re-ranked on the full base: the
    returned distances are the single-precision distances of the returned
    ids, ascending, within the single-precision bound of float64."""
    w, x, q, g, entry, A, B = _tiny_case(metric)
    out = O.search(x, g, entry, q, 10, 32, w.L, w.m, A, B, metric, 0.1, lowp=O.LP_BF16_BASE)
    d, d64 = out["dist"], out["dist64"]
    assert np.all(np.diff(d, axis=1) >= 0)
    u = 2.0 ** -24
    if metric == W.L2:
        assert np.all(np.abs(d - d64) <= (w.d + 2) * u * d64)
    elif metric == W.IP:
        scale = (np.linalg.norm(x.astype(np.float64), axis=1)[out["ids"]]
                 * np.linalg.norm(q.astype(np.float64), axis=1)[:, None])
        assert np.all(np.abs(d - d64) <= (w.d + 2) * u * scale)
    else:
        assert np.all(np.abs(d - d64) <= (w.d + 4) * u)
    # recall is essentially unchanged by the bfloat16 traversal
    ref = O.search(x, g, entry, q, 10, 32, w.L, w.m, A, B, metric, 0.1, precision=32)
    gt, _ = O.brute_force(x, q, 10, metric)
    r_lo = np.mean([len(set(out["ids"][i]) & set(gt[i])) for i in range(len(q))]) / 10
    r_hi = np.mean([len(set(ref["ids"][i]) & set(gt[i])) for i in range(len(q))]) / 10
    assert r_lo >= r_hi - 0.02


@pytest.mark.parametrize("metric", [W.L2, W.ANGULAR, W.IP])
def test_half_test_within_rounding_bound_of_exact_test(metric):
    """The precision-form test (half scalars and table) differs from the
    exact test only by the half rounding: |A' - A| and |H' - H| stay within
    the bound that 2^-11 relative errors of each stored value give, and the
    decision is the same whenever the exact margins exceed that bound."""
    rng = np.random.default_rng(3)
    d, L, m = 32, 4, 16
    A_, B_ = W.make_directions(L, m, d, 5)
    agree = checked = 0
    for _ in range(400):
        xv, xu, xp, q = (rng.normal(size=d).astype(np.float32) for _ in range(4))
        xu = (xv + 0.4 * (xu - xv)).astype(np.float32)
        if metric == W.ANGULAR:
            xv, xu, xp = (v / np.linalg.norm(v) for v in (xv, xu, xp))
            xv, xu, xp = (v.astype(np.float32) for v in (xv, xu, xp))
        p0, A0, H0, T0, k0 = O.test_edge(xv, xu, xp, q, L, m, A_, B_, metric, 0.1)
        p1, A1, H1, T1, k1 = O.test_edge(xv, xu, xp, q, L, m, A_, B_, metric, 0.1,
                                         lowp=O.LP_FP16)
        u = 2.0 ** -11
        e = xu.astype(np.float64) - xv
        ne = np.linalg.norm(e)
        qn = np.linalg.norm(q.astype(np.float64))
        if metric == W.L2:
            g = 0.5 * (np.dot(xu, xu) - np.dot(xv, xv)) / ne
            num_scale = (abs(g) + abs(A0 * qn - g)) / qn
        else:
            num_scale = abs(A0)
        # A' = (g' + diff ie') / |q|: each stored factor off by <= 2^-11
        # relative, the distances by single-precision rounding
        bA = 3 * u * num_scale + 1e-5 * (1 + abs(A0))
        assert abs(A1 - A0) <= bA
        if k0 == 3 and k1 == 3:
            t = O.query_table(q, L, m, A_, B_)
            bH = 3 * u * (np.abs(t).sum() * 2.0)
            assert abs(H1 - H0) <= bH
            bT = abs(T0 - T1)
            if abs(H0 - T0) > bH + 6.6 * bA + 3 * u * abs(T0) + bT:
                checked += 1
                agree += p0 == p1
        elif k0 != 3 and abs(A0) > bA and abs(A0 - 1) > bA:
            checked += 1
            agree += p0 == p1
    assert checked > 100 and agree == checked


def test_half_search_mostly_equals_exact_decisions():
    """Search with half-rounded scalars and tables (same traversal distances):
    most queries take the same path as with exact values; the rest differ
    only where a decision margin is within the rounding."""
    w, x, q, g, entry, A, B = _tiny_case(W.L2, n=2000, nq=100)
    a = O.search(x, g, entry, q, 10, 32, w.L, w.m, A, B, w.metric, 0.1, precision=32)
    b = O.search(x, g, entry, q, 10, 32, w.L, w.m, A, B, w.metric, 0.1, lowp=O.LP_FP16)
    same = np.all(a["ids"] == b["ids"], axis=1) & np.all(a["counters"] == b["counters"], axis=1)
    assert same.mean() >= 0.8
    assert np.array_equal(a["counters"][:, 0] > 0, b["counters"][:, 0] > 0)


@pytest.mark.parametrize("mult", [1, 2, 3])
def test_pool_multiple_of_ef_equals_fixed_pool(mult):
    """pool = -m (a queue of m x each query's ef) equals pool = m x ef when all
    queries share ef, and pool = -1 is the HNSW stopping rule."""
    w = W.TINY.with_sizes(n=1500, nq=40)
    x, q = W.make_base(w), W.make_queries(w)
    g, entry = W.build_graph(x, w.R, w.cand)
    A, B = W.directions_for(w)
    a = O.search(x, g, entry, q, 10, 24, w.L, w.m, A, B, w.metric, 0.1, pool=-mult)
    b = O.search(x, g, entry, q, 10, 24, w.L, w.m, A, B, w.metric, 0.1, pool=mult * 24)
    assert np.array_equal(a["ids"], b["ids"]) and np.array_equal(a["counters"], b["counters"])


# ---------------------------------------------------------------------------
# optional dimension permutation (appendix "Dimension Permutation")
# ---------------------------------------------------------------------------
def test_dimension_permutation_worked_example():
    """d = 4, L = 2, one edge with squared coordinates (4, 1, 3, 2): ascending
    order 1, 3, 2, 0; round 1: dim 1 -> S1 (both sums 0, first set), dim 3 ->
    S2; round 2: dim 2 -> S2 (larger sum 2), dim 0 -> S1; sums 5 and 5."""
    x = np.array([[0, 0, 0, 0], [2, 1, np.sqrt(3), np.sqrt(2)]], np.float32)
    g = np.array([[1], [-1]], np.int32)
    perm, avg = O.dimension_permutation(x, g, 2)
    np.testing.assert_allclose(avg, [4, 1, 3, 2], rtol=1e-6)
    assert perm.tolist() == [1, 0, 3, 2]


def test_dimension_permutation_is_balanced_partition():
    """A valid permutation, d/L dimensions per subspace, and subspace energies
    no less balanced than the identity split (on strongly anisotropic data)."""
    rng = np.random.default_rng(4)
    d, L = 64, 8
    scale = np.exp(rng.normal(0, 1.0, size=d))
    x = (rng.normal(size=(600, d)) * scale).astype(np.float32)
    g, _ = W.build_graph(x, 12, 24)
    perm, avg = O.dimension_permutation(x, g, L)
    assert sorted(perm.tolist()) == list(range(d))
    dp = d // L
    e_perm = avg[perm].reshape(L, dp).sum(1)
    e_id = avg.reshape(L, dp).sum(1)
    assert e_perm.max() - e_perm.min() <= e_id.max() - e_id.min()
    # every round hands out one dimension per subspace, in ascending Avg
    order = np.lexsort((np.arange(d), avg))
    for t in range(dp):
        assert sorted(perm.reshape(L, dp)[:, t].tolist()) == sorted(order[t * L:(t + 1) * L].tolist())
    # the spread is at most the largest single Avg (greedy balancing bound)
    assert e_perm.max() - e_perm.min() <= avg.max() + 1e-12


def test_permuted_test_equals_permuted_directions():
    """Permuting coordinates inside each block is the same as permuting the
    projection vectors' coordinates the other way: the search with such a
    permutation equals the unpermuted search with permuted directions."""
    w = W.TINY.with_sizes(n=1500, nq=40)
    x, q = W.make_base(w), W.make_queries(w)
    g, entry = W.build_graph(x, w.R, w.cand)
    A, B = W.directions_for(w)
    d, L = w.d, w.L
    dp = d // L
    rng = np.random.default_rng(9)
    perm = np.concatenate([i * dp + rng.permutation(dp) for i in range(L)]).astype(np.int32)
    inv = np.argsort(perm)
    # direction coordinate t of block i pairs with original coordinate perm[i*dp+t]
    A2 = np.empty_like(A)
    for i in range(L):
        A2[i][:, perm[i * dp:(i + 1) * dp] - i * dp] = A[i]
    B2 = B[:, inv]
    a = O.search(x, g, entry, q, 10, 32, L, w.m, A, B, w.metric, 0.1, perm=perm, precision=32)
    b = O.search(x, g, entry, q, 10, 32, L, w.m, A2, B2, w.metric, 0.1, precision=32)
    same = (a["fragile"] == 0) & (b["fragile"] == 0)
    assert same.mean() > 0.8
    assert np.array_equal(a["ids"][same], b["ids"][same])
    assert np.array_equal(a["counters"][same], b["counters"][same])


# ---------------------------------------------------------------------------
# SimHash test (Sec. 3 "SimHash Test", residual-edge remedy)
# ---------------------------------------------------------------------------
def test_simhash_collision_rate_is_one_minus_angle_over_pi():
    """The lemma: a random Gaussian direction separates two vectors at angle
    theta with probability theta/pi."""
    rng = np.random.default_rng(2)
    d = 48
    u = rng.normal(size=d)
    for theta in (0.3, 1.0, 2.0):
        w = rng.normal(size=d)
        w -= w.dot(u) / u.dot(u) * u
        q = np.cos(theta) * u / np.linalg.norm(u) + np.sin(theta) * w / np.linalg.norm(w)
        cols = []
        for rep in range(300):
            C = rng.normal(size=(64, d)).astype(np.float32)
            bu = O.simhash_bits(u, C)[0]
            bq = O.simhash_bits(q, C)[0]
            cols.append(64 - bin(int(bu) ^ int(bq)).count("1"))
        frac = np.mean(cols) / 64
        assert abs(frac - (1 - theta / np.pi)) < 4 * np.sqrt(0.25 / (64 * 300))


@pytest.mark.parametrize("eps", [0.1, 0.2])
def test_simhash_test_guarantee(eps):
    """Edges with cos(e, q) above A_r (so d_u < delta) pass with probability
    at least 1 - eps (Hoeffding's bound is conservative), and edges at
    cos(e, q) far below A_r mostly fail."""
    rng = np.random.default_rng(8)
    d, nb = 32, 64
    A_, B_ = W.make_directions(4, 16, d, 5)
    good = bad = ngood = nbad = 0
    for _ in range(3000):
        C = rng.normal(size=(nb, d)).astype(np.float32)
        xv, xp, q = (rng.normal(size=d).astype(np.float32) for _ in range(3))
        xu = (xv + rng.normal(size=d)).astype(np.float32)
        p, A, col, T, kind = O.test_edge(xv, xu, xp, q, 4, 16, A_, B_, W.L2, eps, simhash=C)
        if kind != 3:
            continue
        e = xu.astype(np.float64) - xv
        cos = e.dot(q) / np.linalg.norm(e) / np.linalg.norm(q)
        if cos > A:
            ngood += 1
            good += p
        elif cos < A - 0.5:
            nbad += 1
            bad += p
    assert ngood > 60 and good / ngood >= 1 - eps
    assert nbad > 60 and bad / nbad < 0.5


@pytest.mark.parametrize("metric", [W.L2, W.ANGULAR])
def test_simhash_vanishing_eps_reproduces_exhaustive(metric):
    """As eps -> 0 the Hoeffding margin exceeds nb, only the exact A_r >= 1
    rule prunes, and the search returns the exhaustive search's results."""
    w = W.TINY.with_sizes(n=1500, nq=40)
    x, q = W.make_base(w), W.make_queries(w)
    if metric == W.ANGULAR:
        x /= np.linalg.norm(x, axis=1, keepdims=True)
    g, entry = W.build_graph(x, w.R, w.cand)
    A, B = W.directions_for(w)
    C = np.random.default_rng(3).normal(size=(64, w.d)).astype(np.float32)
    a = O.search(x, g, entry, q, 10, 32, w.L, w.m, A, B, metric, 1e-300, mode=O.MODE_SIMHASH,
                 simhash=C)
    b = O.search(x, g, entry, q, 10, 32, w.L, w.m, A, B, metric, 0.1, mode=O.MODE_EXHAUSTIVE)
    assert np.array_equal(a["ids"], b["ids"])
    assert a["counters"][:, 9].sum() <= b["counters"][:, 9].sum()


# ---------------------------------------------------------------------------
# the compact form (experiments, "Indexing Cost" and "Scalability"): L <= 4,
# w_reg = 1, w_res = 0, 8-bit scalars, quantile table
# ---------------------------------------------------------------------------
def _threshold_w10(A, L, m, eps):
    """T(A) with w_reg = 1, w_res = 0, from scipy's normal quantile."""
    A = np.asarray(A, np.float64)
    return stats.norm.ppf(eps, loc=A * math.sqrt(2 * L * math.log(m)),
                          scale=np.sqrt(1.0 - L * A * A / (L + 1)))


@pytest.mark.parametrize("L,m,eps", [(2, 16, 0.1), (4, 16, 0.2), (1, 128, 0.05), (3, 32, 0.5)])
def test_compact_lut_is_a_conservative_step_of_the_threshold(L, m, eps):
    """Entry b is T(b/256) rounded down to float32; for every A of bin b the
    entry is at most T(A) (T increases with A) and falls short of it by at
    most the rise of T over the bin."""
    lut = O.compact_lut(L, m, eps).astype(np.float64)
    edges = np.arange(O.COMPACT_LUT_BINS) / O.COMPACT_LUT_BINS
    te = _threshold_w10(edges, L, m, eps)
    assert np.all(lut <= te + 1e-12 * np.abs(te) + 1e-15)
    assert np.all(te - lut <= 2.0 ** -22 * np.abs(te) + 1e-15)
    A = np.random.default_rng(L).uniform(0, 1, 20000)
    b = np.floor(A * O.COMPACT_LUT_BINS).astype(int)
    tA = _threshold_w10(A, L, m, eps)
    assert np.all(lut[b] <= tA + 1e-12)
    rise = _threshold_w10((b + 1) / O.COMPACT_LUT_BINS, L, m, eps) - te[b]
    assert np.all(tA - lut[b] <= rise + 2.0 ** -22 * np.abs(te[b]) + 1e-12)


def _compact_case(metric, n=1500):
    w = W.TINY.with_sizes(n=n, nq=40)
    x, q = W.make_base(w), W.make_queries(w)
    if metric == W.ANGULAR:
        x /= np.linalg.norm(x, axis=1, keepdims=True)
    g, entry = W.build_graph(x, w.R, w.cand)
    return w, x, q, g, entry


@pytest.mark.parametrize("metric", [W.L2, W.ANGULAR, W.IP])
def test_compact_codes_decode_within_their_step(metric):
    """Decoded g_e/|e| lies in [exact - g_step, exact] and decoded 1/|e|
    within half an i_step of the exact value (up to the single-precision
    rounding of the values the codes are decided on); the node's ranges are
    the min / max over its edges; a zero-length edge gets code 255."""
    w, x, q, g, entry = _compact_case(metric)
    # a duplicate vector makes one zero-length edge
    u0 = int(g[0, 0])
    x = x.copy()
    x[u0] = x[0]
    L = 2
    hdr, cg, ci = O.compact_tables(x, g, L, metric)
    assert ci[0, 0] == 255
    xs = x.astype(np.float64)
    u = 2.0 ** -24
    nz = 0
    for v in range(0, len(x), 7):
        glo, gstep, ilo, istep = hdr[v].astype(np.float64)
        gps, ies = [], []
        for j, uu in enumerate(g[v]):
            if uu < 0:
                continue
            e = xs[uu] - xs[v]
            ne = np.linalg.norm(e)
            if ne == 0:
                assert ci[v, j] == 255
                continue
            nu2, nv2 = xs[uu] @ xs[uu], xs[v] @ xs[v]
            gp = 0.5 * (nu2 - nv2) / ne if metric == W.L2 else 0.0
            ie = 1.0 / ne
            # single-precision evaluation error of gp and ie
            tg = (w.d + 4) * u * (nu2 + nv2) / ne + 4 * u * abs(gp)
            ti = (w.d + 4) * u * ie
            gh = glo + cg[v, j] * gstep
            ih = ilo + ci[v, j] * istep
            assert gh <= gp + tg + 1e-6 * gstep
            assert gp - gh <= gstep * (1 + 1e-5) + tg
            assert abs(ih - ie) <= 0.5 * istep * (1 + 1e-5) + ti
            gps.append(gp)
            ies.append(ie)
            nz += 1
        if gps:
            assert abs(glo - min(gps)) <= 1e-5 * max(1.0, abs(min(gps)))
            assert abs(glo + 255 * gstep - max(gps)) <= 1e-5 * max(1.0, abs(max(gps)))
            assert abs(ilo - min(ies)) <= 1e-5 * min(ies)
            assert abs(ilo + 254 * istep - max(ies)) <= 1e-5 * max(ies)
    assert nz > 1000


@pytest.mark.parametrize("metric", [W.L2, W.ANGULAR, W.IP])
def test_compact_test_never_overestimates_A_and_passes_what_the_exact_test_passes(metric):
    """With the node's codes, the compact test's A_r is at most the exact
    A_r (scalars unquantized), and the compact test passes every edge that
    the w = (1, 0) test on exact scalars and the exact quantile passes; it
    passes some more (the price of 8-bit scalars and the table)."""
    rng = np.random.default_rng(31 + metric)
    L, m, d, eps = 2, 16, 32, 0.1
    A_, B_ = W.make_directions(L, m, d, 7)
    graph = np.full((9, 8), -1, np.int32)
    graph[0] = np.arange(1, 9)
    extra = checked = 0
    for _ in range(300):
        pts = rng.normal(size=(9, d)) * rng.uniform(0.5, 2.0, size=(9, 1))
        pts[1:] = pts[0] + 0.5 * (pts[1:] - pts[0])
        q = rng.normal(size=d)
        xp = rng.normal(size=d)
        if metric == W.ANGULAR:
            pts /= np.linalg.norm(pts, axis=1, keepdims=True)
            xp /= np.linalg.norm(xp)
        pts, q, xp = (a.astype(np.float32) for a in (pts, q, xp))
        hdr, cg, ci = O.compact_tables(pts, graph, L, metric)
        x64, q64, p64 = pts.astype(np.float64), q.astype(np.float64), xp.astype(np.float64)
        if metric == W.L2:
            dist = lambda y: ((y - q64) ** 2).sum()
        elif metric == W.IP:
            dist = lambda y: -(y @ q64)
        else:
            dist = lambda y: 1.0 - y @ q64 / np.linalg.norm(q64)
        dv, delta = dist(x64[0]), dist(p64)
        table = O.query_table(q, L, m, A_, B_)
        qn = np.linalg.norm(q64)
        for j in range(1, 9):
            codes, _, _ = O.edge_record(pts[0], pts[j], L, m, A_, B_)
            ok, Ac, Hc, Tc, kind = O.compact_test(hdr[0], cg[0, j - 1], ci[0, j - 1], codes, q, L,
                                                  m, A_, B_, metric, eps, dv, delta)
            e = x64[j] - x64[0]
            ne = np.linalg.norm(e)
            if metric == W.L2:
                Aex = (0.5 * (x64[j] @ x64[j] - x64[0] @ x64[0]) + 0.5 * (dv - delta)) / (qn * ne)
            elif metric == W.IP:
                Aex = (dv - delta) / (qn * ne)
            else:
                Aex = (dv - delta) / ne
            assert Ac <= Aex + 1e-6 * (1 + abs(Aex))
            H = sum((-1 if c >= m else 1) * table[i, c % m] for i, c in enumerate(codes) if i >= 1)
            if Aex >= 1:
                ok_ex = False
            elif Aex <= 0:
                ok_ex = True
            else:
                ok_ex = H >= float(_threshold_w10(Aex, L, m, eps))
            if kind == 3:
                assert Hc == pytest.approx(H, rel=1e-12, abs=1e-12)
            if ok_ex:
                assert ok, (Aex, Ac, H, Tc)
            extra += ok and not ok_ex
            checked += 1
    assert checked == 2400 and extra > 0


@pytest.mark.parametrize("metric", [W.L2, W.ANGULAR, W.IP])
def test_compact_vanishing_eps_reproduces_exhaustive_search(metric):
    """eps -> 0+: every table entry goes to -infinity's side, only A_r >= 1
    prunes, and A_r is never overestimated, so the compact search returns
    the exhaustive search's ids and distances with fewer distances."""
    w, x, q, g, entry = _compact_case(metric, n=1000)
    if metric == W.L2:
        o = q[0] - 0.01
        x, q = (x - o).astype(np.float32), (q - o).astype(np.float32)
        g, entry = W.build_graph(x, w.R, w.cand)
    L = 2
    A, B = W.make_directions(L, w.m, w.d, 9)
    ex = O.search(x, g, entry, q, 10, 16, L, w.m, A, B, metric, 0.1, mode=O.MODE_EXHAUSTIVE,
                  precision=32)
    pe = O.search(x, g, entry, q, 10, 16, L, w.m, A, B, metric, 1e-300, lowp=O.LP_COMPACT,
                  precision=32)
    assert np.array_equal(ex["ids"], pe["ids"])
    np.testing.assert_array_equal(ex["dist"], pe["dist"])
    ci = O.COUNTERS.index
    assert np.all(pe["counters"][:, ci("ndist")] <= ex["counters"][:, ci("ndist")])
    assert pe["counters"][:, ci("test_ge1")].sum() > 0


def test_compact_form_needs_L_at_most_4():
    w, x, q, g, entry = _compact_case(W.L2, n=300)
    A, B = W.make_directions(8, w.m, w.d, 9)
    with pytest.raises(ValueError):
        O.search(x, g, entry, q, 10, 16, 8, w.m, A, B, W.L2, 0.1, lowp=O.LP_COMPACT)
    with pytest.raises(ValueError):
        O.compact_tables(x, g, 8, W.L2)


# ---------------------------------------------------------------------------
# entry descent through upper layers (HNSW graphs of the experiments)
# ---------------------------------------------------------------------------
def _dist64(x, q, metric):
    x64, q64 = x.astype(np.float64), q.astype(np.float64)
    if metric == W.L2:
        return ((x64 - q64) ** 2).sum(-1)
    if metric == W.IP:
        return -(x64 @ q64)
    return 1.0 - x64 @ q64 / np.linalg.norm(q64)


@pytest.mark.parametrize("metric", [W.L2, W.ANGULAR, W.IP])
def test_descent_through_a_complete_layer_finds_its_nearest_node(metric):
    """One upper layer whose rows are all linked: one greedy step reaches the
    layer's nearest node to q (distance, then id), the brute-force answer."""
    w, x, q, g, entry = _compact_case(metric, n=600)
    S = np.arange(0, 600, 37)
    k = len(S)
    adj = np.array([[j for j in range(k) if j != i] for i in range(k)], np.int32)
    layers = dict(node=S.astype(np.int32), adj=adj, down=np.full(k, -1, np.int32), top=3)
    ent, nd, frag = O.descend(x, layers, q, metric, precision=64)
    for i in range(len(q)):
        dd = _dist64(x[S], q[i], metric)
        best = S[np.lexsort((S, dd))[0]]
        assert ent[i] == best
        # the start plus one scan from it, plus one scan from the winner if it moved
        assert nd[i] == 1 + (k - 1) * (1 if best == S[3] else 2)


@pytest.mark.parametrize("metric", [W.L2, W.ANGULAR, W.IP])
def test_descent_ends_in_a_local_minimum_of_the_lowest_layer(metric):
    """Built HNSW-style layers: the entry is no farther than its neighbours
    in layer 1 and no farther than the top node; the layers nest."""
    w, x, q, g, entry = _compact_case(metric, n=3000)
    lay = W.build_upper_layers(x, R_up=8, M=8, seed=3)
    node, adj, down, ls = lay["node"], lay["adj"], lay["down"], lay["layer_start"]
    assert len(ls) >= 3  # at least two upper layers at this size
    for r in range(ls[1], len(node)):  # down goes to the same node one layer lower
        lv = np.searchsorted(ls, r, side="right") - 1
        assert ls[lv - 1] <= down[r] < ls[lv] and node[down[r]] == node[r]
    assert np.all(down[:ls[1]] == -1)
    ent, nd, frag = O.descend(x, lay, q, metric, precision=64)
    row_of = {int(node[r]): r for r in range(ls[1])}
    for i in range(len(q)):
        r = row_of[int(ent[i])]
        nbs = node[adj[r][adj[r] >= 0]]
        de = _dist64(x[ent[i]], q[i], metric)
        assert np.all(de <= _dist64(x[nbs], q[i], metric))
        assert de <= _dist64(x[node[lay["top"]]], q[i], metric)


def test_descended_entry_shortens_the_search():
    """Starting the base-layer search at the descent's node instead of the
    medoid takes fewer expansions on average at the same results quality."""
    w = W.TINY.with_sizes(n=6000, nq=100)
    x, q = W.make_base(w), W.make_queries(w)
    g, entry = W.build_graph(x, w.R, w.cand)
    A, B = W.directions_for(w)
    lay = W.build_upper_layers(x, R_up=8, M=8, seed=1)
    ent, _, _ = O.descend(x, lay, q, w.metric, precision=32)
    a = O.search(x, g, entry, q, 10, 32, w.L, w.m, A, B, w.metric, 0.1, pool=32, precision=32)
    b = O.search(x, g, entry, q, 10, 32, w.L, w.m, A, B, w.metric, 0.1, pool=32, precision=32,
                 entries=ent)
    ci = O.COUNTERS.index
    assert b["counters"][:, ci("expansions")].mean() < a["counters"][:, ci("expansions")].mean()
    gt, _ = O.brute_force(x, q, 10, w.metric)
    rec = lambda I: np.mean([len(set(I[i]) & set(gt[i])) for i in range(len(q))]) / 10
    assert rec(b["ids"]) >= rec(a["ids"]) - 0.01
