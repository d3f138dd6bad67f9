"""The compact records (index flag PEOS_FLAG_COMPACT) against the oracle's
compact form: the node headers, code bytes and scalar codes bit for bit (the
integer decisions are taken in single precision in one stated order on both
sides), and the search on non-fragile queries exactly (the quantile table
and the decoded scalars are the same values on both sides up to rounding
that the oracle's fragile flags cover)."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from parity import check_both, compare

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2402_11354_amd")

pytestmark = pytest.mark.gpu

ANGW = W.Workload("compact_ang_5k_d64", 5000, 100, 64, 16, 32, 4, 16, W.ANGULAR, "sphere500", 0.1,
                  10, 32, 1010)
IPW = W.Workload("compact_ip_3k_d64", 3000, 100, 64, 16, 32, 4, 16, W.IP, "gmm10", 0.1, 10, 32,
                 1011)


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda:0"))


class Case:
    def __init__(self, w, L, dup=False):
        self.w, self.L = w, L
        self.x = W.make_base(w)
        self.q = W.make_queries(w)
        self.g, self.entry = W.build_graph(self.x, w.R, w.cand)
        if dup:
            # two identical vectors: zero-length edges in both directions
            self.x[int(self.g[0, 0])] = self.x[0]
        self.A, self.B = W.make_directions(L, w.m, w.d, w.seed + 2000)
        self.xt, self.gt, self.At, self.Bt, self.qt = (T(a) for a in (self.x, self.g, self.A,
                                                                        self.B, self.q))
        self.idx = {}

    def index(self, flags=P.PEOS_FLAG_COMPACT):
        if flags not in self.idx:
            self.idx[flags] = P.peos_build_tables(self.xt, self.gt, self.entry, self.L, self.w.m,
                                                  self.At, self.Bt, self.w.metric, flags=flags)
        return self.idx[flags]

    def run(self, flags, pool, eps=None, mode=P.PEOS_MODE_PEOS, queries=None):
        w = self.w
        q = self.qt if queries is None else queries
        ids, d, st = P.search(self.index(flags), q, w.k, w.ef,
                              eps=w.eps if eps is None else eps, mode=mode, pool=pool)
        torch.cuda.synchronize()
        return ids.cpu().numpy(), d.cpu().numpy(), st.cpu().numpy()

    def oracle(self, lowp, pool, eps=None, mode=O.MODE_PEOS):
        w = self.w
        return O.search(self.x, self.g, self.entry, self.q, w.k, w.ef, self.L, w.m, self.A,
                        self.B, w.metric, w.eps if eps is None else eps, mode=mode, pool=pool,
                        lowp=lowp)


@pytest.fixture(scope="module")
def l2():
    print("[gpu] compact: tiny l2 workload, L = 2", flush=True)
    return Case(W.TINY.with_sizes(n=3000, nq=120), 2, dup=True)


@pytest.fixture(scope="module")
def ang():
    print("[gpu] compact: angular workload, L = 4", flush=True)
    return Case(ANGW, 4)


@pytest.fixture(scope="module")
def ip():
    print("[gpu] compact: inner-product workload, L = 4", flush=True)
    return Case(IPW, 4)


@pytest.mark.parametrize("which", ["l2", "ang", "ip"])
def test_compact_records_match_oracle(which, request):
    case = request.getfixturevalue(which)
    ix = case.index()
    lay = ix.layout()
    R, L = case.g.shape[1], case.L
    assert lay.code_bytes == 4 and lay.scalar_bytes == 2 and lay.codes_offset == 16
    assert lay.node_stride <= 256
    mem = ix._keep[-1].cpu().numpy()
    n = case.x.shape[0]
    rec = mem[:n * lay.node_stride].reshape(n, lay.node_stride)
    hdr = rec[:, :16].copy().view(np.float32)
    codes = rec[:, 16:16 + 4 * R].reshape(n, R, 4)
    sc = rec[:, lay.scalars_offset:lay.scalars_offset + 2 * R].reshape(n, R, 2)
    rh, rcg, rci = O.compact_tables(case.x, case.g, L, case.w.metric)
    rc, _, _ = O.build_tables(case.x, case.g, L, case.w.m, case.A, case.B)
    valid = case.g >= 0
    assert np.array_equal(hdr.view(np.uint32), rh.view(np.uint32))
    assert np.array_equal(codes[..., :L][valid], rc[..., 1:][valid])
    assert np.all(codes[..., L:] == 0)
    assert np.array_equal(sc[..., 0], rcg) and np.array_equal(sc[..., 1], rci)
    if which == "l2":
        assert sc[0, 0, 1] == 255


@pytest.mark.parametrize("which", ["l2", "ang", "ip"])
@pytest.mark.parametrize("pool_mul", [0, 1])
@pytest.mark.parametrize("bf16", [False, True])
def test_compact_search_matches_oracle(which, pool_mul, bf16, request):
    case = request.getfixturevalue(which)
    w = case.w
    flags = P.PEOS_FLAG_COMPACT | (P.PEOS_FLAG_BF16_BASE if bf16 else 0)
    lowp = O.LP_COMPACT | (O.LP_BF16_BASE if bf16 else 0)
    ids, d, st = case.run(flags, pool_mul * w.ef)
    if not bf16:
        # single-precision distances: the FP64 oracle of the compact test
        # is the arbiter, its single-precision replica the stricter check
        check_both((ids, d, st), case.x, case.g, case.entry, case.q, w.k, w.ef, case.L, w.m,
                   case.A, case.B, w.metric, w.eps, pool=pool_mul * w.ef, lowp=lowp,
                   min_checked=0.6, label=f"compact {which} pool={pool_mul * w.ef}")
    else:
        ref = case.oracle(lowp, pool_mul * w.ef)
        res = compare(ids, d, st, ref, w.k)
        print(f"[gpu] compact {which} pool={pool_mul * w.ef} bf16={bf16}: "
              f"checked={res['checked']} fragile={res['fragile']}")
        assert not res["bad"], res["bad"][:5]
        assert res["checked"] >= 0.8 * len(ids)
    if pool_mul == 0 or which == "l2":
        assert st[:, 6].sum() > 0  # H-vs-T tests ran


def test_compact_flag_validation(l2):
    w = l2.w
    A8, B8 = W.make_directions(8, w.m, w.d, 5)
    with pytest.raises(P.PeosError):
        P.peos_build_tables(l2.xt, l2.gt, l2.entry, 8, w.m, T(A8), T(B8), w.metric,
                            flags=P.PEOS_FLAG_COMPACT)
    with pytest.raises(P.PeosError):
        P.peos_build_tables(l2.xt, l2.gt, l2.entry, l2.L, w.m, l2.At, l2.Bt, w.metric,
                            flags=P.PEOS_FLAG_COMPACT | P.PEOS_FLAG_FP16)
