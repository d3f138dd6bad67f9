"""Seeded synthetic workloads for PEOs-routed graph search.

This module only *generates inputs*: base and query vectors, the Gaussian
projection directions of PEOs step (2) (Sec. "PEOs Test"), the proximity
graph that the search walks (the paper treats the graph index as given,
Sec. "Problem Definition"), and exact top-k ground truth for recall.  It holds
none of the routing arithmetic; the HIP library and the CPU oracle both take
what it produces as input and share nothing else.

The paper evaluates on SIFT10M, GIST, DEEP10M and others (Table 1); none are
available here, so each workload below is a synthetic stand-in with the same
shape (dimension, metric, value type) drawn from a seeded mixture model.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

L2 = 0
ANGULAR = 1
IP = 2  # maximum inner product (distance -x.q)

_CHUNK_ROWS = 65536  # fixed so that chunked draws are reproducible


@dataclasses.dataclass(frozen=True)
class Workload:
    """Shape and recipe of one synthetic workload."""
    name: str
    n: int
    nq: int
    d: int
    R: int          # max out-degree of the pruned graph
    cand: int       # exact-NN candidates before pruning
    L: int          # PEOs subspaces
    m: int          # Gaussian directions per subspace
    metric: int
    family: str     # mixture recipe, see _Model
    eps: float
    k: int
    ef: int
    seed: int       # base seed; queries use seed+1000, directions seed+2000
    rand_edges: int = 0  # random long-range edges per node added to the graph

    def with_sizes(self, n=None, nq=None):
        return dataclasses.replace(self, n=self.n if n is None else n,
                                   nq=self.nq if nq is None else nq)


# The five workloads.  Seeds follow 1000+c / 2000+c / 3000+c for workload c.
TINY = Workload("tiny_gmm_2k_d32", 2000, 100, 32, 16, 32, 4, 16, L2, "gmm10", 0.1, 10, 32, 1001)
SIFT_LIKE = Workload("sift_like_1m_d128", 1_000_000, 10_000, 128, 32, 64, 8, 16, L2, "expint100", 0.1, 10, 64, 1002)
GIST_LIKE = Workload("gist_like_1m_d960", 1_000_000, 1_000, 960, 32, 64, 16, 16, L2, "gmm256lowrank", 0.1, 10, 128, 1003, rand_edges=8)
DEEP_LIKE = Workload("deep_like_10m_d96", 10_000_000, 100_000, 96, 32, 64, 8, 16, ANGULAR, "sphere1000", 0.1, 10, 64, 1004)
SERVING = Workload("serving_1m_d256", 1_000_000, 10_000, 256, 32, 64, 8, 16, ANGULAR, "sphere500", 0.1, 10, 64, 1005)

WORKLOADS = {w.name: w for w in (TINY, SIFT_LIKE, GIST_LIKE, DEEP_LIKE, SERVING)}


# ---------------------------------------------------------------------------
# vectors
# ---------------------------------------------------------------------------
class _Model:
    """Mixture parameters, drawn from the base seed so queries share them."""

    def __init__(self, w: Workload):
        rng = np.random.default_rng(w.seed)
        self.w = w
        if w.family == "gmm10":
            # 10 unit-variance components, centres ~ N(0, 4 I).
            self.kind = "gmm"
            self.centers = rng.normal(0.0, 2.0, size=(10, w.d))
            self.scales = np.ones((10, w.d))
            self.weights = np.full(10, 0.1)
        elif w.family == "expint100":
            # 100 clusters, weights ~ 1/(c+1); per-dim exponential means
            # log-uniform in [2, 64]; values floor()ed and clipped to 0..255.
            self.kind = "expint"
            c = np.arange(100)
            wts = 1.0 / (c + 1.0)
            self.weights = wts / wts.sum()
            self.means = np.exp(rng.uniform(math.log(2.0), math.log(64.0), size=(100, w.d)))
        elif w.family == "gmm256lowrank":
            # 256 anisotropic clusters in a 48-dimensional latent space (the
            # strong correlations of global image descriptors): x = mu_c +
            # F (s_c * z) + 0.05 N(0, I), F a fixed d x 48 random factor
            # matrix with unit-norm columns, s_c a decaying latent spectrum
            # (j+1)^-1/2 scaled to norm 24 times a per-cluster LogNormal(0, 0.3)
            # factor, centres N(0, 0.5^2 I) so that neighbouring clusters
            # overlap.
            self.kind = "lowrank"
            k = 48
            self.centers = rng.normal(0.0, 0.5, size=(256, w.d))
            F = rng.normal(size=(w.d, k))
            self.factors = F / np.linalg.norm(F, axis=0, keepdims=True)
            spec = (np.arange(k) + 1.0) ** -0.5
            spec = 24.0 * spec / np.linalg.norm(spec)
            self.latent = spec[None, :] * np.exp(rng.normal(0.0, 0.3, size=(256, k)))
            self.weights = np.full(256, 1.0 / 256)
        elif w.family in ("sphere1000", "sphere500"):
            # vMF-like clusters on the sphere: normalize(mu_c + 2.5 s * z),
            # mu_c uniform on the sphere, z ~ N(0, I), and a decaying
            # per-dimension spectrum s_j ~ (j+1)^-0.8 with |s| = 1, the shape of
            # PCA-compressed descriptors (low intrinsic dimension; the noise
            # norm of 2.5 makes neighbouring clusters overlap, as real
            # descriptor clusters do).
            self.kind = "sphere"
            ncl = 1000 if w.family == "sphere1000" else 500
            mu = rng.normal(size=(ncl, w.d))
            self.centers = mu / np.linalg.norm(mu, axis=1, keepdims=True)
            self.weights = np.full(ncl, 1.0 / ncl)
            spec = (np.arange(w.d) + 1.0) ** -0.8
            self.spectrum = 2.5 * spec / np.linalg.norm(spec)
        else:
            raise ValueError(f"unknown family {w.family}")

    def draw(self, count: int, rng: np.random.Generator) -> np.ndarray:
        out = np.empty((count, self.w.d), dtype=np.float32)
        for s in range(0, count, _CHUNK_ROWS):
            c = min(_CHUNK_ROWS, count - s)
            z = rng.choice(len(self.weights), size=c, p=self.weights)
            if self.kind == "gmm":
                x = self.centers[z] + self.scales[z] * rng.standard_normal((c, self.w.d))
            elif self.kind == "lowrank":
                lat = self.latent[z] * rng.standard_normal((c, self.latent.shape[1]))
                x = (self.centers[z] + lat @ self.factors.T
                     + 0.05 * rng.standard_normal((c, self.w.d)))
            elif self.kind == "expint":
                x = np.minimum(255.0, np.floor(rng.exponential(1.0, size=(c, self.w.d)) * self.means[z]))
            else:
                x = self.centers[z] + self.spectrum * rng.standard_normal((c, self.w.d))
                x /= np.linalg.norm(x, axis=1, keepdims=True)
            out[s:s + c] = x
        return out


def make_base(w: Workload) -> np.ndarray:
    """n x d float32 base vectors (row-major)."""
    model = _Model(w)
    rng = np.random.default_rng([w.seed, 1])
    x = model.draw(w.n, rng)
    if w.metric == ANGULAR:
        x = _renormalize(x)
    return x


def make_queries(w: Workload) -> np.ndarray:
    """nq x d float32 queries: fresh draws from the base's mixture."""
    model = _Model(w)
    rng = np.random.default_rng(w.seed + 1000)
    q = model.draw(w.nq, rng)
    if w.metric == ANGULAR:
        q = _renormalize(q)
    return q


def _renormalize(x: np.ndarray) -> np.ndarray:
    # unit norm in float32 after the cast
    x64 = x.astype(np.float64)
    x64 /= np.linalg.norm(x64, axis=1, keepdims=True)
    return x64.astype(np.float32)


def make_directions(L: int, m: int, d: int, seed: int):
    """Gaussian projection vectors of PEOs step (2).

    Returns (A, B): A is L x m x (d/L) float32 (per-subspace vectors a^i_j),
    B is m x d float32 (full-space vectors b_j).  Entries are N(0, 1).
    """
    if d % L:
        raise ValueError("d must be a multiple of L")
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((L, m, d // L)).astype(np.float32)
    B = rng.standard_normal((m, d)).astype(np.float32)
    return A, B


def directions_for(w: Workload):
    return make_directions(w.L, w.m, w.d, w.seed + 2000)


def query_params(w: Workload, nq: int, seed: int = 0):
    """Per-query k and ef for the batched workload: ef ~ U{32,64,128,256},
    k ~ U{1,10,100}, ef := max(ef, k)."""
    rng = np.random.default_rng([w.seed, 7, seed])
    ef = rng.choice(np.array([32, 64, 128, 256], dtype=np.int32), size=nq)
    k = rng.choice(np.array([1, 10, 100], dtype=np.int32), size=nq)
    return k.astype(np.int32), np.maximum(ef, k).astype(np.int32)


from .graph import build_graph, build_upper_layers, ground_truth, medoid  # noqa: E402,F401


def graph_for(w: Workload, base: np.ndarray, device="cpu", log=None):
    """The workload's graph: pruned kNN graph of degree R from `cand`
    candidates, plus its random long-range edges."""
    return build_graph(base, w.R, w.cand, device=device, log=log, rand_edges=w.rand_edges,
                       seed=w.seed)
