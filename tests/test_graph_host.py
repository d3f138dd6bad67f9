"""Host-side checks of the input graph builder: the IVF neighbour scan used
for bases too large for the exact product.  CPU only."""
import os
import sys

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
from workloads.graph import knn, knn_ivf  # noqa: E402


def _clustered(n=4000, d=16, seed=5):
    rng = np.random.default_rng(seed)
    cent = rng.normal(0.0, 3.0, size=(20, d))
    lab = rng.integers(0, 20, size=n)
    return torch.from_numpy((cent[lab] + rng.normal(size=(n, d))).astype(np.float32))


def test_ivf_neighbours_agree_with_exact_scan():
    x = _clustered()
    k = 10
    ids, dists = knn_ivf(x, k, nlist=32, nprobe=8, iters=4, seed=3)
    ex_i, ex_d = knn(x, x, k, exclude_self=True)
    # rows come back ordered by (distance, id), never containing the row itself
    assert (ids != torch.arange(x.shape[0])[:, None]).all()
    assert (dists[:, 1:] >= dists[:, :-1]).all()
    # the scan only misses neighbours that fall outside the probed lists
    hit = np.mean([len(set(a) & set(b)) / k for a, b in zip(ids.tolist(), ex_i.tolist())])
    assert hit >= 0.95, hit
    # every returned distance is the true squared distance of that pair
    diff = x[:, None, :] - x[ids.clamp(min=0)]
    assert torch.allclose((diff * diff).sum(-1), dists, rtol=1e-4, atol=1e-3)


def test_ivf_scan_is_reproducible():
    x = _clustered(n=3000, seed=9)
    a = knn_ivf(x, 8, nlist=16, nprobe=4, iters=3, seed=1)
    b = knn_ivf(x, 8, nlist=16, nprobe=4, iters=3, seed=1)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
