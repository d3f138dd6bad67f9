"""Host-side logic of bench.py: the algorithmic-byte accounting, the memory
counter record and the one-GPU guard.  No device work."""
import json
import os
import subprocess
import sys
import types

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def layout(**kw):
    base = dict(flags=0, R=32, code_bytes=12, scalar_bytes=16, d=128, L=8, m=16)
    base.update(kw)
    return types.SimpleNamespace(**base)


def one_query(**cols):
    st = np.zeros((1, 14), np.int32)
    for i, v in cols.items():
        st[0, int(i[1:])] = v
    return st


def test_alg_bytes_terms():
    lay = layout()
    fixed = 4 * 128 + 4 * 9 * 16 + 12 * 10
    assert bench.search_alg_bytes(one_query(), lay, 10, 64) == fixed
    # per expansion: R ids; per tested edge: codes + scalars; per distance: a row
    assert bench.search_alg_bytes(one_query(c0=3), lay, 10, 64) == fixed + 3 * 4 * 32
    assert bench.search_alg_bytes(one_query(c3=5), lay, 10, 64) == fixed + 5 * (12 + 16)
    assert bench.search_alg_bytes(one_query(c9=7), lay, 10, 64) == fixed + 7 * 512
    # a compact record adds its node header per expansion that ran the test
    c = layout(flags=8, L=2, code_bytes=4, scalar_bytes=2)
    fixed_c = 4 * 128 + 4 * 3 * 16 + 120
    assert bench.search_alg_bytes(one_query(c3=5, c13=2), c, 10, 64) == fixed_c + 5 * 6 + 2 * 16
    # bfloat16 rows, half tables, and the fp32 re-rank of the final list
    p = layout(flags=3, scalar_bytes=8)
    fixed_p = 4 * 128 + 2 * 9 * 16 + 120 + 4 * 128 * 64
    assert bench.search_alg_bytes(one_query(c9=7), p, 10, 64) == fixed_p + 7 * 256
    # the descent: an id and a row per distance
    assert bench.search_alg_bytes(one_query(c12=4), lay, 10, 64) == fixed + 4 * (512 + 4)
    # per-query k
    st = np.zeros((2, 14), np.int32)
    assert bench.search_alg_bytes(st, lay, np.array([1.0, 100.0]), 0) == 2 * (fixed - 120) + 12 * 101


def test_traffic_record_applies_only_to_the_kernel_it_was_taken_on():
    """A committed memory-counter record gives the benchmark's traffic only
    when it was taken on the search kernel's current sources and the same
    operating point; otherwise the benchmark reports no traffic (null)."""
    recs = []
    for f in os.listdir(os.path.join(ROOT, "profiles")):
        if f.endswith(".md"):
            for line in open(os.path.join(ROOT, "profiles", f)):
                if line.startswith("traffic-record:"):
                    recs.append(json.loads(line.split(":", 1)[1]))
    assert recs
    for rec in recs:
        key = {k: v for k, v in rec.items()
               if k not in ("fetch_kib", "write_kib", "fetch_scale", "write_scale")}
        key["source"] = bench.kernel_digest()  # what the benchmark asks for
        got = bench.traffic_record(key)
        if rec["source"] != bench.kernel_digest():
            assert got is None
            continue
        want = (rec["fetch_kib"] * rec["fetch_scale"] + rec["write_kib"] * rec["write_scale"]) * 1024.0
        assert got == want
        assert bench.traffic_record(dict(key, ef=key["ef"] + 1)) is None
    stale = dict(key, source="0" * 16)
    assert bench.traffic_record(stale) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]
