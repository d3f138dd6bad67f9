"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The oracle (plain C) is rebuilt with -fsanitize=address,undefined and its
  searches, builds, tests, descent, compact form and dimension permutation
  run on small inputs in a child interpreter that preloads the sanitizer
  runtimes; any report fails the test.
* The HIP library (peos_api.hip) is built with the sanitizers on its host
  compilation only, and a C driver
  (tests/host/abi_driver.c) calls every entry point with arguments it must
  reject and the pure host functions with valid ones.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"

pytestmark = pytest.mark.timeout(600)


def _gcc_runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = p.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


ORACLE_SCRIPT = r"""
import numpy as np
import oracle as O
import workloads as W
w = W.TINY.with_sizes(n=600, nq=12)
x, q = W.make_base(w), W.make_queries(w)
g, e = W.build_graph(x, w.R, w.cand)
A, B = W.directions_for(w)
O.build_tables(x, g, w.L, w.m, A, B, nthreads=2)
for prec in (32, 64):
    for pool in (0, 32, -2):
        for mode in (O.MODE_PEOS, O.MODE_EXHAUSTIVE):
            O.search(x, g, e, q, 10, 32, w.L, w.m, A, B, w.metric, 0.1, mode=mode, pool=pool,
                     precision=prec, nthreads=2)
O.search(x, g, e, q, 10, 32, w.L, w.m, A, B, w.metric, 0.1, lowp=O.LP_FP16 | O.LP_BF16_BASE)
C = np.random.default_rng(1).normal(size=(64, w.d)).astype(np.float32)
O.search(x, g, e, q, 10, 32, w.L, w.m, A, B, w.metric, 0.2, mode=O.MODE_SIMHASH, simhash=C)
A2, B2 = W.make_directions(2, w.m, w.d, 3)
O.search(x, g, e, q, 10, 32, 2, w.m, A2, B2, w.metric, 0.1, lowp=O.LP_COMPACT, precision=64)
O.compact_tables(x, g, 2, w.metric)
O.dimension_permutation(x, g, w.L)
lay = W.build_upper_layers(x, R_up=8, M=8, seed=2)
ent, nd, fr = O.descend(x, lay, q, w.metric, precision=64)
O.search(x, g, e, q, 10, 32, w.L, w.m, A, B, w.metric, 0.1, entries=ent)
O.test_edge(x[0], x[1], x[2], q[0], w.L, w.m, A, B, w.metric, 0.1)
print("oracle under sanitizers ok")
"""


def test_oracle_under_asan_and_ubsan(tmp_path):
    asan, ubsan = _gcc_runtime("libasan.so"), _gcc_runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    lib = tmp_path / "liboracle_san.so"
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-fno-omit-frame-pointer", "-fPIC", "-shared", "-pthread",
                           os.path.join(ROOT, "oracle", "peos_oracle.c"), "-o", str(lib), "-lm"])
    env = dict(os.environ, PEOS_ORACLE_LIB=str(lib), LD_PRELOAD=f"{asan}:{ubsan}",
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", ORACLE_SCRIPT], capture_output=True, text=True,
                       env=env, cwd=ROOT, timeout=500)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    assert "oracle under sanitizers ok" in r.stdout


def test_library_host_code_under_asan_and_ubsan(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("ROCm compilers not installed")
    rt = subprocess.run([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"],
                        capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(rt) or not os.path.exists(rt):
        pytest.skip("clang's shared AddressSanitizer runtime not found")
    lib = tmp_path / "libpeos_san.so"
    # the sanitizers go on the host compilation only (nothing here runs on a
    # GPU; the device code is built as usual so that the library loads)
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
                           "-packed-fp32-ops", "-O1", "-g", "-std=c++17", "-fPIC",
                           "-shared", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
                           "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=undefined",
                           "-shared-libsan",
                           os.path.join(ROOT, "paper_2402_11354_amd", "csrc", "peos_api.hip"),
                           "-o", str(lib)], stderr=subprocess.DEVNULL)
    exe = tmp_path / "abi_driver"
    subprocess.check_call([CLANG, "-O1", "-g", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-shared-libsan",
                           os.path.join(ROOT, "tests", "host", "abi_driver.c"), str(lib),
                           f"-Wl,-rpath,{tmp_path}", f"-Wl,-rpath,{os.path.dirname(rt)}",
                           "-o", str(exe)])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
    assert "abi driver ok" in r.stdout
