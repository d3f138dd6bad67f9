"""The C-ABI library loads and exports every entry point of include/peos.h;
its pure host functions validate arguments.  No device work here."""
import ctypes
import os
import re

import pytest

import paper_2402_11354_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "peos.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(peos_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for fn in ("peos_index_bytes", "peos_build_tables", "peos_search", "peos_search_tables",
               "peos_query_tables", "peos_search_ws_bytes", "peos_free", "peos_strerror",
               "peos_last_error", "peos_index_layout"):
        assert fn in names


def test_library_exports_every_declared_symbol():
    lib = P.lib()
    for fn in declared_functions():
        assert hasattr(lib, fn), fn


def test_index_bytes_layout():
    ib, wb = P.peos_index_bytes(1000, 128, 32, 8, 16)
    # per node: R * round_up(B+1, 4) code bytes (B = 8, 16, 32, the kernel's
    # subspace bound >= L) padded to 16, then 4 floats per edge, padded to 128
    assert ib == 1000 * 896 and wb > 0
    ib, _ = P.peos_index_bytes(10, 32, 16, 4, 16)
    assert ib == 10 * 512
    ib, _ = P.peos_index_bytes(10, 96, 16, 12, 16)
    assert ib == 10 * 640
    ib, _ = P.peos_index_bytes(10, 960, 32, 16, 16)
    assert ib == 10 * 1152


@pytest.mark.parametrize("args", [
    (0, 128, 32, 8, 16),      # n < 1
    (10, 130, 32, 8, 16),     # d not a multiple of 4
    (10, 128, 0, 8, 16),      # R < 1
    (10, 128, 65, 8, 16),     # R > 64
    (10, 128, 32, 7, 16),     # L does not divide d
    (10, 96, 32, 32, 16),     # d/L = 3 not a multiple of 4
    (10, 128, 32, 8, 8),      # m < 16
    (10, 128, 32, 8, 24),     # m not a multiple of 16
    (10, 128, 32, 8, 144),    # 2m > 256
])
def test_index_bytes_rejects_bad_shapes(args):
    with pytest.raises(P.PeosError) as e:
        P.peos_index_bytes(*args)
    assert e.value.code == -1


def test_strerror_and_last_error():
    lib = P.lib()
    assert lib.peos_strerror(0) == b"ok"
    assert b"invalid" in lib.peos_strerror(-1)
    with pytest.raises(P.PeosError):
        P.peos_index_bytes(0, 128, 32, 8, 16)
    assert b"n=" in lib.peos_last_error()


def test_null_outputs_rejected():
    lib = P.lib()
    assert lib.peos_index_bytes(10, 32, 16, 4, 16, 0, None, None) == -1
    h = ctypes.c_void_p()
    rc = lib.peos_build_tables(None, 10, 32, None, 16, 0, 4, 16, None, None, 0, 0, None, 0, None,
                               0, None, ctypes.byref(h))
    assert rc == -1 and not h.value


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the built HIP library the binding raises; it has no other path."""
    monkeypatch.setattr(P, "_lib", None)
    monkeypatch.setattr(P, "LIB_PATH", str(tmp_path / "libpeos.so"))
    with pytest.raises(RuntimeError, match="is missing"):
        P.lib()


def test_product_does_not_reach_the_oracle():
    """The package and its kernels share nothing with the oracle: no import of
    it, no include of its sources, no path into its folder."""
    pkg = os.path.join(ROOT, "paper_2402_11354_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if not f.endswith((".py", ".hip", ".hpp", ".h", ".c", ".cpp")):
                continue
            src = open(os.path.join(dirpath, f)).read()
            assert not re.search(r"^\s*(from|import)\s+oracle\b", src, flags=re.M), f
            assert not re.search(r"#\s*include\s*\"[^\"]*oracle", src), f
            assert "peos_oracle" not in src, f


def test_launch_plan_setters_need_an_index():
    """The launch plan belongs to an index: every setter rejects a null one
    (valid values are checked on the GPU, where an index can be built)."""
    lib = P.lib()
    assert lib.peos_set_long_rows(None, 1) == P.PEOS_EINVAL
    assert lib.peos_set_search_tuning(None, 0, 0, 0, 0) == P.PEOS_EINVAL
    assert lib.peos_set_class_tuning(None, 0, 0, 0, 0) == P.PEOS_EINVAL
    assert b"null index" in lib.peos_last_error()
