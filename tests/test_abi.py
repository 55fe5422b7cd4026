"""The C-ABI boundary without a GPU: the built library loads, exports every
entry point that include/ibx.h declares (and no other ib_ symbol), and its
host-only entry points behave as documented.  No kernel is launched."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ibx.h")
LIB = os.path.join(ROOT, "paper_2408_14140_amd", "libibx.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)       # drop comments
    src = re.sub(r"//[^\n]*", " ", src)
    return sorted(set(re.findall(r"\b(ib_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        subprocess.run(["python", os.path.join(ROOT, "paper_2408_14140_amd", "build.py")],
                       check=True)
    return C.CDLL(LIB)


def test_header_declares_the_hot_path_calls():
    names = _declared()
    for n in ("ib_build_markers", "ib_bucket", "ib_interp", "ib_spread",
              "ib_multidirect_force", "ib_particle_reductions", "ib_multidirect_backward"):
        assert n in names


def test_library_exports_exactly_the_declared_symbols(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], check=True, capture_output=True,
                         text=True).stdout
    exported = sorted({ln.split()[-1] for ln in out.splitlines()
                       if re.search(r"\sT\s+ib_", ln)})
    assert exported == _declared()
    for n in _declared():
        assert getattr(lib, n) is not None


def test_version_and_status_strings(lib):
    lib.ib_version.restype = C.c_int
    assert lib.ib_version() == 1
    lib.ib_status_string.restype = C.c_char_p
    texts = [lib.ib_status_string(s).decode() for s in (0, -1, -2, -3, -4, -5)]
    assert texts[0] == "ok" and len(set(texts)) == 6
    assert lib.ib_status_string(7).decode() == "unknown status"


def test_count_markers_matches_the_oracle(lib, oracle_mod):
    f = lib.ib_count_markers
    f.restype = C.c_int64
    f.argtypes = [C.c_int32, C.c_void_p, C.c_double, C.c_void_p]
    rng = np.random.default_rng(3)
    h = 1.0 / 256
    d = rng.uniform(8, 32, 500) * h
    offs = np.zeros(d.size + 1, np.int64)
    total = f(d.size, d.ctypes.data, h, offs.ctypes.data)
    ref = oracle_mod.count_markers(d, h)
    assert total == ref[-1]
    assert np.array_equal(offs, ref)
    # the paper's resolutions: D/h = 16 gives round(256 pi) markers
    one = np.array([16 * h])
    o1 = np.zeros(2, np.int64)
    assert f(1, one.ctypes.data, h, o1.ctypes.data) == 804


@pytest.mark.parametrize("np_, h, d", [(-1, 0.1, 1.0), (1, 0.0, 1.0), (1, 0.1, 0.0),
                                       (1, 0.1, float("nan"))])
def test_count_markers_rejects_bad_arguments(lib, np_, h, d):
    f = lib.ib_count_markers
    f.restype = C.c_int64
    f.argtypes = [C.c_int32, C.c_void_p, C.c_double, C.c_void_p]
    dd = np.array([d])
    offs = np.zeros(2, np.int64)
    assert f(np_, dd.ctypes.data, h, offs.ctypes.data) == -1
    assert f(1, dd.ctypes.data, 0.1, None) == -1


def test_build_entry_calls_both_builders(monkeypatch):
    """build() compiles the library and the oracle (stand-ins record the calls)
    and reaches the library's builder without importing the package first."""
    import importlib

    import __graft_entry__ as ge
    ge = importlib.reload(ge)
    assert ge._library_builder().__module__ == "_libibx_build"
    ob = importlib.import_module("oracle.build")   # the submodule, not the re-exported function
    calls = []
    monkeypatch.setattr(ob, "build", lambda *a, **k: calls.append("oracle"))
    monkeypatch.setattr(ge, "_library_builder", lambda: (lambda: calls.append("library")))
    ge.build()
    assert sorted(calls) == ["library", "oracle"]


def test_bench_refuses_more_than_one_gpu():
    """The library has no multi-GPU path: bench.py --gpus N > 1 exits with a
    message before touching a GPU."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_bench_reports_counted_traffic_only_for_the_counted_variants(tmp_path):
    """bench.py takes the dominant kernel's HBM traffic from a committed
    counter summary (one line per counted tuning variant) only while the
    kernel sources hash as when it was taken, and only the line of the
    variant its plan runs."""
    import sys
    sys.path.insert(0, ROOT)
    import bench
    summary = tmp_path / "summary.txt"
    path = str(summary)                  # absolute: joined to nothing
    summary.write_text("traffic_bytes_per_launch: spread 1000 row_masks=0 interp_tile=8\n"
                       "traffic_bytes_per_launch: spread 900 row_masks=1 interp_tile=8\n"
                       "traffic_bytes_per_launch: spread 1100 row_masks=0 interp_tile=16\n"
                       f"sources_sha256_16: {bench.sources_sha()}\n")
    assert bench.committed_traffic("spread", path) == 1000.0
    assert bench.committed_traffic("spread", path, {"row_masks": 1, "interp_tile": 8}) == 900.0
    assert bench.committed_traffic("spread", path, {"row_masks": 0, "interp_tile": 16}) == 1100.0
    assert bench.committed_traffic("spread", path, {"row_masks": 1, "interp_tile": 16}) is None
    assert bench.committed_traffic("interp_g", path) is None
    summary.write_text("traffic_bytes_per_launch: spread 1000\nsources_sha256_16: 0123456789abcdef\n")
    assert bench.committed_traffic("spread", path) is None
