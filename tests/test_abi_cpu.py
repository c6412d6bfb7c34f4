"""C ABI checks that need no GPU: the library loads, exports every call the
header declares, the header compiles as C99, and host-side argument checks
fail with the documented status before any device work."""

import ctypes
import math
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ara.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(ara_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def ara():
    from paper_1606_04473_amd import ara as mod
    if not os.path.exists(mod.LIB_PATH):
        pytest.fail("libara.so is not built; run __graft_entry__.build()")
    mod.lib()
    return mod


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("ara_create_tables", "ara_run_layers", "ara_risk_metrics", "ara_backward",
              "ara_destroy_tables", "ara_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(ara):
    out = subprocess.run(["nm", "-D", "--defined-only", ara.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (ara_[a-z_]+)\b", out))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    assert set(ara.EXPORTED) <= exported


def test_header_compiles_as_c99(tmp_path):
    src = tmp_path / "h.c"
    src.write_text('#include "ara.h"\nint main(void){ara_layer l; (void)l; return ARA_OK;}\n')
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.dirname(HEADER), "-c",
                    str(src), "-o", str(tmp_path / "h.o")], check=True)


def test_status_strings(ara):
    assert ara.status_string(0) == "ARA_OK"
    assert ara.status_string(ara.ARA_ERR_NOT_READY) == "ARA_ERR_NOT_READY"
    assert ara.status_string(99) == "ARA_ERR_UNKNOWN"


def test_host_side_argument_errors(ara):
    L = ara.lib()
    h = ctypes.c_void_p()
    # NULL out handle / negative sizes / empty catalogue
    assert L.ara_create_tables(None, 0, None, 0, None, 0, 10, 0, None, None) == ara.ARA_ERR_INVALID_ARG
    off = np.array([0, 2], dtype=np.int64)
    assert L.ara_create_tables(off.ctypes.data_as(ctypes.c_void_p), -1, None, 0, None, 0, 10, 0, None,
                               ctypes.byref(h)) == ara.ARA_ERR_INVALID_ARG
    assert L.ara_create_tables(off.ctypes.data_as(ctypes.c_void_p), 1, None, 2, None, 0, 0, 0, None,
                               ctypes.byref(h)) == ara.ARA_ERR_INVALID_ARG
    bad = np.array([1, 2], dtype=np.int64)
    ids = np.zeros(2, dtype=np.uint32)
    assert L.ara_create_tables(bad.ctypes.data_as(ctypes.c_void_p), 1, ids.ctypes.data_as(ctypes.c_void_p),
                               2, None, 0, 4, 0, None, ctypes.byref(h)) == ara.ARA_ERR_INVALID_ARG
    assert "offsets" in ara.lib().ara_last_error().decode()
    # risk metrics: p outside (0,1), no trials
    y = np.zeros(4)
    mean = ctypes.c_double()
    pml = np.zeros(1)
    tv = np.zeros(1)
    for p, n in ((1.0, 4), (0.0, 4), (math.nan, 4), (0.5, 0)):
        pr = np.array([p])
        st = L.ara_risk_metrics(y.ctypes.data_as(ctypes.c_void_p), n, pr.ctypes.data_as(ctypes.c_void_p), 1,
                                ctypes.byref(mean), pml.ctypes.data_as(ctypes.c_void_p),
                                tv.ctypes.data_as(ctypes.c_void_p), 0, None)
        assert st == ara.ARA_ERR_INVALID_ARG
    # run_layers / backward with NULL tables
    arr, keep = ara._c_layers([ara.LayerSpec(np.zeros(1, np.int32), np.zeros(1), np.ones(1), 0.0, 1.0,
                                             0.0, 1.0, 0, 1)])
    out = np.zeros(1)
    assert L.ara_run_layers(None, arr, 1, out.ctypes.data_as(ctypes.c_void_p), 1, 0, None) == \
        ara.ARA_ERR_INVALID_ARG
    assert L.ara_backward(None, arr, 0.99, None, None, 0, None) == ara.ARA_ERR_INVALID_ARG


def test_product_path_has_no_oracle_dependency():
    """The package and its sources never name the oracle."""
    pkg = os.path.join(ROOT, "paper_1606_04473_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "ara_oracle" not in text, f


def test_tail_count_matches_oracle(ara):
    """The library's m (shortest decimal digits of p, exact integer arithmetic)
    equals the oracle's (Python repr of p as an exact fraction) on hand-picked
    and random probabilities over a range of trial counts."""
    import oracle
    rng = np.random.default_rng(20250)
    probs = [0.99, 0.996, 0.989999999999, 0.9899999999999999, 0.5, 0.25, 0.75, 1.0 / 3.0, 2.0 / 3.0,
             0.1, 0.2, 0.3, 0.7, 0.9, 0.95, 0.999, 0.9999, 0.99999999, 1e-300, 5e-324,
             math.nextafter(1.0, 0.0), math.nextafter(0.99, 1.0), math.nextafter(0.99, 0.0),
             0.1 + 0.2, 1e-17, 0.123456789012345678]
    probs += [float(x) for x in rng.random(300)]
    probs += [float(x) for x in 1.0 - 10.0 ** -rng.uniform(1, 16, 100)]
    probs += [round(float(x), int(d)) for x, d in zip(rng.random(200), rng.integers(1, 13, 200))]
    probs = [p for p in probs if 0.0 < p < 1.0]
    sizes = [1, 2, 3, 4, 7, 10, 100, 997, 10_000, 1_000_000, 123_456_789, 10 ** 12, 2 ** 62,
             2 ** 63 - 1]
    for n in sizes:
        for p in probs:
            assert ara.tail_count(n, p) == oracle.tail_count(n, p), (n, p)
    with pytest.raises(ara.AraError):
        ara.tail_count(0, 0.5)
    for bad in (0.0, 1.0, math.nan, -0.5, math.inf):
        with pytest.raises(ara.AraError):
            ara.tail_count(10, bad)
