"""The C ABI without a GPU: the library loads, exports every function
include/exsum.h declares, and rejects bad arguments on the host before any
device work (no compute call is made here)."""
import ctypes
import os
import re

import pytest

import paper_1505_05571_amd as ex

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "exsum.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(exsum_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(ex.library_path()):
        from paper_1505_05571_amd import build
        build.build()
    return ex.load_library()


def test_header_declares_expected_entry_points():
    names = declared_functions()
    assert "exsum_f64" in names and "exsum_segmented_f64" in names
    assert set(names) == set(ex.EXPORTED_SYMBOLS)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = os.popen("nm -D --defined-only %s" % ex.library_path()).read()
    for name in declared_functions():
        assert re.search(r"\bT %s\b" % name, out), name


def test_status_strings(lib):
    assert ex.exsum_status_string(0) == "ok"
    assert ex.exsum_status_string(1) == "invalid argument"
    assert ex.exsum_status_string(99) == "unknown status"


def test_host_side_argument_checks(lib):
    P = ctypes.c_void_p
    assert lib.exsum_f64(None, -1, P(8), None) == 1
    assert lib.exsum_f64(None, 10, P(8), None) == 1          # x NULL with work to do
    assert lib.exsum_f64(P(8), 10, None, None) == 1          # out NULL
    assert lib.exsum_f64(P(8), 1 << 40, P(8), None) == 1     # too many terms
    assert lib.exsum_inexact_f64(None, -5, P(8), None) == 1
    assert lib.exsum_segmented_f64(None, None, -1, None, None) == 1
    assert lib.exsum_segmented_f64(None, None, 0, None, None) == 0   # nothing to do
    assert lib.exsum_segmented_f64(None, P(8), 3, P(8), None) == 1
    assert lib.exsum_f64_cfg(P(8), 4, P(8), None, None) == 1


def test_config_roundtrip_and_validation(lib):
    c0 = ex.exsum_get_config()
    try:
        c = ex.exsum_get_config()
        c.large_block, c.large_vec, c.large_depth, c.large_mode = 512, 3, 2, 0
        ex.exsum_set_config(c)
        assert ex.exsum_get_config().large_vec == 3
        c.large_block, c.large_vec, c.large_depth, c.large_mode = 1024, 4, 2, 1
        ex.exsum_set_config(c)
        assert ex.exsum_get_config().large_mode == 1
        for field, bad in [("large_vec", 8), ("large_block", 128), ("precombine", -1), ("large_mode", 2),
                           ("seg_small_max", 1 << 21), ("large_grid", -3)]:
            c = ex.exsum_get_config()
            setattr(c, field, bad)
            with pytest.raises(ex.ExsumError):
                ex.exsum_set_config(c)
    finally:
        ex.exsum_set_config(c0)
