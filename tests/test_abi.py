"""The C ABI library loads and exports every entry point include/gsr.h declares; host-side
argument checks run before any device work (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2212_11675_amd import gsr

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                      "gsr.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gsr_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_expected_entry_points():
    names = declared_functions()
    assert set(names) == set(gsr.EXPORTS), sorted(set(names) ^ set(gsr.EXPORTS))


def test_library_exports_every_declared_symbol():
    lib = gsr.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert lib.gsr_abi_version() == gsr.ABI_VERSION == 4
    assert lib.gsr_status_string(0) == b"ok"
    assert lib.gsr_status_string(-2) == b"matrix layout violated"


def test_host_side_argument_errors():
    lib = gsr.load()
    out = ctypes.c_void_p()
    assert lib.gsr_lsqr_setup(None, None, None, None, None, None, None, ctypes.byref(out)) == -1
    assert b"dims" in lib.gsr_last_error()
    bad = gsr.make_dims(10, 1, 3, 6)  # n_dfa < 4
    assert lib.gsr_lsqr_setup(ctypes.byref(bad), 16, 16, 16, 16, None, None,
                              ctypes.byref(out)) == -1
    assert b"n_dfa" in lib.gsr_last_error()
    bad = gsr.make_dims(10, 1, 4, 5)  # n_instr < 6
    assert lib.gsr_lsqr_setup(ctypes.byref(bad), 16, 16, 16, 16, None, None,
                              ctypes.byref(out)) == -1
    bad = gsr.make_dims(10, 1, 4, 6, 2)  # n_glob must be 1
    assert lib.gsr_lsqr_setup(ctypes.byref(bad), 16, 16, 16, 16, None, None,
                              ctypes.byref(out)) == -6
    ok = gsr.make_dims(10, 1, 4, 6)
    assert lib.gsr_lsqr_setup(ctypes.byref(ok), None, None, None, None, None, None,
                              ctypes.byref(out)) == -1
    assert lib.gsr_lsqr_setup(ctypes.byref(ok), 8, 16, 16, 16, None, None,
                              ctypes.byref(out)) == -1  # vals not 16-byte aligned
    # batched: k outside {1, 2, 4, 8}
    d = (gsr.Dims * 1)(ok)
    ro = (ctypes.c_int64 * 2)(0, 10)
    assert lib.gsr_batch_setup(1, d, ro, 16, 16, 16, 16, 3, None, None, ctypes.byref(out)) == -6
    # null handles are rejected, destroy(NULL) is a no-op
    assert lib.gsr_aprod1(None, 16, 16, None) == -1
    assert lib.gsr_lsqr_solve(None, 16, 16, None, None, None) == -1
    assert lib.gsr_destroy(None) == 0
    assert lib.gsr_batch_destroy(None) == 0


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(gsr, "_lib", None)
    monkeypatch.setattr(gsr, "LIB_PATH", str(tmp_path / "libgsr.so"))
    with pytest.raises(ImportError, match="no CPU fallback"):
        gsr.load()
