"""CPU checks of the C-ABI library: it loads and exports every symbol the header
declares; host-side planning helpers behave. No GPU compute is called."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ecc.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ecc_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("ecc_create", "ecc_destroy", "ecc_filter_plan_create", "ecc_extended",
              "ecc_match_rotations", "ecc_scale_smooth", "ecc_extended_backward",
              "ecc_workspace_size", "ecc_last_error"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    from paper_2006_13188_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libecc.so is not built (run python -m paper_2006_13188_amd.build)")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    # the binding covers the same names
    assert set(declared_symbols()) <= set(_lib.exported_symbols())


def test_status_strings_without_device():
    from paper_2006_13188_amd import _lib
    lib = _lib.load()
    assert lib.ecc_status_string(0) == b"ok"
    assert lib.ecc_status_string(1) == b"invalid argument"
    assert lib.ecc_last_error(None) == b""
