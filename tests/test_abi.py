"""The C ABI boundary: the built library loads without a GPU and exports every
function that include/rnamg.h declares; the Python binding's signature table
names exactly those functions.  The oracle library likewise exports what
oracle/oracle.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DECL = re.compile(r"^[A-Za-z_][A-Za-z0-9_ ]*?\**\s*\b((?:rn|orc)_[a-z0-9_]+)\s*\(", re.M)


def declared(header):
    text = open(os.path.join(ROOT, header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return sorted(set(DECL.findall(text)))


def test_header_declares_the_entry_points():
    names = declared("include/rnamg.h")
    for want in ("rn_create", "rn_destroy", "rn_strength", "rn_pattern", "rn_tentative", "rn_transpose",
                 "rn_plan_create", "rn_masked_product", "rn_energy_min", "rn_energy_min_bwd",
                 "rn_aggregate_host"):
        assert want in names


def test_library_exports_every_declared_symbol():
    from paper_1610_03154_amd import _lib
    path = _lib.LIB_PATH
    if not os.path.exists(path):
        pytest.fail("librnamg.so is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    missing = [n for n in declared("include/rnamg.h") if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signatures_match_header():
    from paper_1610_03154_amd import _lib
    assert sorted(_lib.SIGNATURES) == declared("include/rnamg.h")


def test_oracle_exports_every_declared_symbol():
    import oracle
    lib = oracle.lib()
    missing = [n for n in declared("oracle/oracle.h") if not hasattr(lib, n)]
    assert not missing, missing


def test_version_string_without_gpu():
    from paper_1610_03154_amd import _lib
    lib = ctypes.CDLL(_lib.LIB_PATH)
    lib.rn_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.rn_version()
