"""The C-ABI library loads and exports every symbol that include/dftpp.h
declares; the binding declares nothing the header lacks (CPU only, no
compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dftpp.h")


def header_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dpp_[A-Za-z0-9_]+)\s*\(", text)))


def test_header_parses():
    syms = header_symbols()
    assert "dpp_apply_H" in syms and "dpp_I" in syms and len(syms) > 30


def test_library_exports_every_header_symbol():
    from paper_1708_03621_amd import dftpp
    lib = dftpp.load()
    missing = [s for s in header_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_matches_header():
    from paper_1708_03621_amd import dftpp
    hs = set(header_symbols())
    assert set(dftpp.exported_symbols()) <= hs
    assert hs <= set(dftpp.exported_symbols())


def test_version_and_error_text():
    from paper_1708_03621_amd import dftpp
    lib = dftpp.load()
    assert lib.dpp_version() >= 1
    # a host-side argument check fails without touching a device
    with pytest.raises(dftpp.DppError) as e:
        dftpp.dpp_grid_info(None)
    assert "null grid" in str(e.value)
