"""The C-ABI library loads and exports every symbol include/eg.h declares (no
compute calls: this runs without a GPU)."""

import ctypes
import os
import re

import paper_1807_01151_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "eg.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(eg_[a-z0-9_]+)\s*\(", txt)))


def test_header_and_binding_agree():
    assert declared_symbols() == sorted(P.EXPORTED_SYMBOLS)


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(P.library_path())
    for s in declared_symbols():
        assert hasattr(L, s), s


def test_library_is_gfx950_code_object():
    data = open(P.library_path(), "rb").read()
    assert b"gfx950" in data
