"""Host-side checks of the C ABI library (no GPU needed, no compute calls):
the library loads and exports every function include/ilg.h declares, and the
product and the oracle share no code."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ilg.h")
LIB = os.path.join(ROOT, "paper_2203_01380_amd", "libilg.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w \*]*?\b(ilg_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_core_calls():
    names = declared_functions()
    for core in ["ilg_create", "ilg_step", "ilg_moments", "ilg_destroy", "ilg_last_error"]:
        assert core in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("libilg.so not built")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def _sources(dirname, exts):
    out = []
    for base, _, files in os.walk(os.path.join(ROOT, dirname)):
        if "_build" in base or "__pycache__" in base:
            continue
        out += [os.path.join(base, f) for f in files if f.endswith(exts)]
    return out


def test_product_and_oracle_share_no_code():
    prod = _sources("paper_2203_01380_amd", (".py", ".cpp", ".hip", ".h"))
    orc = _sources("oracle", (".py", ".c", ".h"))
    assert prod and orc
    for f in prod:
        text = open(f).read()
        assert not re.search(r"^\s*(from|import)\s+oracle\b", text, flags=re.M), f
        assert not re.search(r"#include\s+[<\"].*oracle", text), f
    for f in orc:
        text = open(f).read()
        assert not re.search(r"^\s*(from|import)\s+paper_2203_01380_amd", text, flags=re.M), f
        assert not re.search(r"#include\s+[<\"](ilg|philox|ilg_internal)", text), f
