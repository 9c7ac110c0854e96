"""Host-side checks of the C ABI library (no GPU needed, no compute calls):
the library loads and exports every function include/ilg.h declares, the
host-side fixed-point parameters and configuration checks agree with the
oracle's, and the product and the oracle share no code."""
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


def test_fixed_point_host_logic_matches_oracle():
    """ilg_fixed_point (host code, no device call) against the oracle's
    fixed-point parameters, with every draw-specification flag, and the
    configuration checks that reject flags outside their scope."""
    if not os.path.exists(LIB):
        pytest.skip("libilg.so not built")
    import paper_2203_01380_amd as ilg
    from oracle import exact
    for q in (2, 3, 5):
        for omega in (0.05, 0.7, 1.0, 1.3, 1.8, 1.999, 2.0):
            for rounds in (10, 7):
                for ex in ((False, True) if q == 2 else (False,)):
                    cfg = ilg.make_config(q, 64, 2, omega, 1, rounds=rounds, exchange=ex,
                                          height=4 if q == 5 else 0)
                    fx = ilg.fixed_point(cfg)
                    ref = exact.fixed_point_params(omega, q=q)
                    assert fx.flip == int(ref["flip"])
                    assert fx.p == (ref["P_x"] if ex else ref["P"])
                    if q != 2:
                        assert fx.p_rest == ref["P_rest"]
    for bad in (dict(q=3, exchange=True), dict(q=5, exchange=True, height=4)):
        with pytest.raises(ilg.IlgError):
            ilg.fixed_point(ilg.make_config(bad["q"], 64, 2, 1.5, 1, exchange=True,
                                            height=bad.get("height", 0)))
    cfg = ilg.make_config(3, 64, 2, 1.5, 1)
    cfg.flags |= 1 << 6
    with pytest.raises(ilg.IlgError):
        ilg.fixed_point(cfg)
