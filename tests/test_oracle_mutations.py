"""The oracle's pins catch planted mistakes.

Each case copies oracle/ilg_oracle.c to a scratch directory, plants one
plausible mistake by a textual replacement, compiles the copy, and runs the
pin that should catch it in a child pytest process loading that copy
(ILG_ORACLE_LIB).  The pin must fail.  The unmodified oracle passes the same
pins in the rest of the suite.  CPU only."""
import importlib.util
import os
import subprocess
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "ilg_oracle.c")

# (name, original text, planted text, pin that must fail)
C_MUTATIONS = [
    ("hash multiplier", "0xBF58476D1CE4E5B9ull", "0xBF58476D1CE4E5B8ull",
     "test_oracle_lattice.py::test_hash_single_term_is_splitmix64"),
    ("hash shift", "z = (z ^ (z >> 30))", "z = (z ^ (z >> 29))",
     "test_oracle_lattice.py::test_hash_single_term_is_splitmix64"),
    ("hash position word", "(uint64_t)i) << 32) ^ n", "(uint64_t)i) << 31) ^ n",
     "test_oracle_lattice.py::test_hash_matches_definition"),
    ("flip dropped", "a[i] = pp->flip ? n_in[q - 1 - i] : n_in[i];", "a[i] = n_in[i];",
     "test_oracle_lattice.py::test_full_over_relaxation_is_period_two"),
    ("stream direction reversed", "(int64_t)i - 1;", "1 - (int64_t)i;",
     "test_oracle_lattice.py::test_pure_streaming_moves_by_velocity"),
    ("rest and half tables swapped",
     "m[1] = binomial(M, pp->tab_rest, &s);", "m[1] = binomial(M, pp->tab_half, &s);",
     "test_oracle_sampler.py::test_collision_law_exact_enumeration"),
    ("Philox multiplier", "M0 = 0xD2511F53u", "M0 = 0xD2511F55u",
     "test_oracle_philox.py::test_philox_matches_rocrand"),
    ("Philox key increment", "W1 = 0xBB67AE85u", "W1 = 0xBB67AE84u",
     "test_oracle_philox.py::test_philox_matches_rocrand"),
]


def _build_mutant(tmp_path, original, planted):
    text = open(SRC).read()
    assert text.count(original) >= 1, f"mutation target not found: {original!r}"
    src = tmp_path / "ilg_oracle_mutant.c"
    src.write_text(text.replace(original, planted))
    lib = tmp_path / "libilg_oracle_mutant.so"
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-pthread", str(src), "-o",
                    str(lib), "-lm"], check=True, capture_output=True)
    return str(lib)


@pytest.mark.parametrize("name,original,planted,pin", C_MUTATIONS,
                         ids=[m[0].replace(" ", "_") for m in C_MUTATIONS])
def test_planted_oracle_mistake_fails_its_pin(tmp_path, name, original, planted, pin):
    lib = _build_mutant(tmp_path, original, planted)
    env = dict(os.environ, ILG_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu", os.path.join(HERE, pin)],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1, (f"{name}: the pin {pin} did not fail (rc {r.returncode})\n"
                               f"{r.stdout[-2000:]}")
    assert " failed" in r.stdout, r.stdout[-2000:]


def _load(name, path):
    spec = importlib.util.spec_from_file_location(name, path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_planted_moments_sign_fails_its_pin(tmp_path):
    """A flipped current sign in exact.moments_raw fails the hand-computed
    pin (test_oracle_lattice.py::test_moments_raw_hand_computed run against
    the planted copy)."""
    text = open(os.path.join(ROOT, "oracle", "exact.py")).read()
    original = "(vx[:, None] * s).sum(axis=0)"
    assert original in text
    path = tmp_path / "exact_mutant.py"
    path.write_text(text.replace(original, "(-vx[:, None] * s).sum(axis=0)"))
    pins = _load("pins_lattice", os.path.join(HERE, "test_oracle_lattice.py"))
    pins.test_moments_raw_hand_computed()          # the real oracle passes
    pins.exact = _load("exact_mutant", path)
    with pytest.raises(AssertionError):
        pins.test_moments_raw_hand_computed()
