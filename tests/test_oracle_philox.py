"""Pin the oracle's Philox4x32-10 to an independent library implementation.

rocRAND's Philox4x32-10 engine (host-compiled from its public header by the
helper in tests/golden/rocrand_philox_pin.cpp) is positioned on an arbitrary
counter via (subsequence, offset); its block must equal the oracle's block for
the same (counter, key).  A wrong multiplier, Weyl constant, word order or key
schedule in the oracle fails this test.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_pin(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND pin")
    exe = tmp_path_factory.mktemp("pin") / "rocrand_pin"
    subprocess.run([hipcc, "-O1", "-o", str(exe), os.path.join(HERE, "golden", "rocrand_philox_pin.cpp")],
                   check=True, capture_output=True)
    return str(exe)


def _rocrand_blocks(exe, rows):
    text = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
    out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
    return np.array([[int(v) for v in line.split()] for line in out.strip().splitlines()],
                    dtype=np.uint64)


def test_philox_matches_rocrand(oracle_lib, rocrand_pin):
    rng = np.random.default_rng(123)
    rows = rng.integers(0, 1 << 32, size=(300, 6), dtype=np.uint64)
    rows[0] = 0
    rows[1] = (1 << 32) - 1
    # counters of the form the lattice uses: (x, t, r, b) with small t, r, b
    rows[2:50, 1:4] = rng.integers(0, 8, size=(48, 3))
    want = _rocrand_blocks(rocrand_pin, rows)
    got = np.array([oracle_lib.philox(r[:4], r[4:]) for r in rows], dtype=np.uint64)
    np.testing.assert_array_equal(got, want)


def test_philox_counter_sensitivity(oracle_lib):
    """Every counter and key word enters the block."""
    base = oracle_lib.philox([5, 6, 7, 8], [9, 10])
    for w in range(4):
        c = [5, 6, 7, 8]
        c[w] += 1
        assert not np.array_equal(oracle_lib.philox(c, [9, 10]), base)
    for w in range(2):
        k = [9, 10]
        k[w] += 1
        assert not np.array_equal(oracle_lib.philox([5, 6, 7, 8], k), base)
