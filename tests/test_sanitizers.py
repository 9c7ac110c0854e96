"""Sanitizer builds of the host code (CPU only): the oracle under
AddressSanitizer + UndefinedBehaviorSanitizer and under ThreadSanitizer
(its node-range threads), the serving scheduler under ASan + UBSan.  Each
build must run clean and, for the oracle, reproduce the plain build's hash."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import exact

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HARN = os.path.join(ROOT, "tests", "harness")
CSRC = os.path.join(ROOT, "paper_2203_01380_amd", "csrc")
ORACLE_C = os.path.join(ROOT, "oracle", "ilg_oracle.c")


def _cc(name):
    exe = shutil.which(name)
    if not exe:
        pytest.skip(f"{name} not available")
    return exe


@pytest.fixture(scope="module")
def tables(tmp_path_factory):
    d = tmp_path_factory.mktemp("san")
    p = exact.fixed_point_params(1.7)
    tabs = np.concatenate([exact.binomial_table(p["P"]), exact.binomial_table(p["P_half"]),
                           exact.binomial_table(p["P_rest"])]).astype(np.uint32)
    path = d / "tables.bin"
    tabs.tofile(path)
    return d, str(path)


def _build_oracle(d, flags, tag):
    exe = str(d / f"oracle_{tag}")
    subprocess.run([_cc("gcc"), "-O1", "-g", "-std=c11", "-pthread", *flags,
                    os.path.join(HARN, "oracle_driver.c"), ORACLE_C, "-o", exe], check=True)
    return exe


def _run(exe, args, env_extra=None):
    env = dict(os.environ)
    env.pop("LD_PRELOAD", None)
    env.update(env_extra or {})
    return subprocess.run([exe, *args], capture_output=True, text=True, env=env, timeout=300)


@pytest.mark.parametrize("q,flip", [(3, 1), (2, 0)])
def test_oracle_asan_ubsan_and_tsan(tables, q, flip):
    d, tab = tables
    args = [tab, str(q), "997", "40", str(flip), "4", "77"]
    plain = _run(_build_oracle(d, [], "plain"), args)
    assert plain.returncode == 0, plain.stderr
    asan = _run(_build_oracle(d, ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
                              "asan"), args, {"ASAN_OPTIONS": "detect_leaks=1"})
    assert asan.returncode == 0, asan.stderr
    assert asan.stdout == plain.stdout
    tsan = _run(_build_oracle(d, ["-fsanitize=thread"], "tsan"), args,
                {"TSAN_OPTIONS": "halt_on_error=1"})
    if "FATAL: ThreadSanitizer: unexpected memory mapping" in tsan.stderr:
        pytest.skip("ThreadSanitizer cannot map memory in this environment")
    assert tsan.returncode == 0, tsan.stderr
    assert tsan.stdout == plain.stdout


def test_scheduler_asan_ubsan(tmp_path):
    exe = str(tmp_path / "sched_asan")
    subprocess.run([_cc("g++"), "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-I", CSRC,
                    os.path.join(HARN, "sched_driver.cpp"), os.path.join(HARN, "sched_harness.cpp"),
                    os.path.join(CSRC, "scheduler.cpp"), "-o", exe], check=True)
    r = _run(exe, [], {"ASAN_OPTIONS": "detect_leaks=1"})
    assert r.returncode == 0, r.stdout + r.stderr
