"""Exact lattice-level pins of the oracle: conservation, the omega^j = 2 and
omega* = 1 special cases, streaming direction, window runs and overflow."""
import numpy as np
import pytest

import ilg_workloads as W
from oracle import exact


def _params(oracle_lib, q, omega, flip="auto"):
    return oracle_lib.Params(q, omega, flip=flip)


@pytest.mark.parametrize("q,omega,cb", [(2, 1.5, 4), (3, 1.8, 2), (3, 0.6, 2), (2, 1.95, 2)])
def test_mass_conserved_every_step(oracle_lib, q, omega, cb):
    """sum_i Xi_i = 0: the total count never changes (Integer Lattice Gas section)."""
    st = W.init_poisson_iid(q, 97, 40.0, cb, init_seed=1)
    p = _params(oracle_lib, q, omega)
    m0 = int(st.astype(np.int64).sum())
    cur = st
    for t in range(30):
        cur, _, ov = oracle_lib.run(p, cur, 1, seed=7, t0=t)
        assert not ov
        assert int(cur.astype(np.int64).sum()) == m0


@pytest.mark.parametrize("q", [2, 3])
def test_full_over_relaxation_is_period_two(oracle_lib, q):
    """omega^j = 2 (omega* = 0): flip and streaming only, so every particle
    returns after two steps and the system does not evolve (Results section)."""
    st = W.init_poisson_iid(q, 50, 20.0, 4, init_seed=3)
    p = _params(oracle_lib, q, 2.0)
    assert p.P == 0 and p.flip
    cur = st
    for t in range(0, 20, 2):
        nxt, _, _ = oracle_lib.run(p, cur, 1, seed=1, t0=t)
        assert not np.array_equal(nxt, cur)
        cur, _, _ = oracle_lib.run(p, nxt, 1, seed=1, t0=t + 1)
        np.testing.assert_array_equal(cur, st)


@pytest.mark.parametrize("q", [2, 3])
def test_flip_moot_lattice(oracle_lib, q):
    """omega* = 1 with and without the flip give bit-identical runs."""
    st = W.init_poisson_iid(q, 64, 30.0, 4, init_seed=4)
    a, ha, _ = oracle_lib.run(_params(oracle_lib, q, 1.0, "on"), st, 25, seed=9, hashes=True)
    b, hb, _ = oracle_lib.run(_params(oracle_lib, q, 1.0, "off"), st, 25, seed=9, hashes=True)
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(ha, hb)


@pytest.mark.parametrize("q", [2, 3])
def test_pure_streaming_moves_by_velocity(oracle_lib, q):
    """With no collision and no flip each population moves by v_i per step:
    n_i(x + v_i t, t) = n_i(x, 0)  (left side of Eq. ilgeq)."""
    st = W.init_poisson_iid(q, 41, 10.0, 4, init_seed=5)
    p = _params(oracle_lib, q, 0.5)
    p.tab_p = None       # P = 0
    p.flip = False
    out, _, _ = oracle_lib.run(p, st, 7, seed=1)
    for i, v in enumerate(exact.velocities(q)):
        np.testing.assert_array_equal(out[i], np.roll(st[i], 7 * int(v)))


def test_window_run_matches_periodic(oracle_lib):
    """A light-cone window reproduces the periodic lattice on its valid interior,
    including windows that wrap around x = 0."""
    q, L, T = 3, 300, 20
    st = W.init_poisson_iid(q, L, 50.0, 2, init_seed=6)
    p = _params(oracle_lib, q, 1.7)
    full, _, _ = oracle_lib.run(p, st, T, seed=3, t0=5)
    for x0 in [0, 100, 280]:
        width = 2 * T + 40
        idx = (x0 + np.arange(width)) % L
        win, _ = oracle_lib.run_window(p, st[:, idx], L, x0, T, seed=3, t0=5)
        np.testing.assert_array_equal(win[:, T:width - T], full[:, idx[T:width - T]])


def test_hash_properties(oracle_lib):
    st = W.init_poisson_iid(3, 128, 30.0, 2, init_seed=7)
    h = oracle_lib.state_hash(st)
    assert h == oracle_lib.state_hash(st.copy())
    for i, x in [(0, 0), (1, 64), (2, 127)]:
        s2 = st.copy()
        s2[i, x] += 1
        assert oracle_lib.state_hash(s2) != h
    # a swap of two entries changes it too (positions are mixed in)
    s3 = st.copy()
    s3[0, 3], s3[0, 4] = st[0, 4], st[0, 3]
    if st[0, 3] != st[0, 4]:
        assert oracle_lib.state_hash(s3) != h


def test_overflow_detected(oracle_lib):
    st = np.full((3, 16), 60000, dtype=np.uint16)
    p = _params(oracle_lib, 3, 1.0)
    _, _, ov = oracle_lib.run(p, st, 1, seed=1)
    assert ov


def test_config_one_initial_state():
    spec, st = W.workload_d1q2_l256()
    rho = st.astype(np.int64).sum(axis=0)
    assert int(rho.sum()) == 5120
    assert int((rho % 2).sum()) == 112
    assert np.all(st[1].astype(np.int64) - st[0] == rho % 2)
