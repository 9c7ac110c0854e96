"""GPU parity of draw specification v2 (7-round Philox draws, flag
ILG_DRAWS_PHILOX7) against the oracle run with rounds = 7: every compared
step bit-exact for D1Q2, D1Q3 and D2Q5, both count types, ragged lengths,
multi-chunk counts (Philox blocks drawn on demand), special rates (the zero
collision fraction shares the 10-round kernel), a full 2^24-node D1Q3 lattice
in the benchmark's launch configuration with light-cone samples, and the
rejection of mixed specifications in a batch (batched parity:
test_gpu_batch_specs.py; serving: test_gpu_serve.py)."""
import sys

import numpy as np
import pytest

import ilg_workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ilg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2203_01380_amd as ilg
    return ilg


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run_both(ilg, O, q, L, cb, omega, init, steps, seed=1, r=0, t0=0, flip="auto", theta=0.0,
              height=0, check_every=1):
    _say(f"[philox7] q={q} L={L} h={height} cb={cb} omega={omega} steps={steps} flip={flip}")
    p = O.Params(q, omega, theta=theta or 1.0 / 3.0, flip=flip, rounds=7)
    lat = ilg.Lattice(q, L, cb, omega, seed, init, realization=r, t0=t0, theta=theta, flip=flip,
                      height=height, rounds=7)
    cur = init.copy()
    done = 0
    while done < steps:
        n = min(check_every, steps - done)
        lat.step(n)
        if q == 5:
            cur, _, ov = O.run2d(p, cur, n, seed=seed, realization=r, t0=t0 + done)
        else:
            cur, _, ov = O.run(p, cur, n, seed=seed, realization=r, t0=t0 + done)
        assert not ov
        done += n
        got = lat.state()
        if not np.array_equal(got, cur):
            bad = np.argwhere(got != cur)
            raise AssertionError(f"state mismatch after {done} steps at {bad[:5].tolist()}")
    lat.close()
    return cur


def test_flag_accepted_and_fixed_point_unchanged(ilg):
    a = ilg.fixed_point(ilg.make_config(3, 100, 2, 1.7, 1))
    b = ilg.fixed_point(ilg.make_config(3, 100, 2, 1.7, 1, rounds=7))
    assert (a.flip, a.p, a.p_half, a.p_rest) == (b.flip, b.p, b.p_half, b.p_rest)
    with pytest.raises(ValueError):
        ilg.make_config(3, 100, 2, 1.7, 1, rounds=8)


@pytest.mark.parametrize("q,cb", [(2, 2), (2, 4), (3, 2), (3, 4)])
@pytest.mark.parametrize("L", [1, 3, 64, 1025, 2049, 10007])
def test_lengths_and_types(ilg, oracle_lib, q, cb, L):
    init = W.init_poisson_iid(q, L, 30.0, cb, init_seed=L + 5 * q + cb)
    _run_both(ilg, oracle_lib, q, L, cb, 1.7, init, steps=5, seed=7 + L, r=3)


@pytest.mark.parametrize("q", [2, 3])
def test_multi_chunk_counts(ilg, oracle_lib, q):
    init = W.init_poisson_iid(q, 3000, 150.0, 2, init_seed=19)
    init[:, :40] = 700
    _run_both(ilg, oracle_lib, q, 3000, 2, 1.3, init, steps=6, seed=23, check_every=2)


@pytest.mark.parametrize("q,omega,flip", [(3, 2.0, "auto"), (2, 2.0, "auto"), (3, 1.0, "on"),
                                          (3, 1.0, "off"), (2, 0.5, "auto"), (3, 1.999, "auto")])
def test_special_rates(ilg, oracle_lib, q, omega, flip):
    init = W.init_poisson_iid(q, 777, 25.0, 4, init_seed=29)
    _run_both(ilg, oracle_lib, q, 777, 4, omega, init, steps=8, seed=31, flip=flip)


def test_mixed_middle_chunk_layouts(ilg, oracle_lib):
    rng = np.random.default_rng(37)
    L = 64 * 40 + 9
    init = rng.integers(1, 41, size=(3, L)).astype(np.uint16)
    init[1] = rng.choice([1, 63, 64, 65, 127, 128, 129, 191, 192, 250], L)
    _run_both(ilg, oracle_lib, 3, L, 2, 1.8, init, steps=5, seed=41)


@pytest.mark.parametrize("lx,ly,cb", [(1, 1, 2), (33, 7, 4), (1000, 33, 2)])
def test_d2q5(ilg, oracle_lib, lx, ly, cb):
    rng = np.random.default_rng(lx + ly)
    dt = np.uint16 if cb == 2 else np.uint32
    init = rng.poisson(25.0, size=(5, ly, lx)).astype(dt)
    init[2, :2] = rng.choice([1, 64, 65, 128, 129, 150], size=(min(2, ly), lx))
    _run_both(ilg, oracle_lib, 5, lx, cb, 1.6, init, steps=5, seed=43, height=ly)


def test_differs_from_ten_rounds(ilg):
    init = W.init_poisson_iid(3, 4096, 40.0, 2, init_seed=47)
    a = ilg.Lattice(3, 4096, 2, 1.8, 5, init)
    b = ilg.Lattice(3, 4096, 2, 1.8, 5, init, rounds=7)
    a.step(3)
    b.step(3)
    sa, sb = a.state(), b.state()
    a.close()
    b.close()
    assert (sa != sb).mean() > 0.5
    assert int(sb.astype(np.int64).sum()) == int(init.astype(np.int64).sum())


def test_full_size_d1q3_l2_24_lightcone(ilg, oracle_lib):
    """D1Q3, L = 2^24, uint16, Poisson(50), omega = 1.8, with 7-round draws:
    one full-lattice step against the oracle, then 500 more steps whose
    light-cone windows the oracle recomputes from the initial state."""
    spec, init = W.workload_d1q3_big()
    L, T = spec.length, 500
    p = oracle_lib.Params(3, spec.omega, rounds=7)
    _say("[philox7 full-size] one step")
    lat = ilg.Lattice(3, L, 2, spec.omega, spec.seed, init, rounds=7)
    lat.step(1)
    one, _, _ = oracle_lib.run(p, init, 1, seed=spec.seed)
    np.testing.assert_array_equal(lat.state(), one)
    lat.step(T - 1)
    final = lat.state()
    lat.close()
    assert int(final.astype(np.int64).sum()) == int(init.astype(np.int64).sum())
    width = 2 * T + 256
    for centre in [0, L // 3, L - 77]:
        x0 = (centre - T) % L
        idx = (x0 + np.arange(width)) % L
        _say(f"[philox7 full-size] window at {centre}")
        win, ov = oracle_lib.run_window(p, np.ascontiguousarray(init[:, idx]), L, x0, T,
                                        seed=spec.seed)
        assert not ov
        np.testing.assert_array_equal(win[:, T:T + 256], final[:, idx[T:T + 256]])


def test_batch_needs_one_spec(ilg):
    m = dict(q=3, length=64, count_bytes=2, omega=1.5, seed=1, rounds=7)
    init = np.ones((3, 64), dtype=np.uint16)
    with pytest.raises(ilg.IlgError):
        ilg.Batch([m, dict(m, rounds=10)], [init, init])
