"""GPU parity of the D1Q2 exchange form (draw specification v3, flag
ILG_DRAWS_EXCHANGE) against the oracle run with exchange=True: the
fixed-point crossing probability, every compared step bit-exact over ragged
lengths, both count types, multi-chunk counts, special rates (the zero
collision fraction shares the three-binomial kernel), combined with 7-round
draws, a 2^24-node lattice with light-cone samples, and the rejection of the
flag for q != 2 (plain and serving forms) and in a batch of mixed
specifications (batched parity: test_gpu_batch_specs.py; serving:
test_gpu_serve.py)."""
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


def _run_both(ilg, O, L, cb, omega, init, steps, seed=1, r=0, t0=0, flip="auto", rounds=10,
              check_every=1):
    _say(f"[exchange] L={L} cb={cb} omega={omega} steps={steps} flip={flip} rounds={rounds}")
    p = O.Params(2, omega, flip=flip, rounds=rounds, exchange=True)
    lat = ilg.Lattice(2, L, cb, omega, seed, init, realization=r, t0=t0, flip=flip, rounds=rounds,
                      exchange=True)
    cur = init.copy()
    done = 0
    while done < steps:
        n = min(check_every, steps - done)
        lat.step(n)
        cur, _, ov = O.run(p, cur, n, seed=seed, realization=r, t0=t0 + done)
        assert not ov
        done += n
        got = lat.state()
        if not np.array_equal(got, cur):
            bad = np.argwhere(got != cur)
            raise AssertionError(f"state mismatch after {done} steps at {bad[:5].tolist()}")
    lat.close()
    return cur


def test_crossing_probability(ilg, oracle_lib):
    for omega in [0.3, 0.9, 1.0, 1.25, 1.5, 1.8, 1.999, 2.0]:
        fx = ilg.fixed_point(ilg.make_config(2, 64, 2, omega, 1, exchange=True))
        assert fx.p == oracle_lib.Params(2, omega, exchange=True).P_x


@pytest.mark.parametrize("cb", [2, 4])
@pytest.mark.parametrize("L", [1, 2, 3, 63, 64, 65, 1025, 2049, 10007])
def test_lengths_and_types(ilg, oracle_lib, cb, L):
    init = W.init_poisson_iid(2, L, 30.0, cb, init_seed=L + cb)
    _run_both(ilg, oracle_lib, L, cb, 1.6, init, steps=6, seed=5 + L, r=1)


def test_multi_chunk_counts(ilg, oracle_lib):
    init = W.init_poisson_iid(2, 3000, 150.0, 2, init_seed=41)
    init[:, :40] = 700
    init[0, 40:80] = 0
    _run_both(ilg, oracle_lib, 3000, 2, 1.3, init, steps=6, seed=43, check_every=2)


@pytest.mark.parametrize("omega,flip", [(2.0, "auto"), (1.0, "on"), (1.0, "off"), (0.5, "auto"),
                                        (1.999, "auto"), (0.01, "auto")])
def test_special_rates(ilg, oracle_lib, omega, flip):
    init = W.init_poisson_iid(2, 777, 25.0, 4, init_seed=47)
    _run_both(ilg, oracle_lib, 777, 4, omega, init, steps=8, seed=53, flip=flip)


def test_with_seven_round_draws(ilg, oracle_lib):
    init = W.init_poisson_iid(2, 5000, 40.0, 2, init_seed=59)
    _run_both(ilg, oracle_lib, 5000, 2, 1.7, init, steps=6, seed=61, rounds=7)


def test_full_size_l2_24_lightcone(ilg, oracle_lib):
    """D1Q2, L = 2^24, uint16, Poisson(40), omega = 1.5: one full-lattice step
    against the oracle, then 400 more steps whose light-cone windows the
    oracle recomputes from the initial state."""
    L, T, omega, seed = 1 << 24, 400, 1.5, 3
    init = W.init_poisson_iid(2, L, 40.0, 2, init_seed=67)
    p = oracle_lib.Params(2, omega, exchange=True)
    _say("[exchange full-size] one step")
    lat = ilg.Lattice(2, L, 2, omega, seed, init, exchange=True)
    lat.step(1)
    one, _, _ = oracle_lib.run(p, init, 1, seed=seed)
    np.testing.assert_array_equal(lat.state(), one)
    lat.step(T - 1)
    final = lat.state()
    lat.close()
    assert int(final.astype(np.int64).sum()) == int(init.astype(np.int64).sum())
    width = 2 * T + 256
    for centre in [0, L // 2 + 5, L - 33]:
        x0 = (centre - T) % L
        idx = (x0 + np.arange(width)) % L
        _say(f"[exchange full-size] window at {centre}")
        win, ov = oracle_lib.run_window(p, np.ascontiguousarray(init[:, idx]), L, x0, T, seed=seed)
        assert not ov
        np.testing.assert_array_equal(win[:, T:T + 256], final[:, idx[T:T + 256]])


def test_rejections(ilg):
    with pytest.raises(ilg.IlgError):
        ilg.fixed_point(ilg.make_config(3, 64, 2, 1.5, 1, exchange=True))
    m = dict(q=2, length=64, count_bytes=2, omega=1.5, seed=1, exchange=True)
    init = np.ones((2, 64), dtype=np.uint16)
    with pytest.raises(ilg.IlgError):
        ilg.Batch([m, dict(m, exchange=False)], [init, init])
    srv = ilg.Server(1 << 20, 10)
    try:
        with pytest.raises(ilg.IlgError):
            srv.submit(dict(m, q=3), np.ones((3, 64), dtype=np.uint16), 5)
    finally:
        srv.close()
