"""GPU parity of the plain (single-lattice) form against the CPU oracle.

Bit-exact: every occupation number after every compared step, the per-step
state hash, the fixed-point parameters and the binomial tables.  FP64
diagnostics (A^LG, S(k)) within a tolerance derived from their summation.
"""
import math
import sys

import numpy as np
import pytest

import ilg_workloads as W
from oracle import exact

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


def _run_both(ilg, oracle_lib, q, L, cb, omega, init, steps, seed=1, r=0, t0=0, flip="auto",
              theta=0.0, use_torch=True, check_every=1):
    """Run GPU and oracle side by side, comparing the full state every
    check_every steps and the final state."""
    _say(f"[parity] q={q} L={L} cb={cb} omega={omega} steps={steps} flip={flip} torch={use_torch}")
    p = oracle_lib.Params(q, omega, theta=theta or 1.0 / 3.0, flip=flip)
    lat = ilg.Lattice(q, L, cb, omega, seed, init, realization=r, t0=t0, theta=theta, flip=flip,
                      use_torch=use_torch)
    cur = init.copy()
    done = 0
    while done < steps:
        n = min(check_every, steps - done)
        lat.step(n)
        cur, _, ov = oracle_lib.run(p, cur, n, seed=seed, realization=r, t0=t0 + done)
        assert not ov
        done += n
        got = lat.state()
        if not np.array_equal(got, cur):
            bad = np.argwhere(got != cur)
            raise AssertionError(f"state mismatch after {done} steps at {bad[:5].tolist()} "
                                 f"gpu={got[tuple(bad[0])]} oracle={cur[tuple(bad[0])]}")
    assert lat.t == t0 + steps
    lat.close()
    return cur


def test_fixed_point_parameters_match(ilg):
    for omega in [0.05, 0.5, 0.7, 1.0, 1.0000001, 1.25, 1.5, 1.75, 1.8, 1.9, 1.98, 1.999, 2.0]:
        for theta in [0.0, 0.25, 0.6]:
            for q in [2, 3]:
                cfg = ilg.make_config(q, 16, 2, omega, 1, theta=theta)
                fx = ilg.fixed_point(cfg)
                want = exact.fixed_point_params(omega, theta or 1.0 / 3.0)
                assert fx.flip == int(want["flip"])
                assert fx.p == want["P"]
                assert fx.p_half == want["P_half"]
                if q == 3:
                    assert fx.p_rest == want["P_rest"]


@pytest.mark.parametrize("P", [1, 12345, 85899346, 858993459, 1 << 31, 2863311531,
                               (1 << 32) - 1, 1 << 32])
def test_tables_byte_equal(ilg, P):
    np.testing.assert_array_equal(ilg.binomial_table(P), exact.binomial_table(P))


def test_config1_d1q2_l256_every_step_hash(ilg, oracle_lib):
    """D1Q2, L = 256, uint32, rounded sine split evenly, omega = 1.5, seed 1:
    the GPU hash equals the oracle hash after each of the 1000 steps and the
    states are equal at steps 1, 2, 10 and 1000."""
    spec, init = W.workload_d1q2_l256()
    p = oracle_lib.Params(2, spec.omega)
    _, hashes, ov = oracle_lib.run(p, init, spec.steps, seed=spec.seed, hashes=True)
    assert not ov
    lat = ilg.Lattice(2, spec.length, 4, spec.omega, spec.seed, init)
    cur = init
    for t in range(spec.steps):
        lat.step(1)
        assert lat.hash() == int(hashes[t]), f"hash mismatch after step {t + 1}"
        if t + 1 in (1, 2, 10, spec.steps):
            cur, _, _ = oracle_lib.run(p, init, t + 1, seed=spec.seed)
            np.testing.assert_array_equal(lat.state(), cur)
    m = lat.moments()
    assert m["mass"] == 5120 and m["step"] == spec.steps
    lat.close()


@pytest.mark.parametrize("q,cb", [(2, 2), (2, 4), (3, 2), (3, 4)])
@pytest.mark.parametrize("L", [1, 2, 3, 5, 63, 64, 65, 2047, 2048, 2049, 10007])
def test_lengths_and_types(ilg, oracle_lib, q, cb, L):
    init = W.init_poisson_iid(q, L, 30.0, cb, init_seed=L + 17 * q + cb)
    _run_both(ilg, oracle_lib, q, L, cb, 1.7, init, steps=6, seed=3 + L, r=2)


@pytest.mark.parametrize("q", [2, 3])
def test_multi_chunk_counts(ilg, oracle_lib, q):
    """Occupations above 64 and 128 exercise multi-chunk binomials and Philox
    blocks beyond the ones computed up front."""
    init = W.init_poisson_iid(q, 3000, 150.0, 2, init_seed=9)
    init[:, :40] = 700      # very large counts: many chunks, many blocks
    _run_both(ilg, oracle_lib, q, 3000, 2, 1.3, init, steps=8, seed=11, check_every=2)


@pytest.mark.parametrize("cb,omega", [(2, 1.8), (4, 1.3), (2, 2.0), (4, 0.7)])
def test_mixed_middle_chunk_layouts(ilg, oracle_lib, cb, omega):
    """D1Q3 wavefronts whose middle removal binomial needs one, two or three
    chunks depending on the lane (rest counts around 64, 128 and 192, with the
    edges 64/65, 128/129, 192/193), outer counts 1..40: each block of 64
    nodes gets one layout mix (uniform, two/three chunks, one/two/three, one/two,
    edge values, beyond three chunks).  Rest particles do not stream, so the
    mixes persist over the compared steps."""
    rng = np.random.default_rng(31 + cb)
    nblk = 60
    L = 64 * nblk + 17
    dt = np.uint16 if cb == 2 else np.uint32
    init = np.empty((3, L), dtype=dt)
    init[0] = rng.integers(1, 41, L)
    init[2] = rng.integers(1, 41, L)
    mids = []
    for b in range(nblk + 1):
        mode = b % 6
        if mode == 0:
            v = rng.integers(65, 129, 64)
        elif mode == 1:
            v = rng.integers(65, 193, 64)
        elif mode == 2:
            v = rng.integers(1, 193, 64)
        elif mode == 3:
            v = rng.integers(1, 129, 64)
        elif mode == 4:
            v = rng.choice([1, 63, 64, 65, 127, 128, 129, 191, 192], 64)
        else:
            v = rng.integers(100, 260, 64)
        mids.append(v)
    init[1] = np.concatenate(mids)[:L]
    _run_both(ilg, oracle_lib, 3, L, cb, omega, init, steps=6, seed=13)


@pytest.mark.parametrize("cb,omega", [(2, 1.8), (4, 1.5), (2, 1.0), (4, 0.6)])
def test_two_chunk_outer_layouts(ilg, oracle_lib, cb, omega):
    """D1Q3 wavefronts whose three counts all lie in 1..128 with some outer
    count above 64 (each removal binomial one or two chunks, its draws
    shifted per lane): blocks of 64 nodes with every count two chunks, every
    count random in 1..128, the edges 1/63/64/65/127/128, only the outer
    counts above 64, and a block with one count beyond 128 (the generic
    path).  omega 1.0 and 0.6 collide most particles, so M exceeds one
    chunk and the redistribution goes on from each lane's own word."""
    rng = np.random.default_rng(57 + cb)
    nblk = 50
    L = 64 * nblk + 33
    dt = np.uint16 if cb == 2 else np.uint32
    cols = []
    for b in range(nblk + 1):
        mode = b % 5
        if mode == 0:
            v = rng.integers(65, 129, (3, 64))
        elif mode == 1:
            v = rng.integers(1, 129, (3, 64))
        elif mode == 2:
            v = rng.choice([1, 63, 64, 65, 127, 128], (3, 64))
        elif mode == 3:
            v = np.stack([rng.integers(65, 129, 64), rng.integers(1, 65, 64),
                          rng.integers(65, 129, 64)])
        else:
            v = rng.integers(65, 129, (3, 64))
            v[rng.integers(0, 3), rng.integers(0, 64)] = 129 + rng.integers(0, 100)
        cols.append(v)
    init = np.concatenate(cols, axis=1)[:, :L].astype(dt)
    _run_both(ilg, oracle_lib, 3, L, cb, omega, init, steps=6, seed=19)


@pytest.mark.parametrize("q,omega,theta,mean", [(2, 1.0, 0.0, 60.0), (2, 1.1, 0.0, 60.0),
                                                 (3, 1.0, 0.0, 60.0), (3, 0.9, 0.0, 45.0),
                                                 (3, 1.05, 0.9, 40.0), (3, 1.0, 0.0, 95.0),
                                                 (3, 1.2, 0.0, 70.0)])
def test_multi_chunk_redistribution(ilg, oracle_lib, q, omega, theta, mean):
    """Collision fractions near one remove most particles, so M = sum k_i spans
    one to three chunks (and beyond three for mean 95); theta = 0.9 leaves
    R = M - m_1 above one chunk.  Every lane layout of the redistribution
    draws is compared with the oracle."""
    init = W.init_poisson_iid(q, 5000, mean, 2, init_seed=int(mean) + 7 * q)
    _run_both(ilg, oracle_lib, q, 5000, 2, omega, init, steps=6, seed=17, theta=theta)


@pytest.mark.parametrize("q,omega,flip", [(3, 2.0, "auto"), (2, 2.0, "auto"), (3, 1.0, "on"),
                                          (3, 1.0, "off"), (2, 0.5, "auto"), (3, 0.3, "auto"),
                                          (3, 1.999, "auto"), (2, 0.01, "auto")])
def test_special_rates(ilg, oracle_lib, q, omega, flip):
    init = W.init_poisson_iid(q, 777, 25.0, 4, init_seed=21)
    _run_both(ilg, oracle_lib, q, 777, 4, omega, init, steps=10, seed=5, flip=flip)


def test_full_over_relaxation_period_two_gpu(ilg):
    init = W.init_poisson_iid(3, 5000, 40.0, 2, init_seed=4)
    lat = ilg.Lattice(3, 5000, 2, 2.0, 9, init)
    for _ in range(5):
        lat.step(2)
        np.testing.assert_array_equal(lat.state(), init)
    lat.close()


def test_flip_moot_gpu(ilg):
    init = W.init_poisson_iid(3, 4096, 40.0, 2, init_seed=5)
    a = ilg.Lattice(3, 4096, 2, 1.0, 3, init, flip="on")
    b = ilg.Lattice(3, 4096, 2, 1.0, 3, init, flip="off")
    a.step(20)
    b.step(20)
    np.testing.assert_array_equal(a.state(), b.state())
    a.close()
    b.close()


def test_theta_parameter(ilg, oracle_lib):
    init = W.init_poisson_iid(3, 1500, 40.0, 2, init_seed=6)
    _run_both(ilg, oracle_lib, 3, 1500, 2, 1.6, init, steps=5, theta=0.25)


def test_library_allocated_path(ilg, oracle_lib):
    init = W.init_poisson_iid(3, 3333, 50.0, 2, init_seed=7)
    _run_both(ilg, oracle_lib, 3, 3333, 2, 1.8, init, steps=5, use_torch=False)


def test_large_t0_and_realization(ilg, oracle_lib):
    init = W.init_poisson_iid(2, 999, 30.0, 2, init_seed=8)
    _run_both(ilg, oracle_lib, 2, 999, 2, 1.4, init, steps=4, seed=(1 << 40) + 77,
              r=123456, t0=(1 << 32) - 10)


def test_step_range_error(ilg):
    init = W.init_poisson_iid(2, 64, 10.0, 2, init_seed=1)
    lat = ilg.Lattice(2, 64, 2, 1.4, 1, init, t0=(1 << 32) - 2)
    lat.step(2)
    with pytest.raises(ilg.IlgError) as e:
        lat.step(1)
    assert e.value.code == -5
    lat.close()


def test_overflow_is_reported(ilg):
    init = np.full((3, 256), 60000, dtype=np.uint16)
    lat = ilg.Lattice(3, 256, 2, 1.0, 1, init)
    lat.step(1)
    with pytest.raises(ilg.IlgError) as e:
        lat.state()
    assert e.value.code == -4
    with pytest.raises(ilg.IlgError) as e:
        lat.close()   # destroy reports the sticky error too, and frees the handle
    assert e.value.code == -4


def test_invalid_configs_rejected(ilg):
    init = np.zeros((2, 8), dtype=np.uint16)
    for kw in [dict(omega=0.0), dict(omega=2.5), dict(omega=1.5, flip="off"),
               dict(omega=0.5, flip="on")]:
        with pytest.raises(ilg.IlgError):
            ilg.Lattice(2, 8, 2, kw.pop("omega"), 1, init, **kw)
    with pytest.raises(ilg.IlgError):
        ilg.Lattice(3, 8, 2, 1.5, 1, np.zeros((3, 8), np.uint16), theta=1.5)


def test_checkpoint_resume(ilg, oracle_lib):
    init = W.init_poisson_iid(3, 4321, 50.0, 2, init_seed=10)
    a = ilg.Lattice(3, 4321, 2, 1.8, 7, init)
    a.step(30)
    straight = a.state()
    b = ilg.Lattice(3, 4321, 2, 1.8, 7, init)
    b.step(12)
    ck, t = b.state(), b.t
    b.close()
    c = ilg.Lattice(3, 4321, 2, 1.8, 7, ck, t0=t)
    c.step(18)
    np.testing.assert_array_equal(c.state(), straight)
    d = ilg.Lattice(3, 4321, 2, 1.8, 7, init)
    d.set_state(ck, t)
    d.step(18)
    np.testing.assert_array_equal(d.state(), straight)
    for x in (a, c, d):
        x.close()


@pytest.mark.parametrize("q,cb,L", [(3, 2, 320), (2, 4, 4099), (3, 4, 70001)])
def test_diagnostics(ilg, oracle_lib, q, cb, L):
    w = W.D1Q3_WEIGHTS if q == 3 else W.D1Q2_WEIGHTS
    init = W.init_poisson_sine(w, L, 100.0, 60.0, cb, init_seed=L)
    lat = ilg.Lattice(q, L, cb, 1.5, 2, init)
    lat.step(3)
    p = oracle_lib.Params(q, 1.5)
    ref, _, _ = oracle_lib.run(p, init, 3, seed=2)
    m = lat.moments(per_node=True, nk=16)
    rho, j, e = exact.moments_raw(ref, q)
    np.testing.assert_array_equal(m["rho"], rho)
    np.testing.assert_array_equal(m["j"], j)
    np.testing.assert_array_equal(m["e"], e)
    assert m["mass"] == int(rho.sum())
    assert m["hash"] == oracle_lib.state_hash(ref) == lat.hash()
    # FP64 sums of L terms of size <= N: relative error bounded by ~L * 2^-52
    # against the scale sum_x N(x); 1e-9 leaves a wide margin.
    N = rho.astype(np.float64)
    scale = N.sum() / (L / 2.0)
    assert abs(m["amplitude"] - exact.amplitude_lg(rho)) <= 1e-9 * max(scale, 1.0)
    Sk = exact.structure_factor(rho, 16)
    np.testing.assert_allclose(m["sk"], Sk, rtol=1e-8, atol=1e-9 * N.sum())
    lat.close()
