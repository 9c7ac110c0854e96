"""GPU parity of the batched ensemble form under draw specifications v2
(7-round Philox) and v3 (the D1Q2 exchange form, with 10- or 7-round draws):
ragged members of every length with rates on both sides of one (including
omega = 2 and omega = 1), start steps, both count types, every member
bit-exact against the oracle after two graph runs; every workgroup shape
gives the same bits; the S(k) and A^LG diagnostics follow the oracle."""
import sys
from concurrent.futures import ThreadPoolExecutor

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


def _oracle_member(O, m, init, nsteps, sk_every=0, nk=0, amp_every=0):
    p = O.Params(m["q"], m["omega"], rounds=m["rounds"], exchange=m["exchange"])
    cur, t, end = init, m["t0"], m["t0"] + nsteps
    sk, nsk, amps = np.zeros(nk), 0, []
    every = [e for e in (sk_every, amp_every) if e]
    while t < end:
        nxt = end
        for e in every:
            nxt = min(nxt, (t // e + 1) * e)
        cur, _, ov = O.run(p, cur, nxt - t, seed=m["seed"], realization=m["realization"], t0=t,
                           nthreads=1)
        assert not ov
        t = nxt
        N = cur.astype(np.int64).sum(axis=0)
        if sk_every and t % sk_every == 0:
            sk += exact.structure_factor(N, nk)
            nsk += 1
        if amp_every and t % amp_every == 0:
            amps.append(exact.amplitude_lg(N))
    return cur, sk, nsk, np.array(amps)


def _members(q, cb, n, seed, rounds, exchange):
    rng = np.random.default_rng(seed)
    lens = [1, 2, 3, 63, 64, 65, 1025, 3000] + list(rng.integers(4, 900, size=n - 8))
    omegas = [2.0, 1.0, 0.5, 1.5, 1.98, 0.9]
    members, inits = [], []
    for r, L in enumerate(lens):
        om = omegas[r] if r < len(omegas) else float(rng.uniform(0.3, 2.0))
        members.append(dict(q=q, length=int(L), count_bytes=cb, omega=om, seed=7000 + r,
                            realization=r * 3, t0=int(rng.integers(0, 500)), rounds=rounds,
                            exchange=exchange))
        inits.append(W.init_poisson_iid(q, int(L), 35.0, cb, init_seed=9100 + r))
    # a few members with counts past one chunk
    inits[7][:, :50] = 150
    return members, inits


SPECS = [(2, 2, 7, False), (2, 4, 7, False), (3, 2, 7, False), (3, 4, 7, False),
         (2, 2, 10, True), (2, 4, 10, True), (2, 2, 7, True)]


@pytest.mark.parametrize("q,cb,rounds,exchange", SPECS)
def test_ragged_members_exact(ilg, oracle_lib, q, cb, rounds, exchange):
    members, inits = _members(q, cb, 30, 31 * q + cb + rounds + 5 * exchange, rounds, exchange)
    _say(f"[batch specs] q={q} cb={cb} rounds={rounds} exchange={exchange}")
    b = ilg.Batch(members, inits)
    b.run(12)
    b.run(9)
    with ThreadPoolExecutor(8) as ex:
        refs = list(ex.map(lambda r: _oracle_member(oracle_lib, members[r], inits[r], 21)[0],
                           range(len(members))))
    for r, ref in enumerate(refs):
        np.testing.assert_array_equal(b.state(r), ref, err_msg=f"member {r}")
    b.close()


@pytest.mark.parametrize("rounds,exchange", [(7, False), (10, True)])
def test_every_shape_same_bits(ilg, rounds, exchange):
    members, inits = _members(2, 2, 20, 3, rounds, exchange)
    ref = None
    for shape in range(ilg.Batch.shape_count()):
        b = ilg.Batch(members, inits)
        b.set_shape(shape)
        b.run(10)
        states = [b.state(r) for r in range(len(members))]
        b.close()
        if ref is None:
            ref = states
            continue
        for r in range(len(members)):
            np.testing.assert_array_equal(states[r], ref[r], err_msg=f"shape {shape} member {r}")


@pytest.mark.parametrize("q,rounds,exchange", [(2, 10, True), (3, 7, False)])
def test_diagnostics(ilg, oracle_lib, q, rounds, exchange):
    w = W.D1Q3_WEIGHTS if q == 3 else W.D1Q2_WEIGHTS
    rng = np.random.default_rng(17 + q)
    members, inits = [], []
    for r in range(6):
        L = int(rng.integers(100, 5000))
        members.append(dict(q=q, length=L, count_bytes=4, omega=float(rng.uniform(1.0, 1.95)),
                            seed=400 + r, realization=r, t0=int(rng.integers(0, 9)),
                            rounds=rounds, exchange=exchange))
        inits.append(W.init_poisson_sine(w, L, 80.0, 40.0, 4, init_seed=600 + r))
    nk, steps = 16, 24
    b = ilg.Batch(members, inits, sk_every=5, nk=nk, amp_every=4, max_amp=8)
    b.run(steps)
    sk, nsk = b.structure_factor()
    amp, namp = b.amplitudes()
    for r, m in enumerate(members):
        ref, rsk, rnsk, ramp = _oracle_member(oracle_lib, m, inits[r], steps, sk_every=5, nk=nk,
                                              amp_every=4)
        np.testing.assert_array_equal(b.state(r), ref)
        assert int(nsk[r]) == rnsk and int(namp[r]) == len(ramp)
        mass = float(inits[r].astype(np.int64).sum())
        np.testing.assert_allclose(sk[r], rsk, rtol=1e-9, atol=1e-9 * mass)
        np.testing.assert_allclose(amp[r, :len(ramp)], ramp, rtol=1e-9,
                                   atol=1e-9 * mass / m["length"])
    b.close()


def test_exchange_differs_from_three_binomials_and_equals_plain(ilg):
    members, inits = _members(2, 2, 12, 8, 10, True)
    b = ilg.Batch(members, inits)
    b.run(15)
    b3 = ilg.Batch([dict(m, exchange=False) for m in members], inits)
    b3.run(15)
    differ = 0
    for r in [3, 6, 7, 9, 11]:
        m = members[r]
        lat = ilg.Lattice(2, m["length"], 2, m["omega"], m["seed"], inits[r],
                          realization=m["realization"], t0=m["t0"], exchange=True)
        lat.step(15)
        np.testing.assert_array_equal(b.state(r), lat.state())
        lat.close()
        differ += int((b.state(r) != b3.state(r)).any())
    assert differ >= 4
    b.close()
    b3.close()
