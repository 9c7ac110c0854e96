"""GPU parity of the batched (persistent, graph-replayed) ensemble form.

Every compared member state is bit-exact against the oracle run of the same
configuration; FP64 diagnostics (S(k) sums, A^LG series) agree within a
tolerance derived from the summation length.  Statistical checks of the
ensemble against the paper's Boltzmann limit and diffusion constant use the
GPU output, which the same tests tie bit-exactly to the oracle on sampled
members.
"""
import math
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


def _member(spec):
    return dict(q=spec.q, length=spec.length, count_bytes=spec.count_bytes, omega=spec.omega,
                seed=spec.seed, realization=spec.realization)


def _oracle_member(oracle_lib, m, init, nsteps, t0=0, sk_every=0, nk=0, amp_every=0):
    """Oracle run of one member; also the S(k) sum and A^LG series sampled on
    the member's own step clock (after steps t with t % every == 0)."""
    p = oracle_lib.Params(m["q"], m["omega"], flip=m.get("flip", "auto"))
    cur = init
    sk = np.zeros(nk)
    nsk = 0
    amps = []
    t = t0
    end = t0 + nsteps
    every = [e for e in (sk_every, amp_every) if e]
    while t < end:
        nxt = end
        for e in every:
            nxt = min(nxt, (t // e + 1) * e)
        cur, _, ov = oracle_lib.run(p, cur, nxt - t, seed=m["seed"],
                                    realization=m.get("realization", 0), t0=t, nthreads=1)
        assert not ov
        t = nxt
        N = cur.astype(np.int64).sum(axis=0)
        if sk_every and t % sk_every == 0:
            sk += exact.structure_factor(N, nk)
            nsk += 1
        if amp_every and t % amp_every == 0:
            amps.append(exact.amplitude_lg(N))
    return cur, sk, nsk, np.array(amps)


def _ragged_members(q, cb, n, seed):
    rng = np.random.default_rng(seed)
    lens = [1, 2, 3, 63, 64, 65] + list(rng.integers(4, 700, size=n - 6))
    members, inits = [], []
    omegas = [2.0, 1.0, 0.5, 1.5, 1.98, 0.9]
    for r, L in enumerate(lens):
        om = omegas[r] if r < len(omegas) else float(rng.uniform(0.3, 2.0))
        members.append(dict(q=q, length=int(L), count_bytes=cb, omega=om, seed=5000 + r,
                            realization=r * 7, t0=int(rng.integers(0, 1000))))
        inits.append(W.init_poisson_iid(q, int(L), 35.0, cb, init_seed=9000 + r))
    return members, inits


@pytest.mark.parametrize("q,cb", [(2, 2), (2, 4), (3, 2), (3, 4)])
def test_ragged_ensemble_every_member(ilg, oracle_lib, q, cb):
    """Members of every length (1, 2, 3, ragged), rates on both sides of 1
    (incl. omega^j = 2 and the flip-moot 1) and start steps: two graph runs
    (20 then 17 steps, so the graph is re-captured), all members exact."""
    members, inits = _ragged_members(q, cb, 40, seed=q * 10 + cb)
    _say(f"[batch] ragged q={q} cb={cb}")
    b = ilg.Batch(members, inits)
    b.run(20)
    b.run(17)
    with ThreadPoolExecutor(8) as ex:
        refs = list(ex.map(lambda r: _oracle_member(oracle_lib, members[r], inits[r], 37,
                                                    t0=members[r]["t0"])[0], range(len(members))))
    for r, ref in enumerate(refs):
        np.testing.assert_array_equal(b.state(r), ref, err_msg=f"member {r}")
    b.close()


def test_batched_equals_plain(ilg):
    """The same configurations run alone through the plain API give the same bits."""
    members, inits = _ragged_members(3, 2, 12, seed=77)
    b = ilg.Batch(members, inits)
    b.run(25)
    for r in [0, 3, 5, 7, 11]:
        m = members[r]
        lat = ilg.Lattice(m["q"], m["length"], m["count_bytes"], m["omega"], m["seed"], inits[r],
                          realization=m["realization"], t0=m["t0"])
        lat.step(25)
        np.testing.assert_array_equal(b.state(r), lat.state())
        lat.close()
    b.close()


def test_every_shape_same_bits_and_tune_is_side_effect_free(ilg):
    members, inits = _ragged_members(2, 2, 30, seed=5)
    ref = None
    for shape in range(ilg.Batch.shape_count()):
        b = ilg.Batch(members, inits)
        b.set_shape(shape)
        b.run(15)
        states = [b.state(r) for r in range(len(members))]
        if ref is None:
            ref = states
        else:
            for r in range(len(members)):
                np.testing.assert_array_equal(states[r], ref[r], err_msg=f"shape {shape} member {r}")
        b.close()
    b = ilg.Batch(members, inits)
    before = [b.state(r) for r in range(len(members))]
    chosen = b.tune(10)
    assert 0 <= chosen < ilg.Batch.shape_count()
    for r in range(len(members)):
        np.testing.assert_array_equal(b.state(r), before[r])   # tuning ran on a copy
    b.run(15)
    for r in range(len(members)):
        np.testing.assert_array_equal(b.state(r), ref[r])
    b.close()


@pytest.mark.parametrize("q", [2, 3])
def test_batch_diagnostics(ilg, oracle_lib, q):
    """S(k) sums every 7 steps and A^LG every 5 steps on each member's clock."""
    rng = np.random.default_rng(3 + q)
    w = W.D1Q3_WEIGHTS if q == 3 else W.D1Q2_WEIGHTS
    members, inits = [], []
    for r in range(10):
        L = int(rng.integers(40, 900))
        members.append(dict(q=q, length=L, count_bytes=4, omega=float(rng.uniform(1.0, 1.95)),
                            seed=300 + r, realization=r, t0=int(rng.integers(0, 9))))
        inits.append(W.init_poisson_sine(w, L, 80.0, 40.0, 4, init_seed=700 + r))
    nk, steps = 12, 40
    b = ilg.Batch(members, inits, sk_every=7, nk=nk, amp_every=5, max_amp=16)
    b.run(23)
    b.run(17)
    sk, nsk = b.structure_factor()
    amp, namp = b.amplitudes()
    for r, m in enumerate(members):
        ref, rsk, rnsk, ramp = _oracle_member(oracle_lib, m, inits[r], steps, t0=m["t0"],
                                              sk_every=7, nk=nk, amp_every=5)
        np.testing.assert_array_equal(b.state(r), ref)
        assert int(nsk[r]) == rnsk and int(namp[r]) == len(ramp)
        mass = float(inits[r].astype(np.int64).sum())
        # FP64 sums over L terms bounded by N(x): error << 1e-9 of the scale
        np.testing.assert_allclose(sk[r], rsk, rtol=1e-9, atol=1e-9 * mass)
        np.testing.assert_allclose(amp[r, :len(ramp)], ramp, rtol=1e-9,
                                   atol=1e-9 * mass / m["length"])
    b.close()


@pytest.mark.parametrize("q", [2, 3])
def test_batch_diagnostics_long_members_every_shape(ilg, oracle_lib, q):
    """S(k) and A^LG of members longer than 16 rows of every workgroup shape
    (the twiddle restarts from the run stride), lengths not multiples of the
    workgroup, and one member shorter than a wave; every shape against the
    oracle."""
    w = W.D1Q3_WEIGHTS if q == 3 else W.D1Q2_WEIGHTS
    lens = [40961, 20000, 9000, 2049, 37]
    members, inits = [], []
    for r, L in enumerate(lens):
        members.append(dict(q=q, length=L, count_bytes=4, omega=1.3 + 0.1 * r, seed=900 + r,
                            realization=r))
        inits.append(W.init_poisson_sine(w, L, 60.0, 30.0, 4, init_seed=800 + r))
    nk, steps = 16, 6
    refs = [_oracle_member(oracle_lib, m, inits[r], steps, sk_every=3, nk=nk, amp_every=2)
            for r, m in enumerate(members)]
    for shape in range(ilg.Batch.shape_count()):
        _say(f"[long members] q={q} shape {shape}")
        b = ilg.Batch(members, inits, sk_every=3, nk=nk, amp_every=2, max_amp=4)
        b.set_shape(shape)
        b.run(steps)
        sk, nsk = b.structure_factor()
        amp, namp = b.amplitudes()
        for r, (ref, rsk, rnsk, ramp) in enumerate(refs):
            np.testing.assert_array_equal(b.state(r), ref, err_msg=f"shape {shape} member {r}")
            assert int(nsk[r]) == rnsk and int(namp[r]) == len(ramp)
            mass = float(inits[r].astype(np.int64).sum())
            np.testing.assert_allclose(sk[r], rsk, rtol=1e-9, atol=1e-9 * mass,
                                       err_msg=f"shape {shape} member {r}")
            np.testing.assert_allclose(amp[r, :len(ramp)], ramp, rtol=1e-9,
                                       atol=1e-9 * mass / lens[r],
                                       err_msg=f"shape {shape} member {r}")
        b.close()


@pytest.fixture(scope="module")
def config3_gpu(ilg):
    """4096 D1Q2 members, L log-uniform in [64, 8192], omega ~ U[1, 1.95],
    seed 1000 + r, Poisson(30) uint16, 5000 steps in one graph replay with
    S(k), k = 1..16, every 10 steps: final states and S(k) sums."""
    ens = W.ensemble_ragged_d1q2()
    members = [_member(s) for s in ens.specs]
    b = ilg.Batch(members, ens.inits, sk_every=10, nk=16)
    _say("[config3] tune + run 5000 steps")
    b.tune(10)
    b.run(5000)
    sk, nsk = b.structure_factor()
    states = [b.state(r) for r in range(len(members))]
    b.close()
    return ens, members, states, sk, nsk


def _config3_picks(ens, n=256):
    """n members spread evenly over the length order (shortest and longest
    included)."""
    lens = np.array([s.length for s in ens.specs])
    order = np.argsort(lens, kind="stable")
    return [int(order[i]) for i in np.linspace(0, len(order) - 1, n).round().astype(int)]


def test_config3_ragged_ensemble_diagnostics(config3_gpu, oracle_lib):
    """Exact mass for every member; S(k) sums of 32 members spread by length
    against the oracle's (with their states); equilibrium S(k) ~ 1."""
    ens, members, states, sk, nsk = config3_gpu
    assert np.all(nsk == 500)
    for r in range(len(members)):
        assert int(states[r].astype(np.int64).sum()) == int(ens.inits[r].astype(np.int64).sum())
    picks = _config3_picks(ens, 32)
    _say(f"[config3] oracle with S(k) for {len(picks)} members")
    with ThreadPoolExecutor(16) as ex:
        res = list(ex.map(lambda r: _oracle_member(oracle_lib, members[r], ens.inits[r], 5000,
                                                   sk_every=10, nk=16), picks))
    for r, (ref, rsk, rnsk, _) in zip(picks, res):
        np.testing.assert_array_equal(states[r], ref, err_msg=f"member {r}")
        assert rnsk == 500
        np.testing.assert_allclose(sk[r], rsk, rtol=1e-9)
    # equilibrium S(k) ~ 1 (Poisson occupations), ensemble mean over members
    Sbar = (sk / nsk[:, None]).mean()
    assert abs(Sbar - 1.0) < 0.02


@pytest.mark.parametrize("part", range(4))
def test_config3_ragged_ensemble_members(config3_gpu, oracle_lib, part):
    """256 members spread evenly over the length order (64 per part), each
    whole final state bit-exact against the oracle's 5000-step run."""
    ens, members, states, _, _ = config3_gpu
    picks = _config3_picks(ens, 256)[part::4]
    _say(f"[config3] oracle for {len(picks)} members (part {part})")

    def one(r):
        m = members[r]
        ref, _, ov = oracle_lib.run(oracle_lib.Params(m["q"], m["omega"]), ens.inits[r], 5000,
                                    seed=m["seed"], realization=m["realization"], nthreads=1)
        assert not ov
        return ref

    with ThreadPoolExecutor(16) as ex:
        refs = list(ex.map(one, picks))
    for r, ref in zip(picks, refs):
        np.testing.assert_array_equal(states[r], ref, err_msg=f"member {r}")


def _decay_fit(a0, aT, T):
    return -math.log(aT.sum() / a0.sum()) / T


@pytest.fixture(scope="module")
def config4_gpu(ilg):
    """6 omega x 1024 members of D1Q3, L = 4096, uint32, Poisson sine init
    (mean w_i (100 + 40 sin)), 10^4 steps with A^LG every 100 steps."""
    ens = W.ensemble_decay_sweep()
    members = [_member(s) for s in ens.specs]
    b = ilg.Batch(members, ens.inits, amp_every=100, max_amp=100)
    _say("[config4] run 10000 steps")
    b.run(10000)
    amp, namp = b.amplitudes()
    states = [b.state(r) for r in range(len(members))]
    b.close()
    return ens, members, states, amp, namp


def test_config4_decay_rates(config4_gpu):
    """The fitted decay rate per omega against 4 pi^2 D / L^2, D = theta
    (1/omega^j - 1/2), within 5 of its statistical standard deviations (the
    ensemble cannot resolve 1e-2 here for omega >= 1.75; the gate at the
    paper's geometry is a separate test)."""
    ens, members, states, amp, namp = config4_gpu
    assert np.all(namp == 100)
    L, T, nper = 4096, 10000, 1024
    a0 = np.array([exact.amplitude_lg(x.astype(np.int64).sum(axis=0)) for x in ens.inits])
    aT = amp[:, -1]
    th = exact.theta_of(3)
    for oi, om in enumerate(W.DECAY_SWEEP_OMEGAS):
        sl = slice(oi * nper, (oi + 1) * nper)
        g = _decay_fit(a0[sl], aT[sl], T)
        D = exact.diffusion_constant(om, th)
        gth = 4 * math.pi ** 2 * D / L ** 2
        var_eq = 2 * 100.0 / L
        sig = math.sqrt(var_eq * (1 - math.exp(-2 * gth * T)) / nper) / (40 * math.exp(-gth * T) * gth * T)
        _say(f"[config4] omega={om} gamma/gamma_th={g / gth:.4f} sigma={sig:.4f}")
        assert abs(g / gth - 1) < 5 * sig + 1e-3


@pytest.mark.parametrize("oi", range(len(W.DECAY_SWEEP_OMEGAS)),
                         ids=[f"omega{om}" for om in W.DECAY_SWEEP_OMEGAS])
def test_config4_members(config4_gpu, oracle_lib, oi):
    """16 members of each omega (spread over its 1024), each whole final state
    and its A^LG series against the oracle's 10^4-step run."""
    ens, members, states, amp, _ = config4_gpu
    nper, T = 1024, 10000
    picks = [oi * nper + k for k in range(5, nper, 64)]
    assert len(picks) == 16
    _say(f"[config4] oracle for 16 members of omega {W.DECAY_SWEEP_OMEGAS[oi]}")
    with ThreadPoolExecutor(16) as ex:
        res = list(ex.map(lambda r: _oracle_member(oracle_lib, members[r], ens.inits[r], T,
                                                   amp_every=100), picks))
    for r, (ref, _, _, ramp) in zip(picks, res):
        np.testing.assert_array_equal(states[r], ref, err_msg=f"member {r}")
        np.testing.assert_allclose(amp[r], ramp, rtol=1e-9, atol=1e-9)


def test_decay_rate_gate_paper_geometry(ilg):
    """The paper's geometry (Results section): D1Q3, L = 320, N^ave = 100,
    A_0 = N^ave, Poisson initialisation; 1024 members per omega^j, run for
    T = ceil(1/gamma) steps capped at 2e5.  The fitted rate matches
    4 pi^2 D / L^2 within 1e-2 relative for every omega^j (statistical
    1-sigma below 0.2 %)."""
    L, nave, nper = 320, 100.0, 1024
    th = exact.theta_of(3)
    members, inits, Ts = [], [], []
    omegas = [0.6, 1.0, 1.25, 1.5, 1.75, 1.9, 1.98]
    for oi, om in enumerate(omegas):
        D = exact.diffusion_constant(om, th)
        T = min(int(math.ceil(L ** 2 / (4 * math.pi ** 2 * D))), 200000)
        Ts.append(T)
    # members of one omega share T; run the sweep as one batch per omega
    worst = 0.0
    for oi, om in enumerate(omegas):
        ms, ins = [], []
        for r in range(nper):
            ms.append(dict(q=3, length=L, count_bytes=2, omega=om, seed=20_000_000 + oi * 4096 + r,
                           realization=r))
            ins.append(W.init_poisson_sine(W.D1Q3_WEIGHTS, L, nave, nave, 2,
                                           init_seed=30_000_000 + oi * 4096 + r))
        b = ilg.Batch(ms, ins)
        b.run(Ts[oi])
        a0 = np.array([exact.amplitude_lg(x.astype(np.int64).sum(axis=0)) for x in ins])
        aT = np.array([exact.amplitude_lg(b.state(r).astype(np.int64).sum(axis=0))
                       for r in range(nper)])
        b.close()
        g = _decay_fit(a0, aT, Ts[oi])
        gth = 4 * math.pi ** 2 * exact.diffusion_constant(om, th) / L ** 2
        err = abs(g / gth - 1)
        worst = max(worst, err)
        _say(f"[paper geometry] omega^j={om} T={Ts[oi]} gamma/gamma_th={g / gth:.5f}")
        assert err < 1e-2
