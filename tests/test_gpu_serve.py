"""GPU tests of the continuous-batching server: every request's result is
bit-identical to the same configuration run alone (plain API) and, sampled,
to the oracle; admission respects the memory budget; requests arriving while
others run join the shared launches."""
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


def _requests(n, seed):
    rng = np.random.default_rng(seed)
    lens = [1, 2, 63, 1023, 1024, 1025, 3000, 5000] + list(rng.integers(3, 4000, size=n - 8))
    reqs = []
    for i, L in enumerate(lens):
        q = 2 + int(rng.integers(0, 2))
        cb = 2 if rng.random() < 0.7 else 4
        om = [2.0, 1.0, 0.7][i] if i < 3 else float(rng.uniform(0.5, 1.99))
        m = dict(q=q, length=int(L), count_bytes=cb, omega=om, seed=800 + i, realization=i,
                 t0=int(rng.integers(0, 50)))
        init = W.init_poisson_iid(q, int(L), 40.0, cb, init_seed=1234 + i)
        reqs.append((m, init, int(rng.integers(1, 300))))
    return reqs


def _alone(ilg, m, init, nsteps):
    lat = ilg.Lattice(m["q"], m["length"], m["count_bytes"], m["omega"], m["seed"], init,
                      realization=m.get("realization", 0), t0=m.get("t0", 0),
                      rounds=m.get("rounds", 10), exchange=m.get("exchange", False),
                      height=m.get("height", 0))
    lat.step(nsteps)
    out = lat.state()
    lat.close()
    return out


# Small requests advanced in one workgroup per request (the default), or all
# requests by the per-step launches.
RESIDENT = [None, (0, 0)]
RESIDENT_IDS = ["resident", "steps-only"]


@pytest.mark.parametrize("resident", RESIDENT, ids=RESIDENT_IDS)
def test_mixed_requests_equal_alone_and_oracle(ilg, oracle_lib, resident):
    """40 requests of both velocity sets and count types, lengths from 1 to
    5000, 1..300 steps, submitted in three waves while earlier ones run."""
    reqs = _requests(40, seed=1)
    srv = ilg.Server(64 << 20, quantum_steps=37, resident=resident)
    ids = {}
    for k, (m, init, ns) in enumerate(reqs):
        ids[k] = srv.submit(m, init, ns)
        if k in (10, 25):
            srv.poll()
    polls = 0
    while True:
        st = srv.poll()
        polls += 1
        if st["active"] == 0 and st["queued"] == 0:
            break
        assert polls < 1000
    for k, (m, init, ns) in enumerate(reqs):
        info = srv.info(ids[k])
        assert info["state"] == "done" and info["steps_done"] == ns
        assert info["t_done"] >= info["t_admit"] >= info["t_submit"]
        got = srv.result(ids[k])
        np.testing.assert_array_equal(got, _alone(ilg, m, init, ns), err_msg=f"request {k}")
        if k % 8 == 0:
            p = oracle_lib.Params(m["q"], m["omega"])
            ref, _, _ = oracle_lib.run(p, init, ns, seed=m["seed"], realization=m["realization"],
                                       t0=m["t0"])
            np.testing.assert_array_equal(got, ref, err_msg=f"request {k} vs oracle")
    srv.close()


@pytest.mark.parametrize("resident", RESIDENT, ids=RESIDENT_IDS)
def test_draw_specifications_in_one_server(ilg, oracle_lib, resident):
    """Requests under draw specifications v1, v2 (7 rounds) and v3 (D1Q2
    exchange form, 10 or 7 rounds) share one server (one launch group per
    specification): each result equals the same configuration run alone and,
    for a sample, the oracle."""
    base = _requests(36, seed=4)
    specs = [(10, False), (7, False), (10, True), (7, True)]
    reqs = []
    for i, (m, init, ns) in enumerate(base):
        rounds, exchange = specs[i % 4]
        if exchange and m["q"] != 2:
            exchange = False
        reqs.append((dict(m, rounds=rounds, exchange=exchange), init, ns))
    srv = ilg.Server(64 << 20, quantum_steps=29, resident=resident)
    ids = [srv.submit(m, init, ns) for m, init, ns in reqs]
    polls = 0
    while True:
        st = srv.poll()
        polls += 1
        if st["active"] == 0 and st["queued"] == 0:
            break
        assert polls < 1000
    for k, (m, init, ns) in enumerate(reqs):
        got = srv.result(ids[k])
        np.testing.assert_array_equal(got, _alone(ilg, m, init, ns), err_msg=f"request {k}")
        if k % 5 == 0:
            p = oracle_lib.Params(m["q"], m["omega"], rounds=m["rounds"], exchange=m["exchange"])
            ref, _, _ = oracle_lib.run(p, init, ns, seed=m["seed"], realization=m["realization"],
                                       t0=m["t0"])
            np.testing.assert_array_equal(got, ref, err_msg=f"request {k} vs oracle")
    srv.close()


@pytest.mark.parametrize("resident", RESIDENT, ids=RESIDENT_IDS)
def test_d2q5_requests_with_1d_ones(ilg, oracle_lib, resident):
    """D2Q5 requests (shapes from one node to rows wider than a tile, both
    count types, 10- and 7-round draws, a device-drawn initial state) served
    beside D1Q2/D1Q3 requests: each equals the configuration run alone and,
    sampled, the oracle's 2D run."""
    from oracle import oracle as O
    rng = np.random.default_rng(21)
    shapes = [(1, 1), (33, 7), (64, 64), (1500, 3), (5, 300), (129, 17)]
    reqs = []
    for i, (lx, ly) in enumerate(shapes):
        cb = 2 if i % 2 == 0 else 4
        m = dict(q=5, length=lx, height=ly, count_bytes=cb, omega=[1.8, 0.7, 1.3][i % 3],
                 seed=900 + i, realization=i, t0=int(rng.integers(0, 30)),
                 rounds=7 if i == 4 else 10)
        dt = np.uint16 if cb == 2 else np.uint32
        init = rng.poisson([[[25.0]], [[25.0]], [[50.0]], [[25.0]], [[25.0]]],
                           size=(5, ly, lx)).astype(dt)
        reqs.append((m, init, int(rng.integers(5, 90))))
    reqs += _requests(12, seed=22)
    srv = ilg.Server(64 << 20, quantum_steps=23, resident=resident)
    ids = [srv.submit(m, init, ns) for m, init, ns in reqs]
    drawn = dict(q=5, length=96, height=40, count_bytes=2, omega=1.5, seed=77, realization=3,
                 t0=0)
    did = srv.submit_poisson_sine(drawn, 80.0, 40.0, 9, 33)
    polls = 0
    while True:
        st = srv.poll()
        polls += 1
        if st["active"] == 0 and st["queued"] == 0:
            break
        assert polls < 1000
    for k, (m, init, ns) in enumerate(reqs):
        got = srv.result(ids[k])
        np.testing.assert_array_equal(got, _alone(ilg, m, init, ns), err_msg=f"request {k}")
        if m["q"] == 5 and k % 2 == 0:
            p = oracle_lib.Params(5, m["omega"], rounds=m["rounds"])
            ref, _, ov = oracle_lib.run2d(p, init, ns, seed=m["seed"],
                                          realization=m["realization"], t0=m["t0"])
            assert not ov
            np.testing.assert_array_equal(got, ref, err_msg=f"request {k} vs oracle")
    got = srv.result(did)
    init, ov = O.init_poisson_sine(5, 2, 96, 80.0, 40.0, 9, realization=3, height=40)
    assert not ov
    want, _, _ = oracle_lib.run2d(oracle_lib.Params(5, 1.5), init, 33, seed=77, realization=3)
    np.testing.assert_array_equal(got, want)
    srv.close()


def test_budget_admission_on_gpu(ilg):
    """A budget that holds only a few requests: later requests wait, peak use
    stays within the budget, and results are unchanged."""
    reqs = [(dict(q=3, length=20000, count_bytes=2, omega=1.6, seed=50 + i, realization=i),
             W.init_poisson_iid(3, 20000, 40.0, 2, init_seed=60 + i), 40) for i in range(6)]
    per = 2 * 3 * 20032 * 2 + 2 * (2080 * 4 + 64 * 256)
    budget = 2 * per + 4096
    srv = ilg.Server(budget, quantum_steps=16)
    ids = [srv.submit(m, init, ns) for m, init, ns in reqs]
    first = srv.poll()
    assert first["admitted"] == 2 and first["queued"] == 4
    while True:
        st = srv.poll()
        assert st["bytes_peak"] <= budget
        if st["active"] == 0 and st["queued"] == 0:
            break
    for rid, (m, init, ns) in zip(ids, reqs):
        np.testing.assert_array_equal(srv.result(rid), _alone(ilg, m, init, ns))
    srv.close()


def test_busy_and_cancel(ilg):
    srv = ilg.Server(1 << 20, quantum_steps=10)
    big = dict(q=3, length=200000, count_bytes=2, omega=1.5, seed=1)
    with pytest.raises(ilg.IlgError) as e:
        srv.submit(big, np.zeros((3, 200000), np.uint16), 10)
    assert e.value.code == -6
    m = dict(q=2, length=5000, count_bytes=2, omega=1.5, seed=2)
    init = W.init_poisson_iid(2, 5000, 30.0, 2, init_seed=3)
    a = srv.submit(m, init, 100)
    b = srv.submit(dict(m, seed=3), init, 100)
    srv.poll()
    srv.cancel(a)
    while srv.poll()["active"]:
        pass
    assert srv.info(b)["state"] == "done"
    np.testing.assert_array_equal(srv.result(b), _alone(ilg, dict(m, seed=3, realization=0,
                                                                  t0=0), init, 100))
    srv.close()


def test_request_stream_replay(ilg):
    """A short Poisson request stream of the serving workload's mix (q in
    {2, 3}, L log-uniform 2^8..2^14, 100..600 steps, omega ~ U[1, 1.95]),
    replayed through poll(): all requests finish, results of a sample equal
    the plain runs."""
    reqs = W.request_stream(rate_per_s=400.0, duration_s=0.2, lmax_log2=14, tmax=600)
    pool = W.RequestInitPool(npool=2, lmax_log2=14)
    srv = ilg.Server(256 << 20, quantum_steps=50)
    ids = []
    for i, rq in enumerate(reqs):
        m = dict(q=rq.spec.q, length=rq.spec.length, count_bytes=2, omega=rq.spec.omega,
                 seed=rq.spec.seed, realization=rq.spec.realization)
        ids.append((srv.submit(m, pool.init(i, m["q"], m["length"]), rq.spec.steps), m, i,
                    rq.spec.steps))
        if i % 5 == 4:
            srv.poll()
    while True:
        st = srv.poll()
        if st["active"] == 0 and st["queued"] == 0:
            break
    _say(f"[serve] {len(reqs)} requests done")
    for rid, m, i, ns in ids:
        got = srv.result(rid)
        if i % 7 == 0:
            np.testing.assert_array_equal(
                got, _alone(ilg, dict(m, t0=0), pool.init(i, m["q"], m["length"]), ns))
    srv.close()


def test_device_drawn_initial_states(ilg, oracle_lib):
    """Requests whose Poisson sine initial state is drawn on the device at
    admission (no host state) end exactly where the oracle's draw of that
    state, stepped by the oracle, ends; mixed with host-state requests."""
    from oracle import oracle as O
    cases = [dict(q=3, length=320, count_bytes=2, omega=1.6, seed=31, realization=4, t0=0),
             dict(q=2, length=5000, count_bytes=4, omega=1.2, seed=32, realization=0, t0=9),
             dict(q=3, length=1025, count_bytes=4, omega=0.8, seed=33, realization=7, t0=0)]
    draws = [(100.0, 100.0, 5), (40.0, 15.0, 6), (300.0, 200.0, 7)]
    steps = [120, 45, 77]
    srv = ilg.Server(32 << 20, quantum_steps=25)
    ids = []
    for m, (nave, amp, s), ns in zip(cases, draws, steps):
        ids.append(srv.submit_poisson_sine(m, nave, amp, s, ns))
        m2 = dict(m, seed=m["seed"] + 100)
        srv.submit(m2, W.init_poisson_iid(m["q"], m["length"], 30.0, m["count_bytes"], 3), ns)
    for _ in range(1000):
        st = srv.poll()
        if st["active"] == 0 and st["queued"] == 0:
            break
    for rid, m, (nave, amp, s), ns in zip(ids, cases, draws, steps):
        assert srv.info(rid)["state"] == "done"
        got = srv.result(rid)
        init, ov = O.init_poisson_sine(m["q"], m["count_bytes"], m["length"], nave, amp, s,
                                       realization=m["realization"])
        assert not ov
        want, _, _ = oracle_lib.run(oracle_lib.Params(m["q"], m["omega"]), init, ns,
                                    seed=m["seed"], realization=m["realization"], t0=m["t0"])
        np.testing.assert_array_equal(got, want)
    srv.close()


def _drain(srv, limit=100000):
    failed = 0
    for _ in range(limit):
        st = srv.poll()
        failed += st["failed"]
        if st["active"] == 0 and st["queued"] == 0:
            return failed
    raise AssertionError("server did not drain")


def test_overflowing_request_fails_alone(ilg):
    """One request whose counts overflow uint16 in its first step and one
    whose device-drawn initial state overflows at admission are each retired
    as failed (ILG_E_OVERFLOW from result, naming the request); the requests
    beside them in the same launches finish bit-identical to their runs
    alone, and the server goes on serving."""
    reqs = _requests(12, seed=31)
    srv = ilg.Server(64 << 20, quantum_steps=20)
    ids = [srv.submit(m, init, ns) for m, init, ns in reqs[:6]]
    # omega = 1, no flip: every particle collides; 3 x 40000 particles per
    # node send about 80000 to the rest velocity, beyond 65535
    bad = srv.submit(dict(q=3, length=3000, count_bytes=2, omega=1.0, seed=5),
                     np.full((3, 3000), 40000, np.uint16), 50)
    # Poisson means of 5e5 per velocity do not fit uint16
    bad_init = srv.submit_poisson_sine(dict(q=2, length=700, count_bytes=2, omega=1.5, seed=6),
                                       1.0e6, 0.0, 3, 40)
    ids += [srv.submit(m, init, ns) for m, init, ns in reqs[6:]]
    assert _drain(srv) == 2
    for rid in (bad, bad_init):
        assert srv.info(rid)["state"] == "failed"
        with pytest.raises(ilg.IlgError) as e:
            srv.result(rid)
        assert e.value.code == -4 and f"request {rid}" in str(e.value)
    for rid, (m, init, ns) in zip(ids, reqs):
        assert srv.info(rid)["state"] == "done"
        np.testing.assert_array_equal(srv.result(rid), _alone(ilg, m, init, ns),
                                      err_msg=f"request {rid}")
    m, init, ns = reqs[7]
    rid = srv.submit(m, init, ns)
    assert _drain(srv) == 0
    np.testing.assert_array_equal(srv.result(rid), _alone(ilg, m, init, ns))
    srv.close()


def test_stream_sized_requests_equal_alone_and_oracle(ilg, oracle_lib):
    """Requests at the sizes of the serving workload's largest (2^18..2^20
    nodes, 1024 tiles per slot, hundreds to thousands of steps over many
    quanta) served beside small ones: each equals its run alone, and the
    whole final state of every large request equals the oracle's."""
    large = [(dict(q=3, length=1 << 20, count_bytes=2, omega=1.7, seed=41, realization=1), 2000),
             (dict(q=2, length=(1 << 19) + 12345, count_bytes=2, omega=1.35, seed=42,
                   realization=2, t0=17), 700),
             (dict(q=3, length=1 << 18, count_bytes=4, omega=1.95, seed=43, realization=3), 300),
             (dict(q=2, length=(1 << 20) - 1, count_bytes=2, omega=1.02, seed=44,
                   realization=4), 250)]
    reqs = []
    for i, (m, ns) in enumerate(large):
        m.setdefault("t0", 0)
        reqs.append((m, W.init_poisson_iid(m["q"], m["length"], 40.0, m["count_bytes"],
                                           init_seed=70 + i), ns))
    small = _requests(12, seed=32)
    srv = ilg.Server(1 << 30, quantum_steps=100)
    ids = []
    for k, (m, init, ns) in enumerate(reqs + small):
        ids.append(srv.submit(m, init, ns))
        if k % 3 == 2:
            srv.poll()
    assert _drain(srv) == 0
    _say("[serve] stream-sized requests done")
    for k, (m, init, ns) in enumerate(reqs + small):
        got = srv.result(ids[k])
        np.testing.assert_array_equal(got, _alone(ilg, m, init, ns), err_msg=f"request {k}")
        if k < len(reqs):
            _say(f"[serve] oracle for request {k}: q={m['q']} L={m['length']} steps={ns}")
            p = oracle_lib.Params(m["q"], m["omega"])
            ref, _, ov = oracle_lib.run(p, init, ns, seed=m["seed"], realization=m["realization"],
                                        t0=m["t0"])
            assert not ov
            np.testing.assert_array_equal(got, ref, err_msg=f"request {k} vs oracle")
    srv.close()


def test_resident_advances_beside_large(ilg, oracle_lib):
    """Small requests with long step counts beside a large one: each advances
    by several steps per launch of the large request's quantum (at least one
    per launch, so at least the quantum per poll, and fewer than all of its
    steps); every result equals its run alone and, for a sample, the
    oracle."""
    big = (dict(q=3, length=1 << 20, count_bytes=2, omega=1.6, seed=61, realization=0, t0=0),
           W.init_poisson_iid(3, 1 << 20, 40.0, 2, init_seed=62), 120)
    small = []
    for i, (q, L) in enumerate([(2, 1), (3, 100), (2, 1024), (3, 1025), (3, 4096), (2, 3000)]):
        m = dict(q=q, length=L, count_bytes=2, omega=1.1 + 0.15 * i, seed=70 + i,
                 realization=i, t0=3 * i)
        small.append((m, W.init_poisson_iid(q, L, 40.0, 2, init_seed=80 + i), 4000))
    srv = ilg.Server(256 << 20, quantum_steps=20, resident=(4096, 4000))
    bid = srv.submit(*big)
    sids = [srv.submit(m, init, ns) for m, init, ns in small]
    srv.poll()  # admits all, launches the first quantum
    srv.poll()  # accounts for it
    taken = [srv.info(rid)["steps_done"] for rid in sids]
    _say(f"[serve] small requests' steps after the first quantum: {taken}")
    assert srv.info(bid)["steps_done"] == 20
    assert all(20 <= k < 4000 for k in taken)
    assert _drain(srv) == 0
    np.testing.assert_array_equal(srv.result(bid), _alone(ilg, *big))
    for k, (rid, (m, init, ns)) in enumerate(zip(sids, small)):
        got = srv.result(rid)
        np.testing.assert_array_equal(got, _alone(ilg, m, init, ns), err_msg=f"small {k}")
        if k % 2 == 0:
            p = oracle_lib.Params(m["q"], m["omega"])
            ref, _, _ = oracle_lib.run(p, init, ns, seed=m["seed"], realization=m["realization"],
                                       t0=m["t0"])
            np.testing.assert_array_equal(got, ref, err_msg=f"small {k} vs oracle")
    srv.close()


def test_resident_only_take_full_advances(ilg):
    """With only small requests active, each resident request takes
    min(steps left, the resident step count) in the poll's single launch.
    With more than a group's 128 resident slots, the others go to the tile
    walk (the quantum per poll) and the resident ones then take at least the
    quantum.  All finish bit-identical to their runs alone."""
    reqs = []
    for i in range(300):
        q = 2 + i % 2
        L = 1 + (i * 37) % 4096
        m = dict(q=q, length=L, count_bytes=2, omega=1.05 + 0.003 * i, seed=900 + i,
                 realization=i, t0=0)
        reqs.append((m, W.init_poisson_iid(q, L, 40.0, 2, init_seed=1900 + i), 50 + 3 * i))
    srv = ilg.Server(256 << 20, quantum_steps=10, resident=(4096, 300))
    for part, n in ((reqs[:200], 200), (reqs, 300)):
        ids = [srv.submit(m, init, ns) for m, init, ns in part]
        srv.poll()
        srv.poll()
        taken = [srv.info(rid)["steps_done"] for rid in ids]
        if n == 200:
            assert taken == [min(ns, 300) for _, _, ns in part]
        else:
            walk = sum(1 for k in taken if k == 10)
            _say(f"[serve] tile-walk advances {walk} of {n}")
            assert walk >= 44
            assert all(10 <= k <= min(ns, 300) for k, (_, _, ns) in zip(taken, part))
        assert _drain(srv) == 0
        for k, (rid, (m, init, ns)) in enumerate(zip(ids, part)):
            np.testing.assert_array_equal(srv.result(rid), _alone(ilg, m, init, ns),
                                          err_msg=f"request {k}")
    srv.close()


def test_resident_setting_checked(ilg):
    srv = ilg.Server(1 << 20, quantum_steps=10)
    with pytest.raises(ilg.IlgError) as e:
        srv.set_resident(65537, 100)
    assert e.value.code == -1
    srv.set_resident(0, 0)
    srv.set_resident(65536, 5)
    srv.close()
