"""CPU tests of the serving scheduler (paper_2203_01380_amd/csrc/scheduler.cpp)
with a counting executor: admission under the memory budget, FIFO order,
quantum advances, retirement, cancellation and the arena allocator."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2203_01380_amd", "csrc")
HARNESS = os.path.join(ROOT, "tests", "harness", "sched_harness.cpp")


@pytest.fixture(scope="module")
def H(tmp_path_factory):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    so = tmp_path_factory.mktemp("sched") / "libsched_harness.so"
    subprocess.run([gxx, "-O1", "-g", "-std=c++17", "-fPIC", "-shared", "-Wall", "-I", CSRC,
                    HARNESS, os.path.join(CSRC, "scheduler.cpp"), "-o", str(so)], check=True)
    L = ctypes.CDLL(str(so))
    L.h_new.restype = ctypes.c_void_p
    L.h_new.argtypes = [ctypes.c_uint64, ctypes.c_uint32]
    L.h_free.argtypes = [ctypes.c_void_p]
    L.h_submit.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64,
                           ctypes.POINTER(ctypes.c_uint64)]
    L.h_poll.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32)]
    L.h_state.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64),
                          ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    L.h_cancel.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
    L.h_release.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
    L.h_peak.argtypes = [ctypes.c_void_p]
    L.h_peak.restype = ctypes.c_uint64
    L.h_used.argtypes = [ctypes.c_void_p]
    L.h_used.restype = ctypes.c_uint64
    L.h_violations.argtypes = [ctypes.c_void_p]
    L.h_load_order.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64), ctypes.c_int]
    L.h_submit_nodes.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64,
                                 ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64)]
    L.h_set_step_nodes.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
    L.h_last_launch.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64), ctypes.c_int]
    L.h_fail_load.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
    L.h_fail_wait.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
    L.h_poll5.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32)]
    L.h_set_resident.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32,
                                 ctypes.c_uint32]
    L.h_last_steps.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32), ctypes.c_int]
    return L


class Sched:
    def __init__(self, H, budget, quantum):
        self.H, self.h = H, H.h_new(budget, quantum)

    def submit(self, q, nbytes, steps):
        rid = ctypes.c_uint64()
        rc = self.H.h_submit(self.h, q, nbytes, steps, ctypes.byref(rid))
        return rc, int(rid.value)

    def poll(self):
        out = (ctypes.c_uint32 * 4)()
        assert self.H.h_poll(self.h, out) == 0
        return dict(admitted=out[0], active=out[1], queued=out[2], finished=out[3])

    def state(self, rid):
        d, ta, td = ctypes.c_uint64(), ctypes.c_double(), ctypes.c_double()
        s = self.H.h_state(self.h, rid, ctypes.byref(d), ctypes.byref(ta), ctypes.byref(td))
        return s, int(d.value), ta.value, td.value

    def submit_nodes(self, nodes, steps, nbytes=1000):
        rid = ctypes.c_uint64()
        rc = self.H.h_submit_nodes(self.h, 2, nbytes, steps, nodes, ctypes.byref(rid))
        assert rc == 0
        return int(rid.value)

    def last_launch(self):
        buf = (ctypes.c_uint64 * 4096)()
        n = self.H.h_last_launch(self.h, buf, 4096)
        return list(buf[:n])

    def last_steps(self):
        buf = (ctypes.c_uint32 * 4096)()
        n = self.H.h_last_steps(self.h, buf, 4096)
        return list(buf[:n])

    def load_order(self):
        buf = (ctypes.c_uint64 * 4096)()
        n = self.H.h_load_order(self.h, buf, 4096)
        return list(buf[:n])

    def close(self):
        self.H.h_free(self.h)


def drain(s, limit=100000):
    for _ in range(limit):
        st = s.poll()
        if st["active"] == 0 and st["queued"] == 0:
            return
    raise AssertionError("scheduler did not drain")


def test_all_requests_complete_exactly(H):
    s = Sched(H, 1 << 20, 7)
    ids = [s.submit(2 + (i % 2), 1000 + 37 * i, 1 + 13 * i)[1] for i in range(30)]
    drain(s)
    for rid, i in zip(ids, range(30)):
        st, done, ta, td = s.state(rid)
        assert st == 2 and done == 1 + 13 * i and td > ta
    assert H.h_violations(s.h) == 0 and H.h_used(s.h) == 0
    s.close()


def test_budget_admission_fifo_and_reuse(H):
    budget = 10_000
    s = Sched(H, budget, 5)
    sizes = [4000, 4000, 4000, 1000, 9000, 500]
    ids = [s.submit(3, b, 12)[1] for b in sizes]
    first = s.poll()
    assert first["admitted"] == 2 and first["queued"] == 4   # third 4000 does not fit
    drain(s)
    assert s.load_order() == ids                             # strict FIFO, no overtaking
    assert H.h_peak(s.h) <= budget and H.h_violations(s.h) == 0
    s.close()


def test_request_larger_than_budget_is_refused(H):
    s = Sched(H, 4096, 5)
    rc, _ = s.submit(2, 5000, 10)
    assert rc == -6
    rc, _ = s.submit(2, 4096, 10)
    assert rc == 0
    rc, _ = s.submit(2, 100, 0)      # zero steps is refused too
    assert rc == -6
    drain(s)
    s.close()


def test_cancel_queued_and_active(H):
    s = Sched(H, 8000, 3)
    a = s.submit(2, 5000, 30)[1]
    b = s.submit(2, 5000, 30)[1]       # waits for a
    c = s.submit(2, 2000, 30)[1]
    s.poll()
    assert s.state(a)[0] == 1 and s.state(b)[0] == 0
    assert H.h_cancel(s.h, b) == 0     # queued
    assert H.h_cancel(s.h, a) == 0     # active: memory returns
    assert H.h_used(s.h) <= 2048 + 256
    drain(s)
    assert s.state(c)[0] == 2 and s.state(a)[0] == 3 and s.state(b)[0] == 3
    assert H.h_cancel(s.h, c) != 0     # finished requests cannot be cancelled
    assert H.h_release(s.h, c) == 0 and s.state(c)[0] == -1
    assert H.h_violations(s.h) == 0
    s.close()


def test_step_node_cap_least_remaining_work_first(H):
    """With a node cap a quantum advances the active requests in increasing
    order of remaining work (nodes x steps left, ties by id) that fit the cap
    together, passing over one that does not fit for smaller ones after it;
    every request still completes exactly."""
    s = Sched(H, 1 << 30, 10)
    H.h_set_step_nodes(s.h, 1000)
    # (nodes, steps): works 6000, 2000, 2000, 8000, 900, 10000
    spec = [(600, 10), (100, 20), (200, 10), (800, 10), (90, 10), (1000, 10)]
    ids = [s.submit_nodes(n, t) for n, t in spec]
    s.poll()
    # order by work: id4 (900), id1 (2000, lower id), id2 (2000), id0 (6000),
    # id3 (8000), id5 (10000); 90 + 100 + 200 + 600 = 990 fit, 800 and 1000 not
    assert s.last_launch() == [ids[4], ids[1], ids[2], ids[0]]
    s.poll()   # ids 4, 2, 0 finished after 10 steps; id1 has 10 left (work 1000)
    assert s.last_launch() == [ids[1], ids[3]]            # 100 + 800 <= 1000
    s.poll()   # id1 and id3 finished
    assert s.last_launch() == [ids[5]]                    # alone, at the cap
    drain(s)
    for rid, (n, t) in zip(ids, spec):
        st, done, _, _ = s.state(rid)
        assert st == 2 and done == t
    assert H.h_violations(s.h) == 0
    s.close()


def test_step_node_cap_single_request_above_cap_and_off(H):
    s = Sched(H, 1 << 30, 4)
    H.h_set_step_nodes(s.h, 50)
    big = s.submit_nodes(500, 8)          # above the cap: advanced alone
    s.poll()
    assert s.last_launch() == [big]
    small = s.submit_nodes(10, 8)
    s.poll()
    assert s.last_launch() == [small]     # less remaining work, and both do not fit
    H.h_set_step_nodes(s.h, 0)            # every active request again
    s.poll()
    assert sorted(s.last_launch()) == sorted([big, small])
    drain(s)
    assert s.state(big)[1] == 8 and s.state(small)[1] == 8
    assert H.h_violations(s.h) == 0
    s.close()


def test_step_node_cap_random_workload(H):
    rng = np.random.default_rng(4)
    s = Sched(H, 1 << 22, 7)
    H.h_set_step_nodes(s.h, 5000)
    ids, want = [], {}
    for it in range(400):
        if rng.random() < 0.6:
            n, t = int(rng.integers(1, 3000)), int(rng.integers(1, 60))
            rid = s.submit_nodes(n, t, nbytes=int(rng.integers(100, 50000)))
            ids.append(rid)
            want[rid] = t
        s.poll()
    drain(s)
    for rid in ids:
        st, done, _, _ = s.state(rid)
        assert st == 2 and done == want[rid]
    assert H.h_violations(s.h) == 0 and H.h_used(s.h) == 0
    s.close()


def test_latency_bookkeeping(H):
    s = Sched(H, 1 << 20, 10)
    rid = s.submit(3, 100, 35)[1]
    polls = 0
    while s.state(rid)[0] != 2:
        s.poll()
        polls += 1
    # ceil(35 / 10) = 4 quanta; each poll launches one and the next poll
    # observes its completion, so the request is done after the fifth poll
    assert polls == 5
    _, done, ta, td = s.state(rid)
    assert done == 35 and td > ta
    s.close()


def test_arena_coalescing_allows_full_budget_again(H):
    s = Sched(H, 64 * 1024, 2)
    ids = [s.submit(2, 8 * 1024, 3)[1] for _ in range(8)]
    drain(s)
    assert H.h_used(s.h) == 0
    big = s.submit(2, 64 * 1024, 1)[1]  # needs the whole arena in one block
    st = s.poll()
    assert st["admitted"] == 1
    drain(s)
    assert s.state(big)[0] == 2 and H.h_violations(s.h) == 0
    s.close()


def test_random_stress(H):
    rng = np.random.default_rng(7)
    budget = 200_000
    s = Sched(H, budget, 16)
    live = []
    for it in range(600):
        if rng.random() < 0.6:
            rc, rid = s.submit(int(rng.integers(2, 4)), int(rng.integers(1, 60_000)),
                               int(rng.integers(1, 200)))
            assert rc == 0
            live.append(rid)
        if live and rng.random() < 0.05:
            rid = live.pop(int(rng.integers(len(live))))
            H.h_cancel(s.h, rid)
        s.poll()
        assert H.h_used(s.h) <= budget
    drain(s)
    assert H.h_violations(s.h) == 0 and H.h_used(s.h) == 0
    assert H.h_peak(s.h) <= budget
    s.close()


FAILED = 4


def test_failed_request_retired_alone(H):
    """A request whose quantum reports an overflow is retired as Failed (its
    memory freed, never launched again) while the requests beside it finish
    with all their steps; later polls keep working and the failed request
    can be released."""
    s = Sched(H, 10_000, 10)
    ids = [s.submit(2, 1000, 35)[1] for _ in range(4)]
    H.h_fail_wait(s.h, ids[1])
    failed = 0
    for _ in range(50):
        out = (ctypes.c_uint32 * 5)()
        assert H.h_poll5(s.h, out) == 0
        failed += out[4]
        if out[1] == 0 and out[2] == 0:
            break
    assert failed == 1
    assert s.state(ids[1])[0] == FAILED
    for rid in ids[:1] + ids[2:]:
        st, done, _, _ = s.state(rid)
        assert st == 2 and done == 35
    assert H.h_used(s.h) == 0
    assert H.h_violations(s.h) == 0
    assert H.h_release(s.h, ids[1]) == 0
    # the server still admits and finishes new work
    rid = s.submit(2, 1000, 5)[1]
    for _ in range(5):
        s.poll()
    assert s.state(rid)[0] == 2
    H.h_free(s.h)


def test_failed_admission_retired_alone(H):
    """A request whose admission fails (its drawn initial state overflows) is
    retired as Failed at admission, never launched; FIFO admission goes on
    with the next request."""
    s = Sched(H, 2_500, 10)
    ids = [s.submit(2, 1000, 20)[1] for _ in range(4)]
    H.h_fail_load(s.h, ids[0])
    failed = 0
    for _ in range(50):
        out = (ctypes.c_uint32 * 5)()
        assert H.h_poll5(s.h, out) == 0
        failed += out[4]
        if out[1] == 0 and out[2] == 0:
            break
    assert failed == 1
    assert s.state(ids[0])[0] == FAILED
    assert all(s.state(r)[0] == 2 for r in ids[1:])
    assert H.h_used(s.h) == 0
    assert H.h_violations(s.h) == 0
    H.h_free(s.h)


def test_resident_requests_take_longer_advances(H):
    """Requests of at most the resident node count are advanced by up to the
    resident step count per poll, the others by the quantum; both finish
    with exactly their steps."""
    s = Sched(H, 1 << 20, 10)
    H.h_set_resident(s.h, 100, 50, 0)
    small = s.submit_nodes(64, 120)
    edge = s.submit_nodes(100, 70)
    big = s.submit_nodes(101, 45)
    s.poll()
    assert s.last_launch() == [small, edge, big]
    assert s.last_steps() == [50, 50, 10]
    polls = 1
    while True:
        st = s.poll()
        polls += 1
        if st["active"] == 0 and st["queued"] == 0:
            break
    # big: 45 steps at 10 per poll, so 5 launches, then one poll that retires
    assert polls == 6
    for rid, n in ((small, 120), (edge, 70), (big, 45)):
        st, done, _, _ = s.state(rid)
        assert st == 2 and done == n
    assert H.h_violations(s.h) == 0
    s.close()


def test_resident_advance_ended_early(H):
    """The executor may end a small request's advance early (here after 7 of
    up to 50 steps): the scheduler counts the steps taken, plans the next
    advance from them, and the request still finishes with exactly its
    steps."""
    s = Sched(H, 1 << 20, 10)
    H.h_set_resident(s.h, 100, 50, 7)
    small = s.submit_nodes(64, 120)
    big = s.submit_nodes(1000, 30)
    s.poll()
    assert s.last_steps() == [50, 10]
    s.poll()
    assert s.state(small)[1] == 7
    assert s.last_steps() == [50, 10]
    drain(s)
    st, done, _, _ = s.state(small)
    assert st == 2 and done == 120
    assert s.state(big)[:2] == (2, 30)
    assert H.h_violations(s.h) == 0
    s.close()


def test_resident_random_stress(H):
    """Random small and large requests with resident advances ended early at
    random points, cancellations and the node cap."""
    rng = np.random.default_rng(11)
    budget = 300_000
    s = Sched(H, budget, 16)
    H.h_set_resident(s.h, 500, 200, 0)
    live = []
    for it in range(500):
        if it % 50 == 0:
            H.h_set_resident(s.h, 500, 200, int(rng.integers(0, 40)))
        if it == 250:
            H.h_set_step_nodes(s.h, 3000)
        if rng.random() < 0.6:
            nodes = int(rng.integers(1, 1000))
            live.append(s.submit_nodes(nodes, int(rng.integers(1, 400)),
                                       int(rng.integers(1, 40_000))))
        if live and rng.random() < 0.05:
            H.h_cancel(s.h, live.pop(int(rng.integers(len(live)))))
        s.poll()
    drain(s)
    assert H.h_violations(s.h) == 0 and H.h_used(s.h) == 0
    s.close()


def _correction(H, ranges, w, tile_slot, times, nslots, lo=0.5, hi=2.0):
    f = H.h_tile_cost_correction
    f.restype = None
    f.argtypes = [ctypes.POINTER(ctypes.c_uint32), ctypes.c_uint32,
                  ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_uint32),
                  ctypes.POINTER(ctypes.c_uint64), ctypes.c_uint32, ctypes.c_double,
                  ctypes.c_double, ctypes.POINTER(ctypes.c_double)]
    r = np.ascontiguousarray(ranges, dtype=np.uint32)
    wv = np.ascontiguousarray(w, dtype=np.float64)
    ts = np.ascontiguousarray(tile_slot, dtype=np.uint32)
    tm = np.ascontiguousarray(times, dtype=np.uint64)
    out = np.zeros(nslots, dtype=np.float64)
    f(r.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), len(r) - 1,
      wv.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
      ts.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
      tm.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), nslots, lo, hi,
      out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def test_tile_cost_correction_attribution(H):
    """Slot 0's workgroups took 1.2 times as long per estimated unit as slot
    1's; slot 2 shares one workgroup with slot 1; slot 3 is walked by nobody
    (its workgroup's range is empty)."""
    # tiles: slot 0 x4 (w 1), slot 1 x4 (w 1), slot 2 x2 (w 2)
    w = [1.0] * 8 + [2.0, 2.0]
    slot = [0] * 4 + [1] * 4 + [2, 2]
    ranges = [0, 2, 4, 6, 10, 10]   # wg 2: slot 1 (2 tiles); wg 3: slot 1 + slot 2
    times = [240, 240, 200, 600, 999_999]
    c = _correction(H, ranges, w, slot, times, 4)
    # estimated 2, 2, 2, 6 units (wg 4 ignored): scale 12 / 1280 per tick,
    # ratios 1.125, 1.125, 0.9375, 0.9375 -- slot 0 at 1.2 times the others,
    # and the estimate-weighted mean ratio is 1
    np.testing.assert_allclose(c, [1.125, 0.9375, 0.9375, 1.0])
    # clamping
    c = _correction(H, ranges, w, slot, [900, 900, 100, 300, 0], 4, lo=0.8, hi=1.25)
    assert c[0] == 1.25 and c[1] == 0.8 and c[2] == 0.8 and c[3] == 1.0
    # no time measured: no correction
    np.testing.assert_array_equal(_correction(H, ranges, w, slot, [0] * 5, 4), [1.0] * 4)


def test_tile_cost_correction_shared_workgroup(H):
    """A workgroup's ratio goes to every slot of its range in proportion to
    the slot's estimated work there."""
    w = [3.0, 1.0, 1.0, 1.0, 1.0, 1.0]
    slot = [0, 1, 2, 2, 2, 2]
    ranges = [0, 2, 6]              # wg 0: slot 0 (3) + slot 1 (1); wg 1: slot 2 (4)
    c = _correction(H, ranges, w, slot, [150, 100], 3)
    # scale 8/250; ratios 150*8/250/4 = 1.2, 100*8/250/4 = 0.8
    np.testing.assert_allclose(c, [1.2, 1.2, 0.8])


def _split(w, grid):
    """The executor's split: boundary b where the running weight passes
    b / grid of the total, each tile to the range holding its larger half."""
    total = sum(w)
    out, acc, t = [0], 0.0, 0
    for b in range(1, grid):
        target = total * b / grid
        while t < len(w) and acc + 0.5 * w[t] < target:
            acc += w[t]
            t += 1
        out.append(t)
    out.append(len(w))
    return out


def test_tile_cost_correction_balances_the_walk(H):
    """Requests whose true cost per tile departs from the model by up to
    +-30 %: a few rounds of correction bring the slowest workgroup of the
    split within a few per cent of the mean."""
    rng = np.random.default_rng(3)
    nslots, grid = 64, 256
    ntile = rng.integers(8, 200, size=nslots)
    model = 1.0 + rng.uniform(0.05, 1.0, size=nslots)
    true = model * rng.uniform(0.7, 1.3, size=nslots)
    factor = np.ones(nslots)

    def walk():
        w, slot = [], []
        for s in range(nslots):
            for k in range(ntile[s]):
                w.append(model[s] * factor[s])
                slot.append(s)
        r = _split(w, grid)
        times = [int(1000 * sum(true[slot[t]] for t in range(r[b], r[b + 1])))
                 for b in range(grid)]
        return w, slot, r, times

    imb = []
    for _ in range(6):
        w, slot, r, times = walk()
        tv = np.array(times, dtype=np.float64)
        imb.append(tv.max() / tv[tv > 0].mean())
        factor *= _correction(H, r, w, slot, times, nslots, lo=0.75, hi=1.33)
    assert imb[0] > 1.15
    assert imb[-1] < 1.05 and imb[-1] < imb[0]


def test_tile_cost_correction_invariances(H):
    """Times proportional to the estimates leave every slot at 1, and a
    change of clock (all times scaled) leaves the corrections unchanged;
    an empty walk corrects nothing."""
    rng = np.random.default_rng(9)
    nslots, grid = 12, 40
    ntile = rng.integers(1, 30, size=nslots)
    w, slot = [], []
    for s in range(nslots):
        for k in range(ntile[s]):
            w.append(float(rng.uniform(1.0, 2.0)))
            slot.append(s)
    r = _split(w, grid)
    est = [sum(w[r[b]:r[b + 1]]) for b in range(grid)]
    times = [int(round(1e6 * e)) for e in est]
    np.testing.assert_allclose(_correction(H, r, w, slot, times, nslots), 1.0, rtol=1e-5)
    skew = [int(t * (1.0 + 0.3 * ((b * 7) % 5) / 4)) for b, t in enumerate(times)]
    c1 = _correction(H, r, w, slot, skew, nslots)
    c2 = _correction(H, r, w, slot, [3 * t for t in skew], nslots)
    np.testing.assert_allclose(c1, c2, rtol=1e-12)
    assert not np.allclose(c1, 1.0)
    np.testing.assert_array_equal(_correction(H, [0], [], [], [], 3), [1.0, 1.0, 1.0])
