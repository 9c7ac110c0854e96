"""GPU test of ilg_step_noalloc (the entry point for callers that cannot
allocate device memory), called through the C ABI: its results equal the
same configuration stepped through ilg_create_on + ilg_step, on two calls in
a row with different configurations (the second a smaller lattice), and its
sticky overflow report is raised once and then cleared."""
import ctypes

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


def _device_state(q, L, cb, init, height=0):
    import torch
    nodes = L * (height if q == 5 else 1)
    pitch = (nodes + 63) // 64 * 64
    dt = torch.int16 if cb == 2 else torch.int32
    b0 = torch.zeros((q, pitch), dtype=dt, device="cuda")
    b1 = torch.zeros_like(b0)
    host = np.ascontiguousarray(init).reshape(q, nodes).view(np.int16 if cb == 2 else np.int32)
    b0[:, :nodes] = torch.from_numpy(host).to("cuda")
    return b0, b1, nodes


def _noalloc(ilg, m, init, nsteps, sync=1):
    import torch
    q, L, cb = m["q"], m["length"], m["count_bytes"]
    b0, b1, nodes = _device_state(q, L, cb, init, m.get("height", 0))
    cfg = ilg.make_config(q, L, cb, m["omega"], m["seed"], m.get("realization", 0),
                          m.get("t0", 0), 0.0, "auto", m.get("height", 0), m.get("rounds", 10),
                          m.get("exchange", False))
    st = torch.cuda.current_stream()
    rc = ilg.lib.ilg_step_noalloc(ctypes.byref(cfg), ctypes.c_void_p(b0.data_ptr()),
                                  ctypes.c_void_p(b1.data_ptr()), nsteps,
                                  ctypes.c_void_p(st.cuda_stream), sync)
    torch.cuda.synchronize()
    out = (b1 if nsteps & 1 else b0)[:, :nodes].cpu().numpy()
    dt = np.uint16 if cb == 2 else np.uint32
    return rc, out.view(dt).reshape(init.shape)


def _alone(ilg, m, init, nsteps):
    lat = ilg.Lattice(m["q"], m["length"], m["count_bytes"], m["omega"], m["seed"], init,
                      realization=m.get("realization", 0), t0=m.get("t0", 0),
                      height=m.get("height", 0), rounds=m.get("rounds", 10),
                      exchange=m.get("exchange", False))
    lat.step(nsteps)
    out = lat.state()
    lat.close()
    return out


def test_noalloc_equals_step_on_two_calls(ilg):
    big = dict(q=3, length=100003, count_bytes=2, omega=1.8, seed=5, realization=1, t0=3)
    init_big = W.init_poisson_iid(3, big["length"], 50.0, 2, init_seed=11)
    rc, got = _noalloc(ilg, big, init_big, 37)
    assert rc == 0, ilg.lib.ilg_last_error()
    np.testing.assert_array_equal(got, _alone(ilg, big, init_big, 37))
    # a second call, smaller and with other rates, count type and seed: the
    # scratch array's tables are rewritten
    small = dict(q=2, length=4099, count_bytes=4, omega=1.3, seed=9, realization=2, t0=0)
    init_small = W.init_poisson_iid(2, small["length"], 40.0, 4, init_seed=12)
    rc, got = _noalloc(ilg, small, init_small, 20)
    assert rc == 0, ilg.lib.ilg_last_error()
    np.testing.assert_array_equal(got, _alone(ilg, small, init_small, 20))


def test_noalloc_other_forms(ilg):
    """D2Q5 and the D1Q2 exchange form with 7-round draws, asynchronous."""
    rng = np.random.default_rng(3)
    d2 = dict(q=5, length=70, height=30, count_bytes=2, omega=1.6, seed=4, t0=11)
    init = rng.poisson(30.0, size=(5, 30, 70)).astype(np.uint16)
    rc, got = _noalloc(ilg, d2, init, 9, sync=0)
    assert rc == 0, ilg.lib.ilg_last_error()
    np.testing.assert_array_equal(got, _alone(ilg, d2, init, 9))
    ex = dict(q=2, length=3001, count_bytes=2, omega=1.7, seed=8, rounds=7, exchange=True)
    init = W.init_poisson_iid(2, 3001, 40.0, 2, init_seed=13)
    rc, got = _noalloc(ilg, ex, init, 12)
    assert rc == 0, ilg.lib.ilg_last_error()
    np.testing.assert_array_equal(got, _alone(ilg, ex, init, 12))


def test_noalloc_overflow_reported_once(ilg):
    """omega = 1, no flip, 3 x 40000 particles per node: about 80000 go to the
    rest velocity, beyond uint16.  The synchronous call reports it; the
    report clears the word, so the next clean call succeeds."""
    bad = dict(q=3, length=2000, count_bytes=2, omega=1.0, seed=1)
    rc, _ = _noalloc(ilg, bad, np.full((3, 2000), 40000, np.uint16), 1, sync=1)
    assert rc == -4
    ok = dict(q=3, length=5000, count_bytes=2, omega=1.5, seed=2)
    init = W.init_poisson_iid(3, 5000, 30.0, 2, init_seed=14)
    rc, got = _noalloc(ilg, ok, init, 4, sync=1)
    assert rc == 0, ilg.lib.ilg_last_error()
    np.testing.assert_array_equal(got, _alone(ilg, ok, init, 4))


def test_noalloc_rejects_bad_arguments(ilg):
    m = dict(q=3, length=100, count_bytes=2, omega=1.5, seed=1)
    b0, b1, _ = _device_state(3, 100, 2, np.zeros((3, 100), np.uint16))
    cfg = ilg.make_config(3, 100, 2, 1.5, 1, 0, 0, 0.0, "auto", 0, 10, False)
    assert ilg.lib.ilg_step_noalloc(ctypes.byref(cfg), ctypes.c_void_p(b0.data_ptr()),
                                    ctypes.c_void_p(b0.data_ptr()), 1, None, 1) == -1
    cfg.t0 = (1 << 32) - 1
    assert ilg.lib.ilg_step_noalloc(ctypes.byref(cfg), ctypes.c_void_p(b0.data_ptr()),
                                    ctypes.c_void_p(b1.data_ptr()), 2, None, 1) == -5
