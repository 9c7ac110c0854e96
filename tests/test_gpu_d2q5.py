"""GPU parity of the D2Q5 lattice gas with the flip (the paper's flip on a
two-dimensional five-velocity set) against the oracle: every compared step
bit-exact over lattice shapes whose 1024-node tiles wrap rows, both count
types, special rates, multi-chunk counts, per-step hashes, moments, the
device-drawn initial state, a 2048 x 2048 lattice, and the layout checks of
the batched and serving forms."""
import sys

import numpy as np
import pytest

from oracle import oracle as O

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


def _run_both(ilg, lx, ly, cb, omega, init, steps, seed=1, r=0, t0=0, flip="auto", theta=0.0,
              use_torch=True, check_every=1):
    _say(f"[d2q5] {lx}x{ly} cb={cb} omega={omega} steps={steps} flip={flip} theta={theta}")
    p = O.Params(5, omega, theta=theta or 1.0 / 3.0, flip=flip)
    lat = ilg.Lattice(5, lx, cb, omega, seed, init, realization=r, t0=t0, theta=theta, flip=flip,
                      use_torch=use_torch, height=ly)
    cur = init.copy()
    done = 0
    while done < steps:
        n = min(check_every, steps - done)
        lat.step(n)
        cur, hs, ov = O.run2d(p, cur, n, seed=seed, realization=r, t0=t0 + done, hashes=True)
        assert not ov
        done += n
        got = lat.state()
        if not np.array_equal(got, cur):
            bad = np.argwhere(got != cur)
            raise AssertionError(f"state mismatch after {done} steps at {bad[:5].tolist()}")
        assert lat.hash() == int(hs[-1])
    lat.close()
    return cur


@pytest.mark.parametrize("lx,ly", [(1, 1), (1, 7), (7, 1), (3, 5), (64, 64), (1023, 3),
                                   (1000, 33), (2049, 2), (31, 257)])
@pytest.mark.parametrize("cb", [2, 4])
def test_shapes_and_types(ilg, lx, ly, cb):
    rng = np.random.default_rng(lx * 1000 + ly + cb)
    dt = np.uint16 if cb == 2 else np.uint32
    init = rng.poisson(25.0, size=(5, ly, lx)).astype(dt)
    _run_both(ilg, lx, ly, cb, 1.6, init, steps=5, seed=3 + lx, r=2)


@pytest.mark.parametrize("omega,flip,theta", [(2.0, "auto", 0.0), (1.0, "off", 0.0),
                                              (1.0, "on", 0.0), (0.3, "auto", 0.0),
                                              (1.9, "auto", 0.2), (0.7, "auto", 0.45),
                                              (1.05, "auto", 0.0)])
def test_special_rates(ilg, omega, flip, theta):
    rng = np.random.default_rng(17)
    init = rng.poisson(30.0, size=(5, 40, 50)).astype(np.uint32)
    _run_both(ilg, 50, 40, 4, omega, init, steps=6, seed=9, flip=flip, theta=theta)


@pytest.mark.parametrize("omega", [1.0, 1.3, 1.5, 1.62])
def test_collided_beyond_one_chunk(ilg, omega):
    """Movers' counts in one chunk, rest counts in one or two, and more than
    64 collided particles in some or all lanes of a wave (M is about omega*
    times the density 150): the redistribution continues chunk by chunk
    after the straight-line removal."""
    rng = np.random.default_rng(int(omega * 100))
    means = np.array([25.0, 25.0, 50.0, 25.0, 25.0])[:, None, None]
    init = rng.poisson(means, size=(5, 80, 96)).astype(np.uint16)
    _run_both(ilg, 96, 80, 2, omega, init, steps=8, seed=21, r=5)


@pytest.mark.parametrize("cb,omega", [(2, 1.0), (4, 1.0), (2, 1.15)])
def test_redistribution_layouts(ilg, cb, omega):
    """Rows of 64 nodes (one wave each) whose counts put M = sum k_i in
    129..192 with some rest removals of two chunks (the last split's word is
    then the thirteenth), M near 192 (R above two chunks: the generic
    redistribution), M above 192, M in 65..128, and M about 180 (m_x or m_y
    above one chunk in some lanes: the last two splits chunk by chunk)."""
    rng = np.random.default_rng(77 + cb)
    lx, ly = 64, 40
    dt = np.uint16 if cb == 2 else np.uint32
    init = np.empty((5, ly, lx), dtype=dt)
    for y in range(ly):
        mode = y % 5
        if mode == 0:
            mov, rest = (18, 27), (58, 72)
        elif mode == 1:
            mov, rest = (30, 33), (58, 65)
        elif mode == 2:
            mov, rest = (38, 45), (60, 70)
        elif mode == 3:
            mov, rest = (10, 21), (30, 51)
        else:
            mov, rest = (28, 31), (60, 66)
        for i in (0, 1, 3, 4):
            init[i, y] = rng.integers(mov[0], mov[1], lx)
        init[2, y] = rng.integers(rest[0], rest[1], lx)
    _run_both(ilg, lx, ly, cb, omega, init, steps=4, seed=23, r=2)


def test_multi_chunk_counts(ilg):
    """Counts above 64 (several chunks, draws past the eager blocks)."""
    rng = np.random.default_rng(4)
    init = rng.poisson(150.0, size=(5, 30, 70)).astype(np.uint16)
    init[:, :3, :5] = 900
    _run_both(ilg, 70, 30, 2, 1.3, init, steps=6, seed=11, check_every=2)
    _run_both(ilg, 70, 30, 2, 1.0, init, steps=3, seed=12, use_torch=False)


def test_moments_d2q5(ilg):
    """Per-node rho, J_x and E of the GPU after three steps against the raw
    moments of the oracle's state after the same three steps."""
    from oracle import exact
    rng = np.random.default_rng(5)
    init = rng.poisson(20.0, size=(5, 12, 33)).astype(np.uint16)
    lat = ilg.Lattice(5, 33, 2, 1.4, 1, init, height=12)
    lat.step(3)
    m = lat.moments(per_node=True)
    lat.close()
    ref, _, _ = O.run2d(O.Params(5, 1.4), init, 3, seed=1)
    rho, j, e = exact.moments_raw(ref, 5)
    assert m["mass"] == int(init.astype(np.int64).sum())
    np.testing.assert_array_equal(m["rho"], rho)
    np.testing.assert_array_equal(m["j"], j)
    np.testing.assert_array_equal(m["e"], e)


def test_device_init_d2q5(ilg):
    lx, ly = 97, 41
    lat = ilg.Lattice(5, lx, 2, 1.7, 6, None, realization=3, height=ly)
    lat.init_poisson_sine(120.0, 80.0, 44)
    got = lat.state()
    want, ov = O.init_poisson_sine(5, 2, lx, 120.0, 80.0, 44, realization=3, height=ly)
    assert not ov
    np.testing.assert_array_equal(got, want)
    lat.step(4)
    after = lat.state()
    lat.close()
    ref, _, _ = O.run2d(O.Params(5, 1.7), want, 4, seed=6, realization=3)
    np.testing.assert_array_equal(after, ref)


def test_full_size_2048(ilg):
    """2048 x 2048 nodes, uint16: one whole-lattice step against the oracle,
    then 20 more steps conserve the mass."""
    lx = ly = 2048
    _say("[d2q5] 2048 x 2048")
    lat = ilg.Lattice(5, lx, 2, 1.8, 1, None, height=ly)
    lat.init_poisson_sine(150.0, 0.0, 2)
    init = lat.state()
    lat.step(1)
    ref, _, _ = O.run2d(O.Params(5, 1.8), init, 1, seed=1)
    np.testing.assert_array_equal(lat.state(), ref)
    lat.step(20)
    assert lat.moments()["mass"] == int(init.astype(np.int64).sum())
    lat.close()


def test_batch_and_server_check_d2q5_layouts(ilg):
    """The batched and serving forms take D2Q5 members as [5][height][length]
    (parity in test_gpu_batch_d2q5.py and test_gpu_serve.py): a flattened
    state is refused, and so are the 1D diagnostics for a D2Q5 batch."""
    m = dict(q=5, length=8, count_bytes=2, omega=1.5, seed=1, height=4)
    init = np.zeros((5, 4, 8), dtype=np.uint16)
    with pytest.raises(ValueError):
        ilg.Batch([m], [init.reshape(5, 32)])
    with pytest.raises(ilg.IlgError):
        ilg.Batch([m], [init], sk_every=2, nk=2)
    srv = ilg.Server(1 << 20, 10)
    try:
        with pytest.raises(ValueError):
            srv.submit(m, init.reshape(5, 32), 5)
        rid = srv.submit(m, init, 5)
        while srv.poll()["active"]:
            pass
        np.testing.assert_array_equal(srv.result(rid), init)   # an empty lattice stays empty
    finally:
        srv.close()


def test_rest_count_chunk_layouts(ilg):
    """Rest counts around one and two chunks (64/65, 128/129) mixed within
    wavefronts, movers 1..40: the straight-line path with a per-lane shift
    of the later draws, and the generic path past 128."""
    rng = np.random.default_rng(23)
    lx, ly = 256, 24
    init = rng.integers(1, 41, size=(5, ly, lx)).astype(np.uint16)
    init[2] = rng.choice([1, 40, 64, 65, 100, 128, 129, 150], size=(ly, lx))
    init[2, :8] = rng.integers(60, 129, size=(8, lx))      # rows inside the fast path
    _run_both(ilg, lx, ly, 2, 1.8, init, steps=6, seed=29)
    _run_both(ilg, lx, ly, 2, 1.2, init, steps=4, seed=30)
