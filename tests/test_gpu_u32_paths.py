"""uint32 lattices take the straight-line and generic sampler paths in
32-bit arithmetic while every count of the wavefront is below 2^29, and the
generic path in 64-bit arithmetic otherwise.  Parity at both sides of that
switch: one wavefront holding a count of 2^29 - 1 and another holding
2^29 + 7 (each a binomial of about 2^23 chunks) against the oracle, and
states near 2^32 under pure streaming (a zero collision fraction) against
the exact flip-and-stream map."""
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


@pytest.mark.parametrize("q", [2, 3])
def test_counts_either_side_of_the_32_bit_switch(ilg, oracle_lib, q):
    L = 128                                     # two wavefronts
    init = W.init_poisson_iid(q, L, 30.0, 4, init_seed=91 + q)
    init[q // 2, 10] = (1 << 29) - 1            # wavefront 0: 32-bit generic path
    init[0, 70] = (1 << 29) + 7                 # wavefront 1: 64-bit generic path
    _say(f"[u32 paths] q={q}: one step with counts 2^29 - 1 and 2^29 + 7")
    lat = ilg.Lattice(q, L, 4, 1.5, 5, init)
    lat.step(1)
    got = lat.state()
    lat.close()
    ref, _, ov = oracle_lib.run(oracle_lib.Params(q, 1.5), init, 1, seed=5)
    assert not ov
    np.testing.assert_array_equal(got, ref)
    assert int(got.astype(np.int64).sum()) == int(init.astype(np.int64).sum())


def test_streaming_near_the_count_limit(ilg):
    """omega = 2: no particle collides (flip, then streaming only), so counts
    up to 2^32 - 1 move without overflow, exactly as the flip-and-stream map
    moves them."""
    rng = np.random.default_rng(7)
    L = 200
    init = rng.integers((1 << 32) - 5000, (1 << 32) - 1, size=(3, L), dtype=np.uint64)
    init = init.astype(np.uint32)
    lat = ilg.Lattice(3, L, 4, 2.0, 9, init)
    lat.step(5)
    got = lat.state()
    lat.close()
    # (the oracle would take one draw per chunk of 2^32 counts: the exact map
    # is the reference here)
    want = init.copy()
    for _ in range(5):
        f = want[::-1].copy()                   # flip: a_i = n_{q-1-i}
        want = np.stack([np.roll(f[0], -1), f[1], np.roll(f[2], 1)])
    np.testing.assert_array_equal(got, want)
