"""Lattices whose state buffer passes 2^31 bytes (offsets beyond 32-bit
signed range): one full-lattice step against the oracle for D1Q2 (uint32,
L = 2^28, 2 GiB per state buffer) and D2Q5 (uint32, 10800 x 10000 nodes,
2.16 GB), with the initial states drawn on the device, then mass
conservation over more steps."""
import ctypes
import sys

import numpy as np
import pytest

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


def _state_bytes(ilg, cfg):
    return int(ilg.lib.ilg_state_bytes(ctypes.byref(cfg)))


def test_d1q2_u32_l2p28(ilg, oracle_lib):
    L = 1 << 28
    assert _state_bytes(ilg, ilg.make_config(2, L, 4, 1.6, 3)) >= 1 << 31
    _say("[large] D1Q2 uint32 L=2^28: device init")
    lat = ilg.Lattice(2, L, 4, 1.6, 3, None, realization=1)
    lat.init_poisson_sine(30.0, 10.0, 8)
    init = lat.state()
    mass0 = int(init.astype(np.int64).sum())
    lat.step(1)
    got = lat.state()
    _say("[large] oracle step")
    ref, _, ov = oracle_lib.run(oracle_lib.Params(2, 1.6), init, 1, seed=3, realization=1)
    assert not ov
    np.testing.assert_array_equal(got, ref)
    del init, ref, got
    lat.step(9)
    assert lat.moments()["mass"] == mass0
    lat.close()


def test_d2q5_u32_10800x10000(ilg, oracle_lib):
    lx, ly = 10800, 10000
    assert _state_bytes(ilg, ilg.make_config(5, lx, 4, 1.7, 5, height=ly)) >= 1 << 31
    _say("[large] D2Q5 uint32 10800 x 10000: device init")
    lat = ilg.Lattice(5, lx, 4, 1.7, 5, None, height=ly)
    lat.init_poisson_sine(60.0, 20.0, 9)
    init = lat.state()
    mass0 = int(init.astype(np.int64).sum())
    lat.step(1)
    got = lat.state()
    _say("[large] oracle step")
    ref, _, ov = oracle_lib.run2d(oracle_lib.Params(5, 1.7), init, 1, seed=5)
    assert not ov
    np.testing.assert_array_equal(got, ref)
    del init, ref, got
    lat.step(5)
    assert lat.moments()["mass"] == mass0
    lat.close()
