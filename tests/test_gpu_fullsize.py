"""Full-state parity at the full sizes of the benchmark workloads.

The D1Q3 lattice of 2^24 nodes (uint16, Poisson(50), omega = 1.8, 2000 steps)
runs on the GPU once, in the launch configuration the benchmark times (one
step kernel launch per step), keeping the whole state at steps 1, 2, 10 and
every 250 steps to 2000.  The oracle then runs the same 2000 steps from the
same initial state, in segments of 250 steps (one test each, in order; each
segment continues from the oracle's own state), and every kept state must be
equal to the oracle's entry by entry, with equal state hashes.  The oracle
takes its inputs only from the workload generator and its own earlier
output."""
import sys

import numpy as np
import pytest

import ilg_workloads as W

pytestmark = pytest.mark.gpu

CHECKS = (1, 2, 10) + tuple(range(250, 2001, 250))
SEGMENTS = [(s, s + 250) for s in range(0, 2000, 250)]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ilg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2203_01380_amd as ilg
    return ilg


@pytest.fixture(scope="module")
def headline_gpu(ilg):
    """GPU states and hashes of the 2^24-node lattice at every checked step."""
    spec, init = W.workload_d1q3_big()
    assert spec.steps == CHECKS[-1]
    lat = ilg.Lattice(spec.q, spec.length, spec.count_bytes, spec.omega, spec.seed, init)
    states, hashes = {}, {}
    t = 0
    for c in CHECKS:
        lat.step(c - t)
        t = c
        states[c] = lat.state()
        hashes[c] = lat.hash()
    lat.close()
    return spec, init, states, hashes


_ORACLE = {}


@pytest.mark.parametrize("seg", SEGMENTS, ids=[f"steps{a}-{b}" for a, b in SEGMENTS])
def test_headline_lattice_full_state(headline_gpu, oracle_lib, seg):
    spec, init, states, hashes = headline_gpu
    a, b = seg
    if a == 0:
        _ORACLE.clear()
        _ORACLE.update(t=0, state=init)
    assert _ORACLE.get("t") == a, "segments run in order, each from the previous one's state"
    p = oracle_lib.Params(spec.q, spec.omega)
    for c in [c for c in CHECKS if a < c <= b]:
        _say(f"[full-size D1Q3 2^24] oracle steps {_ORACLE['t']}..{c}")
        cur, _, ov = oracle_lib.run(p, _ORACLE["state"], c - _ORACLE["t"], seed=spec.seed,
                                    t0=_ORACLE["t"])
        assert not ov
        _ORACLE.update(t=c, state=cur)
        got = states[c]
        if not np.array_equal(got, cur):
            bad = np.argwhere(got != cur)
            raise AssertionError(f"step {c}: {len(bad)} entries differ, first (i, x) = "
                                 f"{tuple(bad[0])}")
        assert hashes[c] == oracle_lib.state_hash(cur), f"step {c}: hash"
    assert int(_ORACLE["state"].astype(np.int64).sum()) == int(init.astype(np.int64).sum())
