"""GPU parity of batched D2Q5 ensembles: members of many shapes (1 x 1,
single rows and columns, widths below, at and above a workgroup, ragged),
rates on both sides of one (omega = 2, 1 and 0.5 included), start steps,
both count types, 10- and 7-round draws; every member bit-exact against the
oracle's 2D run after two graph runs; every workgroup shape the same bits;
the plain form gives the same bits; 1D diagnostics rejected."""
import sys
from concurrent.futures import ThreadPoolExecutor

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


SHAPES = [(1, 1), (2, 3), (1, 40), (40, 1), (33, 7), (64, 64), (100, 3), (7, 150), (1025, 2),
          (513, 5), (90, 90), (17, 61)]


def _members(cb, seed, rounds=10):
    rng = np.random.default_rng(seed)
    dt = np.uint16 if cb == 2 else np.uint32
    omegas = [2.0, 1.0, 0.5, 1.5, 1.98, 0.9]
    members, inits = [], []
    for r, (lx, ly) in enumerate(SHAPES):
        om = omegas[r] if r < len(omegas) else float(rng.uniform(0.3, 2.0))
        members.append(dict(q=5, length=lx, height=ly, count_bytes=cb, omega=om,
                            seed=3000 + r, realization=r, t0=int(rng.integers(0, 400)),
                            rounds=rounds))
        init = rng.poisson([[[25.0]], [[25.0]], [[50.0]], [[25.0]], [[25.0]]],
                           size=(5, ly, lx)).astype(dt)
        if r == 5:
            init[2, :3] = 150    # rest populations past one chunk
        inits.append(init)
    return members, inits


def _oracle(O, m, init, steps):
    p = O.Params(5, m["omega"], rounds=m["rounds"])
    out, _, ov = O.run2d(p, init, steps, seed=m["seed"], realization=m["realization"],
                         t0=m["t0"])
    assert not ov
    return out


@pytest.mark.parametrize("cb,rounds", [(2, 10), (4, 10), (2, 7)])
def test_members_exact(ilg, oracle_lib, cb, rounds):
    members, inits = _members(cb, 11 + cb + rounds, rounds)
    _say(f"[batch d2q5] cb={cb} rounds={rounds}")
    b = ilg.Batch(members, inits)
    b.run(9)
    b.run(8)
    with ThreadPoolExecutor(6) as ex:
        refs = list(ex.map(lambda r: _oracle(oracle_lib, members[r], inits[r], 17),
                           range(len(members))))
    for r, ref in enumerate(refs):
        got = b.state(r)
        assert got.shape == (5, members[r]["height"], members[r]["length"])
        np.testing.assert_array_equal(got, ref, err_msg=f"member {r} {SHAPES[r]}")
    b.close()


def test_every_shape_same_bits_and_plain(ilg):
    members, inits = _members(2, 5)
    ref = None
    for shape in range(ilg.Batch.shape_count()):
        b = ilg.Batch(members, inits)
        b.set_shape(shape)
        b.run(7)
        states = [b.state(r) for r in range(len(members))]
        b.close()
        if ref is None:
            ref = states
            continue
        for r in range(len(members)):
            np.testing.assert_array_equal(states[r], ref[r], err_msg=f"shape {shape} member {r}")
    for r in [0, 4, 5, 8, 10]:
        m = members[r]
        lat = ilg.Lattice(5, m["length"], 2, m["omega"], m["seed"], inits[r], height=m["height"],
                          realization=m["realization"], t0=m["t0"])
        lat.step(7)
        np.testing.assert_array_equal(lat.state(), ref[r], err_msg=f"member {r} plain")
        lat.close()


def test_mass_conserved_and_diagnostics_rejected(ilg):
    members, inits = _members(4, 9)
    b = ilg.Batch(members, inits)
    b.tune(5)
    b.run(40)
    for r in range(len(members)):
        assert int(b.state(r).astype(np.int64).sum()) == int(inits[r].astype(np.int64).sum())
    b.close()
    with pytest.raises(ilg.IlgError):
        ilg.Batch(members, inits, sk_every=5, nk=4)
    with pytest.raises(ilg.IlgError):
        ilg.Batch(members, inits, amp_every=5, max_amp=4)
