"""Pins of the D1Q2 exchange form (draw specification v3).

The paper's D1Q2 sampling collision removes each particle with probability
omega* and sends it to either velocity with probability 1/2, so a particle
ends on the opposite velocity with probability omega*/2, independently of the
others.  The exchange form draws the two crossing counts directly.  Pinned
here: the exact law of the exchange form equals the paper's collision law
(independent-particle transition matrix) whenever the fixed-point crossing
probability is exactly half the removal probability; the oracle's samples
follow the exact exchange law (chi-square); the draw order (crossings from -1
first, then from +1, chunk by chunk, none for an empty velocity) recomputed
from the Philox words and the exact tables; the fixed-point rounding of the
crossing probability; and a lattice run conserving mass and differing from
the three-binomial form."""
import itertools
import math

import numpy as np
import pytest
from scipy import stats

from oracle import exact
from oracle import oracle as O


def test_crossing_probability_fixed_point():
    # omega* = 2 - omega with the flip; P_x = round-half-even(omega* 2^31)
    assert exact.fixed_point_params(1.5, q=2)["P_x"] == 1 << 30
    assert exact.fixed_point_params(2.0, q=2)["P_x"] == 0
    assert exact.fixed_point_params(1.0, flip="off", q=2)["P_x"] == 1 << 31
    fp = exact.fixed_point_params(1.8, q=2)
    assert fp["P_x"] == round((2.0 - 1.8) * 2.0 ** 31)
    assert abs(fp["P_x"] - fp["P"] / 2) <= 0.5


@pytest.mark.parametrize("P", [2 * 12345, 1 << 31, 2 * 858993459, 2 * 2000000000 - 2])
@pytest.mark.parametrize("flip", [False, True])
def test_exchange_law_is_the_collision_law(P, flip):
    """With P = 2 P_x the crossing law and the paper's collision law (remove
    with p, redistribute with 1/2 each) are the same distribution."""
    for a in itertools.product(range(6), repeat=2):
        ex = exact.collision_law_exchange(a, P // 2, flip)
        ref = exact.collision_law_particles(a, 2, P, 0, flip)
        keys = set(ex) | set(ref)
        for k in keys:
            assert ex.get(k, 0) == ref.get(k, 0), (a, k)


def test_three_binomial_law_differs_when_probabilities_differ():
    """Guard: the comparison above is sensitive (a wrong crossing
    probability changes the law)."""
    a = (3, 2)
    ex = exact.collision_law_exchange(a, 1 << 29, False)
    ref = exact.collision_law_particles(a, 2, 1 << 31, 0, False)
    assert any(ex.get(k, 0) != ref.get(k, 0) for k in set(ex) | set(ref))


@pytest.mark.parametrize("omega,rounds", [(1.5, 10), (1.8, 10), (1.1, 10), (0.6, 10), (1.7, 7)])
def test_oracle_samples_follow_exchange_law(omega, rounds):
    params = O.Params(2, omega, rounds=rounds, exchange=True)
    N = 20000
    worst = 1.0
    for a in itertools.product(range(7), repeat=2):
        if sum(a) == 0:
            continue
        law = exact.collision_law_exchange(a, params.P_x, params.flip)
        samples = O.collide_samples(params, a, N, seed=(a[0] * 13 + a[1]) & 0xFFFF, t=5)
        assert np.all(samples.sum(axis=1) == sum(a))
        hist = {}
        for s in samples:
            k = tuple(int(v) for v in s)
            hist[k] = hist.get(k, 0) + 1
        assert set(hist) <= {k for k, v in law.items() if v > 0}
        outcomes = sorted(law)
        exp = np.array([float(law[k]) * N for k in outcomes])
        obs = np.array([hist.get(k, 0) for k in outcomes], dtype=np.float64)
        keep = exp >= 5
        if keep.sum() < 2:
            continue
        chi2 = ((obs[keep] - exp[keep]) ** 2 / exp[keep]).sum()
        worst = min(worst, stats.chi2.sf(chi2, int(keep.sum()) - 1))
    assert worst > 1e-5


def _chunk_count(tab, m, u):
    base = (m - 1) * m // 2
    row = tab[base:base + m]
    return int(np.sum(row <= np.uint32(u)))


@pytest.mark.parametrize("a", [(5, 9), (0, 9), (7, 0), (70, 3), (3, 130), (64, 64)])
def test_draw_order(a):
    """Crossing counts recomputed from the Philox words: X over the chunks of
    a_- first, then Y over the chunks of a_+ (flip off: omega <= 1)."""
    params = O.Params(2, 0.9, exchange=True)
    seed, t, x = 77, 11, 3
    key = [seed & 0xFFFFFFFF, seed >> 32]
    words = []
    for b in range(3):
        words.extend(int(w) for w in O.philox([x, t, 0, b], key))
    j = 0

    def binom(n):
        nonlocal j
        total = 0
        while n > 0:
            m = min(64, n)
            total += _chunk_count(params.tab_p, m, words[j])
            j += 1
            n -= m
        return total

    X = binom(a[0])
    Y = binom(a[1])
    want = (a[0] - X + Y, a[1] - Y + X)
    # collide_samples keys sample s at node index s: run x + 1 samples
    got = O.collide_samples(params, a, x + 1, seed=seed, t=t)[x]
    assert tuple(int(v) for v in got) == want


def test_lattice_run_conserves_mass_and_differs_from_three_binomials():
    rng = np.random.default_rng(6)
    init = rng.poisson(30, size=(2, 700)).astype(np.uint16)
    a, _, _ = O.run(O.Params(2, 1.6), init, 6, seed=8)
    b, _, ov = O.run(O.Params(2, 1.6, exchange=True), init, 6, seed=8)
    assert not ov
    assert int(b.astype(np.int64).sum()) == int(init.astype(np.int64).sum())
    assert (a != b).mean() > 0.3


def test_exchange_needs_d1q2():
    with pytest.raises(ValueError):
        O.Params(3, 1.5, exchange=True)


def test_mean_crossing_rate():
    """Mean of c_- after one collision: a_- (1 - p_x) + a_+ p_x (ideal
    binomial means), within five standard errors."""
    params = O.Params(2, 1.3, exchange=True)
    a = (40, 10)
    a_f = (a[1], a[0])          # omega > 1: flipped first
    px = params.P_x / 2.0 ** 32
    s = O.collide_samples(params, a, 40000, seed=3, t=1).astype(np.float64)
    mean = a_f[0] * (1 - px) + a_f[1] * px
    var = (a_f[0] + a_f[1]) * px * (1 - px)
    assert abs(s[:, 0].mean() - mean) < 5 * math.sqrt(var / s.shape[0])
