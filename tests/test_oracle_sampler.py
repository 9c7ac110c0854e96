"""Pins for the oracle's fixed-point binomial tables and sampling collision.

Tables are checked against the textbook binomial CDF written directly with
binomial coefficients (the oracle builds them by repeated convolution); the
sampler's histograms are checked against exact laws in rational arithmetic,
the collision law being the independent-particle reading of the paper's
sampling collision (Integer Lattice Gas section: a fraction omega* of the
particles, picked at random, redistributed to velocity i with probability w_i).
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

from oracle import exact

TWO32 = 1 << 32
P_VALUES = [1, 85899346, 858993459, 1 << 31, 2863311531, TWO32 - 1, TWO32]


def _cdf_floor_direct(m, P, j):
    """floor(2^32 * sum_{i<=j} C(m,i) p^i (1-p)^(m-i)) with p = P/2^32."""
    p = Fraction(P, TWO32)
    cdf = sum(Fraction(math.comb(m, i)) * p ** i * (1 - p) ** (m - i) for i in range(j + 1))
    return math.floor(cdf * TWO32)


def test_fixed_point_parameters():
    fp = exact.fixed_point_params(1.8)
    assert fp["flip"] and fp["P"] == 858993459
    assert exact.fixed_point_params(1.0)["P"] == TWO32 and not exact.fixed_point_params(1.0)["flip"]
    assert exact.fixed_point_params(2.0)["P"] == 0
    assert exact.fixed_point_params(0.5)["P"] == 1 << 31
    assert exact.fixed_point_params(1.5)["P"] == 1 << 31
    assert exact.fixed_point_params(1.0, flip="on")["P"] == TWO32
    assert exact.fixed_point_params(1.8)["P_rest"] == 2863311531
    with pytest.raises(ValueError):
        exact.fixed_point_params(2.5)
    with pytest.raises(ValueError):
        exact.fixed_point_params(0.5, flip="on")


def test_half_table_is_textbook():
    tab = exact.binomial_table(1 << 31)
    for m in range(1, 65):
        row = exact.table_row(tab, m)
        acc = 0
        for j in range(m):
            acc += math.comb(m, j)
            # floor(2^32 * acc / 2^m)
            assert int(row[j]) == (acc << 32) >> m


@pytest.mark.parametrize("P", [1, 85899346, 858993459, 2863311531, TWO32 - 1])
def test_table_matches_direct_definition(P):
    tab = exact.binomial_table(P)
    for m in [1, 2, 3, 7, 31, 64]:
        row = exact.table_row(tab, m)
        for j in range(m):
            assert int(row[j]) == _cdf_floor_direct(m, P, j), (m, j)


@pytest.mark.parametrize("P", P_VALUES)
def test_table_shape_and_bounds(P):
    tab = exact.binomial_table(P)
    assert tab.shape == (2080,)
    for m in range(1, 65):
        row = exact.table_row(tab, m).astype(np.int64)
        assert np.all(np.diff(row) >= 0)
        # quantized pmf within 2^-32 of the exact pmf for every outcome
        qp = exact.quantized_chunk_pmf(tab, m)
        ip = exact.ideal_binomial_pmf(m, Fraction(P, TWO32))
        assert max(abs(a - b) for a, b in zip(qp, ip)) < Fraction(1, TWO32)
    if P == TWO32:
        assert not tab.any()   # p = 1: every particle collides


def test_zero_probability_table():
    assert exact.binomial_table(0) is None


@pytest.mark.parametrize("n", [1, 5, 63, 64, 65, 130, 200])
@pytest.mark.parametrize("P", [858993459, 1 << 31])
def test_binomial_sampler_law(oracle_lib, n, P):
    tab = exact.binomial_table(P)
    N = 100000
    x = oracle_lib.binomial_samples(n, tab, N, seed=11 + n)
    pmf = np.array([float(v) for v in exact.quantized_binomial_pmf(n, tab)])
    counts = np.bincount(x.astype(np.int64), minlength=n + 1)
    exp = pmf * N
    keep = exp >= 5
    chi2 = (((counts - exp) ** 2)[keep] / exp[keep]).sum() + 0.0
    dof = max(int(keep.sum()) - 1, 1)
    assert stats.chi2.sf(chi2, dof) > 1e-4
    assert counts[~keep].sum() <= 5 * max(exp[~keep].sum(), 1.0) + 10
    # mean against the exact binomial mean n p
    assert abs(x.mean() - n * P / TWO32) < 5 * math.sqrt(n * 0.25 / N) + 1e-9


def test_binomial_extremes(oracle_lib):
    assert not oracle_lib.binomial_samples(100, None, 1000, seed=1).any()
    full = exact.binomial_table(TWO32)
    assert np.all(oracle_lib.binomial_samples(137, full, 1000, seed=1) == 137)


def _inputs(q, total_max):
    for a in itertools.product(range(total_max + 1), repeat=q):
        if 0 < sum(a) <= total_max:
            yield a


@pytest.mark.parametrize("q", [2, 3])
@pytest.mark.parametrize("omega,flip", [(1.5, "auto"), (1.8, "auto"), (1.98, "auto"),
                                        (1.0, "on"), (0.7, "auto")])
def test_collision_law_exact_enumeration(oracle_lib, q, omega, flip):
    """Histograms of the oracle's collision for every input with sum <= 6 (q=2)
    or <= 5 (q=3) against the exact independent-particle law."""
    params = oracle_lib.Params(q, omega, flip=flip)
    total_max = 6 if q == 2 else 5
    N = 20000
    worst = 1.0
    for a in _inputs(q, total_max):
        law = exact.collision_law_particles(a, q, params.P, params.P_rest, params.flip)
        # the fixed-point sampler's own exact law is within quantization of it
        slaw = exact.collision_law_sampler(a, q, params.tab_p, params.tab_half, params.tab_rest,
                                           params.flip)
        tv = sum(abs(law.get(k, 0) - slaw.get(k, 0)) for k in set(law) | set(slaw)) / 2
        assert tv < Fraction(1, 1 << 24)
        samples = oracle_lib.collide_samples(params, a, N, seed=hash(a) & 0xFFFF, t=3)
        assert np.all(samples.sum(axis=1) == sum(a))  # mass conserved
        keys = [tuple(int(v) for v in s) for s in samples]
        hist = {}
        for k in keys:
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
    # about 100 inputs per case: a family-wise threshold
    assert worst > 1e-5


def test_flip_moot_at_full_collision(oracle_lib):
    """omega* = 1: all particles collide, so flip on and flip off give
    identical samples (Over-relaxation section: the flip becomes moot)."""
    on = oracle_lib.Params(3, 1.0, flip="on")
    off = oracle_lib.Params(3, 1.0, flip="off")
    for a in [(3, 0, 1), (10, 20, 30), (0, 7, 0)]:
        s1 = oracle_lib.collide_samples(on, a, 2000, seed=5)
        s2 = oracle_lib.collide_samples(off, a, 2000, seed=5)
        np.testing.assert_array_equal(s1, s2)
