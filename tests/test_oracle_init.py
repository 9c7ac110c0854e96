"""Pins of the oracle's Poisson sine initial state (init v1): the paper draws
each occupation as a Poisson variate with expectation w_i times the sine
density profile (Results section).  The oracle is checked against the
mathematics, not against itself: the sine and exponential it builds from
correctly rounded operations against the library functions and their exact
values, the counts against the Poisson distribution (chi-square on the exact
pmf), the per-node means against the sine profile, and the edge cases
(empty profile, zero density at the trough, overflow, windows)."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O


def test_sine_exact_points():
    for L in (8, 320, 1 << 20, 999_992):
        assert O.sin2pi_frac(0, L) == 0.0
        assert O.sin2pi_frac(L // 4, L) == 1.0
        assert O.sin2pi_frac(L // 2, L) == 0.0
        assert O.sin2pi_frac(3 * L // 4, L) == -1.0
        assert abs(O.sin2pi_frac(L // 8, L) - math.sqrt(0.5)) <= 2.3e-16


@pytest.mark.parametrize("L", [1, 2, 3, 7, 320, 1000, 4099, 1 << 24])
def test_sine_against_library(L):
    rng = np.random.default_rng(L)
    xs = range(L) if L <= 5000 else rng.integers(0, L, 20000)
    err = max(abs(O.sin2pi_frac(int(x), L) - math.sin(2.0 * math.pi * int(x) / L)) for x in xs)
    assert err <= 2e-15


def test_sine_symmetries_exact():
    """sin(2 pi (L - x) / L) = -sin(2 pi x / L) and sin(2 pi (L/2 - x) / L) =
    sin(2 pi x / L) hold exactly in the octant construction, except at odd
    multiples of pi/4, where one side evaluates the sine polynomial and the
    other the cosine polynomial at pi/4 (equal to one ulp)."""
    L = 4096
    for x in range(1, L // 2):
        a, b, c = O.sin2pi_frac(x, L), O.sin2pi_frac(L - x, L), O.sin2pi_frac(L // 2 - x, L)
        if (8 * x) % L == 0 and (8 * x // L) % 2 == 1:
            assert abs(a + b) <= 2.3e-16 and abs(a - c) <= 2.3e-16
        else:
            assert b == -a and c == a


def test_exp_against_library():
    ms = np.concatenate([np.linspace(0.0, 256.0, 20001), [1e-12, 0.5, math.log(2), 255.9999]])
    rel = max(abs(O.exp_neg(float(m)) / math.exp(-float(m)) - 1.0) for m in ms)
    assert rel <= 4.5e-16
    assert O.exp_neg(0.0) == 1.0
    vals = [O.exp_neg(float(m)) for m in np.linspace(0.0, 256.0, 5001)]
    assert all(a > b for a, b in zip(vals, vals[1:]))


def _chi2_poisson(samples, mu):
    """Chi-square p-value of integer samples against Poisson(mu), bins with
    expected count >= 5 (tails pooled)."""
    n = samples.size
    kmax = int(samples.max())
    k = np.arange(kmax + 1)
    pmf = stats.poisson.pmf(k, mu)
    obs = np.bincount(samples, minlength=kmax + 1).astype(float)
    exp = pmf * n
    # pool from both ends until every bin expects >= 5
    lo = 0
    while exp[: lo + 1].sum() < 5:
        lo += 1
    hi = kmax
    while exp[hi:].sum() < 5:
        hi -= 1
    o = np.concatenate([[obs[: lo + 1].sum()], obs[lo + 1: hi], [obs[hi:].sum()]])
    e = np.concatenate([[stats.poisson.cdf(lo, mu) * n], exp[lo + 1: hi],
                        [stats.poisson.sf(hi - 1, mu) * n]])
    chi2 = ((o - e) ** 2 / e).sum()
    return stats.chi2.sf(chi2, len(o) - 1)


@pytest.mark.parametrize("mu", [0.7, 4.5, 30.0, 100.0, 255.0, 300.0, 900.0])
def test_counts_are_poisson(mu):
    """Constant profile (amp = 0), D1Q2 weights 1/2: every count is
    Poisson(mu); means above 256 are split into parts (300 -> 2, 900 -> 4)."""
    L = 120_000
    out, ov = O.init_poisson_sine(2, 4, L, 2.0 * mu, 0.0, seed=77 + int(mu))
    assert not ov
    s = out.reshape(-1).astype(np.int64)
    assert _chi2_poisson(s, mu) > 1e-4
    z_mean = (s.mean() - mu) / math.sqrt(mu / s.size)
    assert abs(z_mean) < 4.5
    # variance of a Poisson sample variance: (mu + 2 mu^2) / n approximately
    z_var = (s.var(ddof=1) - mu) / math.sqrt((mu + 2 * mu * mu) / s.size)
    assert abs(z_var) < 4.5


def test_sine_profile_means():
    """Per-node means over realizations follow w_i (N + A sin(2 pi x / L)),
    weights (theta/2, 1 - theta, theta/2)."""
    q, L, N, A, R = 3, 40, 60.0, 45.0, 3000
    acc = np.zeros((q, L))
    for r in range(R):
        out, _ = O.init_poisson_sine(q, 2, L, N, A, seed=5, realization=r)
        acc += out
    mean = acc / R
    x = np.arange(L)
    w = np.array([1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0])
    expect = np.outer(w, N + A * np.sin(2 * np.pi * x / L))
    z = (mean - expect) / np.sqrt(np.maximum(expect, 1e-9) / R)
    assert np.abs(z).max() < 4.5


def test_velocities_and_realizations_independent():
    L = 200_000
    a, _ = O.init_poisson_sine(3, 2, L, 90.0, 0.0, seed=9, realization=0)
    b, _ = O.init_poisson_sine(3, 2, L, 90.0, 0.0, seed=9, realization=1)
    lim = 4.5 / math.sqrt(L)
    assert abs(np.corrcoef(a[0], a[2])[0, 1]) < lim
    assert abs(np.corrcoef(a[0], a[1])[0, 1]) < lim
    assert abs(np.corrcoef(a[1], b[1])[0, 1]) < lim


def test_edge_cases():
    z, ov = O.init_poisson_sine(3, 2, 1000, 0.0, 0.0, seed=1)
    assert not ov and not z.any()
    # amp = nave: density exactly zero at x = 3L/4, so every count there is 0
    L = 400
    t, _ = O.init_poisson_sine(3, 2, L, 80.0, 80.0, seed=2)
    assert not t[:, 3 * L // 4].any()
    assert t[:, L // 4].sum() > 0
    # uint16 overflow is flagged: mean 1e5 per velocity
    _, ov = O.init_poisson_sine(2, 2, 64, 2.0e5, 0.0, seed=3)
    assert ov
    _, ov = O.init_poisson_sine(2, 4, 64, 2.0e5, 0.0, seed=3)
    assert not ov


def test_windows_match_full_state():
    L = 1009
    full, _ = O.init_poisson_sine(3, 4, L, 70.0, 30.0, seed=4, realization=2)
    for x0, width in [(0, 17), (500, 509), (1000, 30), (3, 1009)]:
        win, _ = O.init_poisson_sine(3, 4, L, 70.0, 30.0, seed=4, realization=2, x0=x0,
                                     width=width)
        idx = (x0 + np.arange(width)) % L
        np.testing.assert_array_equal(win, full[:, idx])


def test_seed_changes_draws():
    a, _ = O.init_poisson_sine(2, 2, 5000, 40.0, 10.0, seed=1)
    b, _ = O.init_poisson_sine(2, 2, 5000, 40.0, 10.0, seed=2)
    assert (a != b).mean() > 0.8


def test_d2q5_profile_and_weights():
    """D2Q5: means w_i (N + A sin(2 pi x / Lx)) with weights (theta/2, theta/2,
    1 - 2 theta, theta/2, theta/2), constant along y; the fifth velocity takes
    its word from a second Philox block and is independent of the first."""
    lx, ly, N, A, R = 16, 3, 60.0, 40.0, 2500
    acc = np.zeros((5, ly, lx))
    for r in range(R):
        out, _ = O.init_poisson_sine(5, 2, lx, N, A, seed=13, realization=r, height=ly)
        acc += out
    mean = acc / R
    w = np.array([1 / 6, 1 / 6, 1 / 3, 1 / 6, 1 / 6])
    prof = N + A * np.sin(2 * np.pi * np.arange(lx) / lx)
    expect = w[:, None, None] * prof[None, None, :] * np.ones((1, ly, 1))
    z = (mean - expect) / np.sqrt(expect / R)
    assert np.abs(z).max() < 4.5
    big, _ = O.init_poisson_sine(5, 2, 400, 90.0, 0.0, seed=2, height=500)
    flat = big.reshape(5, -1).astype(np.float64)
    assert abs(np.corrcoef(flat[0], flat[4])[0, 1]) < 4.5 / math.sqrt(flat.shape[1])
