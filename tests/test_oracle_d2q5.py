"""Pins of the D2Q5 extension of the oracle (the paper's flip, Eq. flip, on
a two-dimensional five-velocity set; the paper states the general rule that
odd moments change sign and even moments do not).

* The FP64 Boltzmann iteration with flip relaxes a density wave at the rate
  D |k|^2 with D = theta (1/omega^j - 1/2) along x, y and the diagonal
  (isotropy), the same law as the paper's 1D result.
* One collision of the integer oracle has the law of independent particles:
  each stays with probability 1 - omega* or moves to velocity j with
  probability omega* w_j (enumerated exactly; chi-square on samples).
* The lattice mean follows the Boltzmann iteration (z-tests over
  realizations); omega^j = 2 is a pure permutation of period two; mass is
  conserved and the hash is the one of the state."""
import itertools
import math

import numpy as np
import pytest
from scipy import stats

from oracle import exact
from oracle import oracle as O

TH = 1.0 / 3.0


@pytest.mark.parametrize("omega", [0.4, 1.0, 1.3, 1.7, 1.95])
@pytest.mark.parametrize("direction", [(1, 0), (0, 1), (1, 1)])
def test_boltzmann_diffusion_rate(omega, direction):
    fp = exact.fixed_point_params(omega, TH, "auto", q=5)
    D = exact.diffusion_constant(omega, exact.theta_of(5, TH))
    for k in (2 * math.pi / 128, 2 * math.pi / 512):
        kx, ky = k * direction[0], k * direction[1]
        k2 = kx * kx + ky * ky
        rate = exact.lb_slow_rate_2d(kx, ky, fp["omega_star"], fp["flip"], TH)
        assert abs(rate / k2 - D) <= 1.5 * k2 + 1e-12


def test_boltzmann_isotropy_and_mass():
    fp = exact.fixed_point_params(1.6, TH, "auto", q=5)
    for k in (0.05, 0.3):
        a = exact.lb_slow_rate_2d(k, 0.0, fp["omega_star"], fp["flip"], TH)
        b = exact.lb_slow_rate_2d(0.0, k, fp["omega_star"], fp["flip"], TH)
        assert abs(a - b) < 1e-13
    rng = np.random.default_rng(3)
    f = rng.random((5, 6, 7))
    g = exact.lb_step_flip_2d(f, fp["omega_star"], fp["flip"], TH)
    assert abs(g.sum() - f.sum()) < 1e-12


def _ideal_collision_law(a, omega_star, flip, P_rest):
    """Exact law of the post-collision counts: flip, then every particle
    independently stays (1 - p) or goes to j with probability p w_j, with
    p = P / 2^32 and the rest weight P_rest / 2^32 (the fixed-point values
    the sampler uses)."""
    p = omega_star
    w_rest = P_rest / 2.0 ** 32
    w_move = (1.0 - w_rest) / 4.0
    w = np.array([w_move, w_move, w_rest, w_move, w_move])
    if flip:
        a = a[::-1]
    law = {tuple([0] * 5): 1.0}
    for i, ai in enumerate(a):
        for _ in range(int(ai)):
            nxt = {}
            for key, pr in law.items():
                for j in range(5):
                    pj = (1 - p) * (1.0 if j == i else 0.0) + p * w[j]
                    if pj == 0.0:
                        continue
                    kk = list(key)
                    kk[j] += 1
                    kk = tuple(kk)
                    nxt[kk] = nxt.get(kk, 0.0) + pr * pj
            law = nxt
    return law


@pytest.mark.parametrize("omega,a", [(0.7, (2, 1, 3, 0, 2)), (1.45, (3, 0, 1, 2, 1)),
                                      (1.0, (1, 2, 0, 1, 3))])
def test_single_collision_law(omega, a):
    prm = O.Params(5, omega, TH)
    n = 200_000
    out = O.collide_samples(prm, np.array(a, dtype=np.uint64), n, seed=101)
    law = _ideal_collision_law(np.array(a), prm.P / 2.0 ** 32, prm.flip, prm.P_rest)
    keys = list(law)
    idx = {k: i for i, k in enumerate(keys)}
    obs = np.zeros(len(keys))
    for row in map(tuple, out.astype(np.int64)):
        obs[idx[row]] += 1          # a KeyError would be an impossible outcome
    exp = np.array([law[k] for k in keys]) * n
    big = exp >= 5
    o = np.append(obs[big], obs[~big].sum())
    e = np.append(exp[big], exp[~big].sum())
    if e[-1] < 5:
        o, e = o[:-1], e[:-1]
    pval = stats.chisquare(o, e * o.sum() / e.sum()).pvalue
    assert pval > 1e-4
    assert (out.sum(axis=1) == sum(a)).all()


def test_lattice_mean_follows_boltzmann():
    lx, ly, R, T, om = 6, 5, 3000, 6, 1.35
    prm = O.Params(5, om, TH)
    rng = np.random.default_rng(11)
    base = rng.integers(5, 40, size=(5, ly, lx)).astype(np.uint16)
    acc = np.zeros((5, ly, lx))
    acc2 = np.zeros((5, ly, lx))
    for r in range(R):
        s, _, ov = O.run2d(prm, base, T, seed=7, realization=r, nthreads=1)
        assert not ov
        acc += s
        acc2 += s.astype(np.float64) ** 2
    mean = acc / R
    var = acc2 / R - mean ** 2
    f = base.astype(np.float64)
    for _ in range(T):
        f = exact.lb_step_flip_2d(f, prm.P / 2.0 ** 32, prm.flip, TH)
    z = (mean - f) / np.sqrt(np.maximum(var, 1e-9) / R)
    assert np.abs(z).max() < 5.0


def test_omega_two_is_a_period_two_permutation():
    prm = O.Params(5, 2.0, TH)
    rng = np.random.default_rng(5)
    s0 = rng.integers(0, 50, size=(5, 4, 7)).astype(np.uint32)
    s1, _, _ = O.run2d(prm, s0, 1, seed=1)
    # one step: out_i(x + v_i) = n_{4-i}(x)
    want = np.empty_like(s0)
    for i, (vx, vy) in enumerate(exact.velocities(5)):
        want[i] = np.roll(np.roll(s0[4 - i], int(vx), axis=1), int(vy), axis=0)
    np.testing.assert_array_equal(s1, want)
    s2, _, _ = O.run2d(prm, s0, 2, seed=1)
    np.testing.assert_array_equal(s2, s0)


def test_mass_and_hash():
    prm = O.Params(5, 1.2, TH)
    rng = np.random.default_rng(8)
    s0 = rng.poisson(30, size=(5, 9, 11)).astype(np.uint16)
    s, hs, ov = O.run2d(prm, s0, 4, seed=2, hashes=True)
    assert not ov and int(s.astype(np.int64).sum()) == int(s0.astype(np.int64).sum())
    assert int(hs[-1]) == O.state_hash(s)
    # the node index is x + Lx y: a transposed lattice is a different state
    assert O.state_hash(s) != O.state_hash(np.ascontiguousarray(s.transpose(0, 2, 1)))
