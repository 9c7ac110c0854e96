"""Statistical pins of the oracle's lattice gas against its Boltzmann limit.

f_i = <n_i> (Integer Lattice Gas section) evolves by the lattice Boltzmann
equation with the flip (Boltzmann-approximation section).  Under the
independent-particle reading of the sampling collision this holds exactly in
expectation, so ensembles of the oracle are compared with FP64 LB runs by
z-scores; the decay of a sine mode is compared with D = theta(1/omega^j - 1/2)
(Eq. ampdecay).  All seeds are fixed, so these tests are deterministic.
"""
import math
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
from scipy import stats

import ilg_workloads as W
from oracle import exact


def _pool():
    return ThreadPoolExecutor(max_workers=8)


@pytest.mark.parametrize("q,omega", [(3, 1.6), (2, 1.3), (3, 0.8)])
def test_single_particle_propagator(oracle_lib, q, omega):
    """One particle on a ring of 16 nodes is a Markov chain whose transition
    matrix is the LB operator; its position histogram after t steps equals the
    matrix power applied to the start state."""
    L, T, R = 16, 9, 40000
    p = oracle_lib.Params(q, omega)
    st = np.zeros((q, L), dtype=np.uint32)
    st[0, 5] = 1
    A = exact.lb_operator(q, L, p.omega_star, p.flip)
    prob = np.linalg.matrix_power(A, T) @ st.reshape(-1).astype(np.float64)

    def one(r):
        out, _, _ = oracle_lib.run(p, st, T, seed=77, realization=r, nthreads=1)
        return int(np.flatnonzero(out.reshape(-1))[0])

    with _pool() as ex:
        where = list(ex.map(one, range(R)))
    hist = np.bincount(where, minlength=q * L).astype(np.float64)
    exp = prob * R
    keep = exp >= 5
    chi2 = ((hist[keep] - exp[keep]) ** 2 / exp[keep]).sum()
    assert stats.chi2.sf(chi2, int(keep.sum()) - 1) > 1e-4
    assert hist[~keep].sum() <= 3 * exp[~keep].sum() + 10


@pytest.mark.parametrize("q,omega", [(3, 1.6), (3, 1.95), (2, 1.4), (3, 0.7)])
def test_poisson_closure_against_lb(oracle_lib, q, omega):
    """Poisson initial occupations stay Poisson with the LB mean f_i(x, t):
    ensemble mean and variance per (i, x) against the FP64 run."""
    L, T, R = 24, 12, 3000
    w = W.D1Q3_WEIGHTS if q == 3 else W.D1Q2_WEIGHTS
    p = oracle_lib.Params(q, omega)
    x = np.arange(L)
    rho0 = 60.0 * (1 + 0.8 * np.sin(2 * math.pi * x / L))
    f = exact.weights(q)[:, None] * rho0[None, :]
    fT = exact.lb_run(f, q, p.omega_star, p.flip, T)

    def one(r):
        init = W.init_poisson_sine(w, L, 60.0, 48.0, 4, init_seed=1000 + r)
        out, _, _ = oracle_lib.run(p, init, T, seed=31, realization=r, nthreads=1)
        return out.astype(np.float64)

    with _pool() as ex:
        outs = np.stack(list(ex.map(one, range(R))))
    mean = outs.mean(axis=0)
    var = outs.var(axis=0, ddof=1)
    z = (mean - fT) / np.sqrt(fT / R)
    n = z.size
    assert np.abs(z).max() < 4.5
    assert stats.chi2.sf((z ** 2).sum(), n) > 1e-4
    # Poisson: variance equals the mean; sd of the sample variance ~ f sqrt(2/R)
    zv = (var - fT) / (np.sqrt(2.0 / R) * fT + np.sqrt(fT / R))
    assert np.abs(zv).max() < 5.0


def test_equilibrium_structure_factor(oracle_lib):
    """At equilibrium the occupations are independent Poisson, so S(k) = 1 for
    k != 0 (S normalised by the total mass)."""
    q, L, R = 3, 256, 48
    p = oracle_lib.Params(q, 1.7)

    def one(r):
        init = W.init_poisson_iid(q, L, 40.0, 2, init_seed=500 + r)
        out, _, _ = oracle_lib.run(p, init, 400, seed=5, realization=r, nthreads=1)
        return exact.structure_factor(out.astype(np.int64).sum(axis=0), 16)

    with _pool() as ex:
        S = np.stack(list(ex.map(one, range(R))))
    # each S(k) is ~ Exp(1): mean over R*16 samples has sd 1/sqrt(768)
    assert abs(S.mean() - 1.0) < 4.0 / math.sqrt(S.size)


def _decay_sigma(nave, L, R, D, T, A0):
    """1-sigma relative error of gamma = -ln(sum A(T) / sum A(0)) / T:
    the amplitude noise around its conditional mean has variance
    Var_eq (1 - exp(-2 gamma T)) with Var_eq = 2 nave / L."""
    g = 4 * math.pi ** 2 * D / L ** 2
    var_eq = 2.0 * nave / L
    return math.sqrt(var_eq * (1 - math.exp(-2 * g * T)) / R) / (A0 * math.exp(-g * T) * g * T)


@pytest.mark.parametrize("omega_j", [0.8, 1.5])
def test_decay_rate_matches_diffusion_constant(oracle_lib, omega_j):
    """Sine-mode decay (Results section): D1Q3, L = 320, N^ave = 100, Poisson
    initialisation; the fitted rate matches 4 pi^2 D / L^2 within 4 sigma of
    its statistical error (reduced ensemble; the full ensemble runs on the GPU)."""
    q, L, R, T, nave = 3, 320, 256, 2000, 100.0
    p = oracle_lib.Params(q, omega_j)
    D = exact.diffusion_constant(omega_j, exact.theta_of(q))

    def one(r):
        init = W.init_poisson_sine(W.D1Q3_WEIGHTS, L, nave, nave, 4, init_seed=2000 + r)
        a0 = exact.amplitude_lg(init.astype(np.int64).sum(axis=0))
        out, _, _ = oracle_lib.run(p, init, T, seed=4242, realization=r, nthreads=1)
        return a0, exact.amplitude_lg(out.astype(np.int64).sum(axis=0))

    with _pool() as ex:
        res = np.array(list(ex.map(one, range(R))))
    gamma = -math.log(res[:, 1].sum() / res[:, 0].sum()) / T
    g_th = 4 * math.pi ** 2 * D / L ** 2
    sig = _decay_sigma(nave, L, R, D, T, nave)
    assert abs(gamma / g_th - 1.0) < 4 * sig + 1e-3
