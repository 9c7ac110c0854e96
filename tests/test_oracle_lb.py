"""Pins of the FP64 lattice Boltzmann limit and the paper's closed forms
(Boltzmann-approximation section)."""
import math

import numpy as np
import pytest

from oracle import exact

CASES = [(2, 0.7, False), (2, 0.5, True), (3, 0.2, True), (3, 0.9, False), (3, 0.02, True),
         (3, 1.0, True)]


@pytest.mark.parametrize("theta", [1.0 / 3.0, 0.25, 0.6])
def test_moment_matrix_orthonormal(theta):
    """sum_i m_i^a w_i m_i^b = delta^ab and sum_a m_i^a w_j m_j^a = delta_ij."""
    m = exact.moment_matrix(3, theta)
    w = exact.weights(3, theta)
    np.testing.assert_allclose(m @ np.diag(w) @ m.T, np.eye(3), atol=1e-14)
    np.testing.assert_allclose((m.T @ m) * w[None, :], np.eye(3), atol=1e-14)
    assert exact.theta_of(3, theta) == pytest.approx(theta)


def test_equilibrium_and_flip_in_moment_space():
    """Equilibrium moments are (rho, 0, 0) (Eq. momentspacef0); the flip maps
    (rho, j, Pi) to (rho, -j, Pi) (Eq. momentspaceFm)."""
    rng = np.random.default_rng(0)
    m = exact.moment_matrix(3)
    f = rng.uniform(0, 10, size=(3, 5))
    feq = exact.lb_equilibrium(f, 3, 1.0 / 3.0)
    M0 = m @ feq
    np.testing.assert_allclose(M0[0], f.sum(axis=0))
    np.testing.assert_allclose(M0[1:], 0.0, atol=1e-12)
    Mf = m @ f[::-1]
    Mo = m @ f
    np.testing.assert_allclose(Mf, Mo * np.array([1, -1, 1])[:, None], atol=1e-12)


@pytest.mark.parametrize("q,omega_star,flip", CASES)
def test_flip_lb_equals_mrt(q, omega_star, flip):
    """The Boltzmann average with flip equals the MRT scheme with
    omega^j = 2 - omega* and omega^Pi = omega* (Eqs. omegaj, MRTLB)."""
    rng = np.random.default_rng(1)
    f = rng.uniform(0, 5, size=(q, 17))
    a = exact.lb_step_flip(f, q, omega_star, flip)
    b = exact.mrt_step(f, q, omega_star, flip)
    np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-12)


@pytest.mark.parametrize("q,omega_star,flip", CASES)
def test_lb_conserves_mass(q, omega_star, flip):
    f = np.random.default_rng(2).uniform(0, 5, size=(q, 11))
    g = exact.lb_step_flip(f, q, omega_star, flip)
    assert g.sum() == pytest.approx(f.sum(), rel=1e-14)


def test_lb_full_over_relaxation_period_two():
    f = np.random.default_rng(3).uniform(0, 5, size=(3, 13))
    g = exact.lb_step_flip(exact.lb_step_flip(f, 3, 0.0, True), 3, 0.0, True)
    np.testing.assert_array_equal(g, f)


@pytest.mark.parametrize("q", [2, 3])
@pytest.mark.parametrize("omega_j", [0.6, 1.0, 1.25, 1.5, 1.75, 1.9, 1.98])
@pytest.mark.parametrize("L", [256, 320, 4096])
def test_lb_mode_decay_matches_diffusion_constant(q, omega_j, L):
    """The slow eigenvalue of mode k = 2 pi/L decays at D k^2 with
    D = theta (1/omega^j - 1/2); the diffusion equation is the leading order in
    k, so the relative deviation is O(k^2) (coefficient below 1.3 for these
    rates)."""
    flip = omega_j > 1.0
    omega_star = 2.0 - omega_j if flip else omega_j
    th = exact.theta_of(q)
    D = exact.diffusion_constant(omega_j, th)
    rate = exact.lb_slow_rate(q, L, omega_star, flip)
    k = 2.0 * math.pi / L
    assert abs(rate / D - 1.0) < 1.5 * k * k


def test_lb_sine_amplitude_follows_eigenvalue():
    """A sine density evolved by the LB keeps its shape to first order and its
    A^LG amplitude decays like the theory line of Eq. ampdecay."""
    q, L, omega_j = 3, 320, 1.5
    x = np.arange(L)
    rho = 100.0 * (1 + np.sin(2 * math.pi * x / L))
    f0 = exact.weights(q)[:, None] * rho[None, :]
    T = 4000
    f = exact.lb_run(f0, q, 2.0 - omega_j, True, T)
    A = exact.amplitude_lg(f.sum(axis=0))
    D = exact.diffusion_constant(omega_j, exact.theta_of(q))
    assert A == pytest.approx(float(exact.amplitude_theory(T, 100.0, D, L)), rel=2e-3)


def test_amplitude_and_structure_factor_definitions():
    L = 64
    x = np.arange(L)
    N = 30.0 + 7.5 * np.sin(2 * math.pi * x / L)
    assert exact.amplitude_lg(N) == pytest.approx(7.5, rel=1e-12)
    rng = np.random.default_rng(4)
    n = rng.poisson(20, size=L).astype(np.float64)
    S = exact.structure_factor(n, 5)
    ft = np.fft.fft(n)
    np.testing.assert_allclose(S, np.abs(ft[1:6]) ** 2 / n.sum(), rtol=1e-10)


def test_diffusion_constant_closed_form():
    assert exact.diffusion_constant(1.0, 1.0 / 3.0) == pytest.approx(1.0 / 6.0)
    assert exact.diffusion_constant(2.0, 1.0 / 3.0) == 0.0
    assert exact.theta_of(2) == 1.0
