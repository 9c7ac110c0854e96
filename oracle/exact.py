"""Exact and FP64 reference tools for the diffusive integer lattice gas.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product package.

Contents, each tied to the paper (Strand & Wagner, "Over-Relaxation in
Diffusive Integer Lattice Gas"):
  * fixed-point collision parameters from the relaxation rate (Over-relaxation
    section: omega* in [0,1] after the flip; Boltzmann-approximation section,
    Eq. omegaj: omega^j = 2 - omega*);
  * exact fixed-point binomial CDF tables with Python big integers;
  * exact post-collision laws in rational arithmetic (the sampling collision of
    the Integer Lattice Gas section read as independent particles);
  * the FP64 lattice Boltzmann limit with the flip (Boltzmann-approximation
    section, first equation) and its MRT moment-space form (Eqs. transform,
    momentspaceFm, momentspaceOm, MRTLB);
  * closed forms: theta (Eq. Thetadef), D (the diffusion constant after
    Eq. diffusioneqn), the amplitude decay (Eq. ampdecay), the measured
    amplitude A^LG (Results section).
"""
from __future__ import annotations

import math
from fractions import Fraction
from typing import Dict, List, Optional, Sequence

import numpy as np

TWO32 = 1 << 32
CHUNK = 64
TABLE_ENTRIES = CHUNK * (CHUNK + 1) // 2  # rows m = 1..64, m entries each


# --------------------------------------------------------------- parameters

def velocities(q: int) -> np.ndarray:
    """Index order of the velocity sets: D1Q2 (-1, +1), D1Q3 (-1, 0, +1);
    D2Q5 as rows (vx, vy): (-1,0), (0,-1), (0,0), (0,+1), (+1,0), so that the
    mirror -v_i of index i is index q-1-i in every set."""
    if q == 2:
        return np.array([-1, 1], dtype=np.int64)
    if q == 3:
        return np.array([-1, 0, 1], dtype=np.int64)
    if q == 5:
        return np.array([[-1, 0], [0, -1], [0, 0], [0, 1], [1, 0]], dtype=np.int64)
    raise ValueError("q must be 2, 3 or 5")


def weights(q: int, theta: float = 1.0 / 3.0) -> np.ndarray:
    """Lattice weights: D1Q2 (1/2, 1/2); D1Q3 (theta/2, 1-theta, theta/2).

    The D1Q3 form is the one for which the transformation matrix of
    Eq. transform is orthonormal in the Hermite norm for any theta."""
    if q == 2:
        return np.array([0.5, 0.5])
    if q == 5:
        # D2Q5 (reading: the paper works the flip out in 1D; the 2D set takes
        # the same isotropic second moment theta = sum_i w_i v_ix^2 = sum_i w_i v_iy^2)
        return np.array([theta / 2.0, theta / 2.0, 1.0 - 2.0 * theta, theta / 2.0, theta / 2.0])
    return np.array([theta / 2.0, 1.0 - theta, theta / 2.0])


def theta_of(q: int, theta: float = 1.0 / 3.0) -> float:
    """theta = sum_i w_i v_i^2 (Eq. Thetadef); for D2Q5 the x component."""
    v = velocities(q)
    if v.ndim == 2:
        v = v[:, 0]
    return float(np.sum(weights(q, theta) * v ** 2))


def fixed_point_params(omega: float, theta: float = 1.0 / 3.0, flip: str = "auto",
                       q: int = 3) -> Dict:
    """Collision parameters for a target relaxation rate omega (= omega^j).

    flip == "auto": the flip is applied iff omega > 1 (over-relaxation); then
    the collision fraction is omega* = 2 - omega (Eq. omegaj), otherwise
    omega* = omega (plain Seekins collision, omega <= 1).  "on"/"off" force it.
    P = round-half-even(omega* 2^32), the removal probability in 32-bit fixed
    point; P_half = 2^31; P_rest = round-half-even(w_rest 2^32), the rest
    weight: 1 - theta (D1Q3) or 1 - 2 theta (D2Q5, theta < 1/2)."""
    if not (0.0 < omega <= 2.0):
        raise ValueError("omega must lie in (0, 2]")
    if flip == "auto":
        do_flip = omega > 1.0
    elif flip == "on":
        if omega < 1.0:
            raise ValueError("a forced flip needs omega >= 1")
        do_flip = True
    elif flip == "off":
        if omega > 1.0:
            raise ValueError("omega > 1 needs the flip")
        do_flip = False
    else:
        raise ValueError("flip must be auto, on or off")
    omega_star = (2.0 - omega) if do_flip else omega
    P = round(omega_star * float(TWO32))   # Python rounds floats half-to-even
    if q == 5:
        if not (0.0 < theta < 0.5):
            raise ValueError("D2Q5 theta must lie in (0, 1/2)")
        P_rest = round((1.0 - 2.0 * theta) * float(TWO32))
    else:
        if not (0.0 < theta < 1.0):
            raise ValueError("theta must lie in (0, 1)")
        P_rest = round((1.0 - theta) * float(TWO32))
    # D1Q2 exchange form: crossing probability omega*/2, i.e.
    # round-half-even(omega* 2^31) in the same fixed point.
    P_x = round(omega_star * float(1 << 31))
    return dict(flip=do_flip, omega_star=omega_star, P=int(P), P_half=1 << 31, P_rest=int(P_rest),
                P_x=int(P_x))


# ------------------------------------------------------ fixed-point tables

def scaled_binomial_pmf(n: int, P: int) -> List[int]:
    """C(n,i) P^i (2^32-P)^(n-i) for i = 0..n, as exact integers (sum 2^(32n)),
    built by n convolutions with (2^32-P, P): the law of n independent trials."""
    pmf = [1]
    for _ in range(n):
        nxt = [0] * (len(pmf) + 1)
        for i, v in enumerate(pmf):
            nxt[i] += v * (TWO32 - P)
            nxt[i + 1] += v * P
        pmf = nxt
    return pmf


def binomial_table(P: int) -> Optional[np.ndarray]:
    """T_P[m][j] = floor(2^32 CDF_{m,P/2^32}(j)) for m = 1..64, j = 0..m-1,
    flattened with row m starting at (m-1)m/2.  P = 0 returns None (the
    sampler then returns 0)."""
    if not (0 <= P <= TWO32):
        raise ValueError("P out of range")
    if P == 0:
        return None
    out = np.zeros(TABLE_ENTRIES, dtype=np.uint32)
    for m in range(1, CHUNK + 1):
        pmf = scaled_binomial_pmf(m, P)
        acc = 0
        base = (m - 1) * m // 2
        for j in range(m):
            acc += pmf[j]
            val = acc >> (32 * (m - 1))
            assert val < TWO32
            out[base + j] = val
    return out


def table_row(table: np.ndarray, m: int) -> np.ndarray:
    base = (m - 1) * m // 2
    return table[base:base + m]


def quantized_chunk_pmf(table: Optional[np.ndarray], m: int) -> List[Fraction]:
    """Exact law of #{j < m : T[m][j] <= U} for U uniform on [0, 2^32)."""
    if table is None:
        return [Fraction(1)] + [Fraction(0)] * m
    row = [int(v) for v in table_row(table, m)]
    edges = [0] + row + [TWO32]
    # count == c  <=>  T[c-1] <= U < T[c]   (T[-1] = 0, T[m] = 2^32)
    return [Fraction(edges[c + 1] - edges[c], TWO32) for c in range(m + 1)]


def convolve_pmf(a: Sequence[Fraction], b: Sequence[Fraction]) -> List[Fraction]:
    out = [Fraction(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        if x == 0:
            continue
        for j, y in enumerate(b):
            if y:
                out[i + j] += x * y
    return out


def quantized_binomial_pmf(n: int, table: Optional[np.ndarray]) -> List[Fraction]:
    """Exact law of the chunked sampler for Bin(n, P): sum of independent chunks."""
    pmf = [Fraction(1)]
    left = n
    while left > 0:
        m = min(CHUNK, left)
        pmf = convolve_pmf(pmf, quantized_chunk_pmf(table, m))
        left -= m
    return pmf


def ideal_binomial_pmf(n: int, p: Fraction) -> List[Fraction]:
    return [Fraction(math.comb(n, i)) * p ** i * (1 - p) ** (n - i) for i in range(n + 1)]


# --------------------------------------------------- exact collision laws

def particle_transition(q: int, P: int, P_rest: int) -> List[List[Fraction]]:
    """Single-particle law of the sampling collision (no flip): a particle of
    velocity i is picked with probability p = P/2^32 and then sent to velocity
    j with probability w_j; otherwise it keeps velocity i.
    T_ij = (1-p) delta_ij + p w_j, with the fixed-point weights
    (1/2, 1/2) or ((1-wr)/2, wr, (1-wr)/2), wr = P_rest/2^32."""
    p = Fraction(P, TWO32)
    if q == 2:
        w = [Fraction(1, 2), Fraction(1, 2)]
    else:
        wr = Fraction(P_rest, TWO32)
        w = [(1 - wr) / 2, wr, (1 - wr) / 2]
    return [[(1 - p) * (1 if i == j else 0) + p * w[j] for j in range(q)] for i in range(q)]


def _multinomial_law(n: int, probs: Sequence[Fraction]) -> Dict[tuple, Fraction]:
    """Law of the destination counts of n independent particles."""
    law: Dict[tuple, Fraction] = {tuple([0] * len(probs)): Fraction(1)}
    for _ in range(n):
        nxt: Dict[tuple, Fraction] = {}
        for key, pr in law.items():
            for j, pj in enumerate(probs):
                if pj == 0:
                    continue
                k2 = list(key)
                k2[j] += 1
                k2 = tuple(k2)
                nxt[k2] = nxt.get(k2, Fraction(0)) + pr * pj
        law = nxt
    return law


def collision_law_particles(n_in: Sequence[int], q: int, P: int, P_rest: int,
                            flip: bool) -> Dict[tuple, Fraction]:
    """Exact law of the post-collision counts c (before streaming) for input n,
    by independent particles: flip first (Eq. LGflip), then each of the a_i
    particles of velocity i moves with the row T_i. of particle_transition."""
    a = list(reversed(n_in)) if flip else list(n_in)
    T = particle_transition(q, P, P_rest)
    law: Dict[tuple, Fraction] = {tuple([0] * q): Fraction(1)}
    for i in range(q):
        part = _multinomial_law(a[i], T[i])
        nxt: Dict[tuple, Fraction] = {}
        for k1, p1 in law.items():
            for k2, p2 in part.items():
                kk = tuple(x + y for x, y in zip(k1, k2))
                nxt[kk] = nxt.get(kk, Fraction(0)) + p1 * p2
        law = nxt
    return law


def collision_law_exchange(n_in: Sequence[int], P_x: int, flip: bool) -> Dict[tuple, Fraction]:
    """Exact law of the D1Q2 post-collision counts when every particle
    crosses to the opposite velocity with probability P_x / 2^32, independently
    (the flip applied first)."""
    a = list(reversed(n_in)) if flip else list(n_in)
    px = Fraction(P_x, TWO32)
    bx = ideal_binomial_pmf(a[0], px)
    by = ideal_binomial_pmf(a[1], px)
    law: Dict[tuple, Fraction] = {}
    for X, pX in enumerate(bx):
        for Y, pY in enumerate(by):
            c = (a[0] - X + Y, a[1] - Y + X)
            law[c] = law.get(c, Fraction(0)) + pX * pY
    return law


def collision_law_sampler(n_in: Sequence[int], q: int, tab_p, tab_half, tab_rest,
                          flip: bool) -> Dict[tuple, Fraction]:
    """Exact law of the fixed-point sampler itself: removal k_i ~ Qbin(a_i, P),
    M = sum k, then M split by the quantized redistribution binomials."""
    a = list(reversed(n_in)) if flip else list(n_in)
    kl = [quantized_binomial_pmf(a[i], tab_p) for i in range(q)]
    law: Dict[tuple, Fraction] = {}

    def add(c, pr):
        law[c] = law.get(c, Fraction(0)) + pr

    import itertools
    for ks in itertools.product(*[range(a[i] + 1) for i in range(q)]):
        pk = Fraction(1)
        for i in range(q):
            pk *= kl[i][ks[i]]
        if pk == 0:
            continue
        M = sum(ks)
        if q == 2:
            for m0, pm in enumerate(quantized_binomial_pmf(M, tab_half)):
                if pm:
                    add((a[0] - ks[0] + m0, a[1] - ks[1] + (M - m0)), pk * pm)
        else:
            for m1, p1 in enumerate(quantized_binomial_pmf(M, tab_rest)):
                if not p1:
                    continue
                R = M - m1
                for m0, p0 in enumerate(quantized_binomial_pmf(R, tab_half)):
                    if p0:
                        add((a[0] - ks[0] + m0, a[1] - ks[1] + m1, a[2] - ks[2] + (R - m0)),
                            pk * p1 * p0)
    return law


# ------------------------------------------------- lattice Boltzmann (FP64)

def lb_equilibrium(f: np.ndarray, q: int, theta: float) -> np.ndarray:
    """f_i^0 = rho w_i with rho = sum_i f_i."""
    rho = f.sum(axis=0)
    return weights(q, theta)[:, None] * rho[None, :]


def lb_step_flip(f: np.ndarray, q: int, omega_star: float, flip: bool,
                 theta: float = 1.0 / 3.0) -> np.ndarray:
    """Boltzmann average of the lattice gas with flip (first equation of the
    Boltzmann-approximation section):
        f_i(x + v_i, t + 1) = F_i[f] + omega* (f_i^0 - F_i[f]),
    periodic in x.  Without the flip this is the BGK lattice Boltzmann step."""
    a = f[::-1].copy() if flip else f.copy()
    post = a + omega_star * (lb_equilibrium(a, q, theta) - a)
    out = np.empty_like(post)
    for i, v in enumerate(velocities(q)):
        out[i] = np.roll(post[i], int(v))
    return out


def moment_matrix(q: int, theta: float = 1.0 / 3.0) -> np.ndarray:
    """Transformation matrix m_i^a (rows a, columns i).  D1Q3: Eq. transform;
    D1Q2: rows (1, 1) and (-1, 1) (theta = 1)."""
    if q == 2:
        return np.array([[1.0, 1.0], [-1.0, 1.0]])
    s = math.sqrt(1.0 / theta)
    return np.array([[1.0, 1.0, 1.0],
                     [-s, 0.0, s],
                     [math.sqrt((1 - theta) / theta), -math.sqrt(theta / (1 - theta)),
                      math.sqrt((1 - theta) / theta)]])


def mrt_rates(q: int, omega_star: float, flip: bool) -> np.ndarray:
    """(omega^rho, omega^j[, omega^Pi]): the flip negates the odd moment j
    (Eq. momentspaceFm) so j relaxes with omega^j = 2 - omega* (Eq. omegaj);
    the even ghost moment Pi relaxes with omega*.  omega^rho is arbitrary
    (rho is conserved); 1 is used."""
    wj = (2.0 - omega_star) if flip else omega_star
    return np.array([1.0, wj]) if q == 2 else np.array([1.0, wj, omega_star])


def mrt_step(f: np.ndarray, q: int, omega_star: float, flip: bool,
             theta: float = 1.0 / 3.0) -> np.ndarray:
    """MRT form of the same step (Eq. MRTLB read with the equilibrium restored):
        f_i(x+v_i, t+1) = f_i^0 + sum_a w_i m_i^a (1 - omega^a) sum_j m_j^a (f_j - f_j^0)."""
    m = moment_matrix(q, theta)
    w = weights(q, theta)
    feq = lb_equilibrium(f, q, theta)
    dev = m @ (f - feq)                          # moments of the non-equilibrium part
    dev = (1.0 - mrt_rates(q, omega_star, flip))[:, None] * dev
    post = feq + w[:, None] * (m.T @ dev)
    out = np.empty_like(post)
    for i, v in enumerate(velocities(q)):
        out[i] = np.roll(post[i], int(v))
    return out


def lb_run(f0: np.ndarray, q: int, omega_star: float, flip: bool, steps: int,
           theta: float = 1.0 / 3.0, every: int = 0):
    """Iterate lb_step_flip; with every > 0 also return the states at multiples of every."""
    f = np.array(f0, dtype=np.float64)
    snaps = []
    for s in range(steps):
        if every and s % every == 0:
            snaps.append(f.copy())
        f = lb_step_flip(f, q, omega_star, flip, theta)
    if every:
        snaps.append(f.copy())
        return f, snaps
    return f


def lb_step_flip_2d(f: np.ndarray, omega_star: float, flip: bool,
                    theta: float = 1.0 / 3.0) -> np.ndarray:
    """D2Q5 Boltzmann average with flip, f of shape [5][Ly][Lx] (periodic):
    a = F[f] (a_i = f_{4-i}), post = a + omega* (w_i rho - a), then
    f_i(x + v_i) = post_i(x)."""
    w = weights(5, theta)
    a = f[::-1].copy() if flip else f.copy()
    rho = a.sum(axis=0)
    post = a + omega_star * (w[:, None, None] * rho[None] - a)
    out = np.empty_like(post)
    for i, (vx, vy) in enumerate(velocities(5)):
        out[i] = np.roll(np.roll(post[i], int(vx), axis=1), int(vy), axis=0)
    return out


def lb_mode_matrix_2d(kx: float, ky: float, omega_star: float, flip: bool,
                      theta: float = 1.0 / 3.0) -> np.ndarray:
    """One D2Q5 step on a plane wave f_i(x) = g_i exp(i k.x): the collision
    ((1 - omega*) I + omega* w 1^T) after the flip permutation, then streaming,
    which multiplies component i by exp(-i k.v_i)."""
    w = weights(5, theta)
    Pm = np.eye(5)[::-1] if flip else np.eye(5)
    C = (1.0 - omega_star) * np.eye(5) + omega_star * np.outer(w, np.ones(5))
    v = velocities(5)
    S = np.diag(np.exp(-1j * (kx * v[:, 0] + ky * v[:, 1])))
    return S @ C @ Pm


def lb_slow_rate_2d(kx: float, ky: float, omega_star: float, flip: bool,
                    theta: float = 1.0 / 3.0) -> float:
    """-log |lambda| of the eigenvalue of lb_mode_matrix_2d closest to 1 (the
    density mode)."""
    ev = np.linalg.eigvals(lb_mode_matrix_2d(kx, ky, omega_star, flip, theta))
    lam = ev[np.argmin(np.abs(ev - 1.0))]
    return float(-math.log(abs(lam)))


def lb_operator(q: int, length: int, omega_star: float, flip: bool,
                theta: float = 1.0 / 3.0) -> np.ndarray:
    """Dense matrix A of one step on the flattened state (index i*L + x)."""
    n = q * length
    A = np.zeros((n, n))
    for col in range(n):
        e = np.zeros(n)
        e[col] = 1.0
        A[:, col] = lb_step_flip(e.reshape(q, length), q, omega_star, flip, theta).reshape(-1)
    return A


def lb_mode_matrix(q: int, k: float, omega_star: float, flip: bool,
                   theta: float = 1.0 / 3.0) -> np.ndarray:
    """One step acting on a plane wave f_i(x) = g_i exp(i k x): collision with
    flip, C = [(1-omega*) I + omega* w 1^T] F, then streaming by v_i, which
    multiplies component i by exp(-i k v_i)."""
    w = weights(q, theta)
    F = np.eye(q)[::-1] if flip else np.eye(q)
    C = ((1.0 - omega_star) * np.eye(q) + omega_star * np.outer(w, np.ones(q))) @ F
    S = np.diag(np.exp(-1j * k * velocities(q)))
    return S @ C


def lb_slow_rate(q: int, length: int, omega_star: float, flip: bool,
                 theta: float = 1.0 / 3.0, mode: int = 1) -> float:
    """-ln(lambda)/k^2 for the eigenvalue lambda of mode k = 2 pi mode / L
    closest to 1 (the diffusive density mode)."""
    k = 2.0 * math.pi * mode / length
    ev = np.linalg.eigvals(lb_mode_matrix(q, k, omega_star, flip, theta))
    lam = ev[np.argmin(np.abs(ev - 1.0))]
    return float(-math.log(abs(lam)) / k ** 2)


# ------------------------------------------------------------ closed forms

def diffusion_constant(omega_j: float, theta_val: float) -> float:
    """D = theta (1/omega^j - 1/2) (after Eq. diffusioneqn; Integer Lattice Gas
    section for omega <= 1)."""
    return theta_val * (1.0 / omega_j - 0.5)


def amplitude_theory(t, nave: float, D: float, length: int):
    """A^th(t) = N^ave exp(-4 pi^2 D t / L^2)  (Eq. ampdecay)."""
    return nave * np.exp(-4.0 * math.pi ** 2 * D * np.asarray(t, dtype=np.float64) / length ** 2)


def amplitude_lg(N: np.ndarray) -> float:
    """A^LG = sum_x sin(2 pi x/L) N(x) / sum_x sin^2(2 pi x/L)  (Results section)."""
    L = N.shape[-1]
    s = np.sin(2.0 * math.pi * np.arange(L) / L)
    return float(np.dot(s, N.astype(np.float64)) / np.dot(s, s))


def structure_factor(N: np.ndarray, kmax: int) -> np.ndarray:
    """S(k) = |sum_x N(x) exp(-2 pi i k x / L)|^2 / sum_x N(x), k = 1..kmax,
    by direct summation (Poisson equilibrium gives 1)."""
    L = N.shape[-1]
    x = np.arange(L)
    Nf = N.astype(np.float64)
    out = np.empty(kmax)
    for k in range(1, kmax + 1):
        ang = 2.0 * math.pi * k * x / L
        re = np.dot(Nf, np.cos(ang))
        im = -np.dot(Nf, np.sin(ang))
        out[k - 1] = (re * re + im * im) / Nf.sum()
    return out


def moments_raw(state: np.ndarray, q: int):
    """Per-node exact integer moments (the density and current of the named
    moments, Eq. transform, before their Hermite normalisation): rho =
    sum_i n_i, J = sum_i v_i n_i, E = sum_i |v_i|^2 n_i.  D2Q5 ([5][nodes] or
    [5][Ly][Lx]): J is the x component sum_i v_ix n_i."""
    s = state.astype(np.int64).reshape(q, -1)
    v = velocities(q)
    vx = v[:, 0] if v.ndim == 2 else v
    v2 = (v * v).sum(axis=1) if v.ndim == 2 else v * v
    shape = state.shape[1:]
    return (s.sum(axis=0).reshape(shape), (vx[:, None] * s).sum(axis=0).reshape(shape),
            (v2[:, None] * s).sum(axis=0).reshape(shape))
