"""Seeded synthetic inputs for the diffusive integer lattice gas.

This module is shared by the CPU oracle tests, the GPU parity tests, the
benchmark and the smoke check. It only draws initial occupation numbers and run
parameters (lattice length, relaxation rate, Philox seed, realization id, step
count); it holds none of the lattice-gas arithmetic (no flip, no collision, no
streaming, no fixed-point conversion, no diagnostics).

Recipes follow the paper's validation workload (sine density initialised with
Poisson occupations, Results section, Eqs. sineinit and the Poisson
initialisation that follows the figure) and the benchmark workloads at their
stated sizes. Every generator is deterministic in its seed.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence

import numpy as np

# Qian weights of the two velocity sets, as input data for the Poisson
# initialisers (means per velocity are weight * local density).
D1Q2_WEIGHTS = (0.5, 0.5)
D1Q3_WEIGHTS = (1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0)


def count_dtype(count_bytes: int):
    if count_bytes == 2:
        return np.uint16
    if count_bytes == 4:
        return np.uint32
    raise ValueError(f"count_bytes must be 2 or 4, got {count_bytes}")


@dataclasses.dataclass(frozen=True)
class RunSpec:
    """One lattice run: parameters plus how its initial state is drawn."""
    q: int
    length: int
    count_bytes: int
    omega: float
    seed: int
    realization: int
    steps: int
    theta: float = 1.0 / 3.0


# ---------------------------------------------------------------- initial states

def init_round_sine_split(length: int, mean: float = 20.0, amp: float = 10.0,
                          count_bytes: int = 4) -> np.ndarray:
    """D1Q2 state with rho(x) = round(mean + amp*sin(2 pi x / L)) split evenly.

    Odd rho puts the extra particle on the +1 velocity: n_-1 = floor(rho/2),
    n_+1 = rho - floor(rho/2).  Layout [2][L] (velocity-major).
    """
    x = np.arange(length, dtype=np.float64)
    rho = np.rint(mean + amp * np.sin(2.0 * np.pi * x / length)).astype(np.int64)
    out = np.empty((2, length), dtype=count_dtype(count_bytes))
    out[0] = rho // 2
    out[1] = rho - rho // 2
    return out


def init_poisson_iid(q: int, length: int, mean: float, count_bytes: int,
                     init_seed: int) -> np.ndarray:
    """Independent Poisson(mean) occupation on every (velocity, node)."""
    rng = np.random.default_rng(init_seed)
    vals = rng.poisson(mean, size=(q, length))
    return vals.astype(count_dtype(count_bytes))


def init_poisson_sine(weights: Sequence[float], length: int, nave: float, amp: float,
                      count_bytes: int, init_seed: int) -> np.ndarray:
    """Poisson occupations with mean w_i * (nave + amp*sin(2 pi x / L)).

    This is the paper's initialisation of a sine density profile with integer
    occupation numbers (Results section, after the amplitude-decay figure).
    """
    rng = np.random.default_rng(init_seed)
    x = np.arange(length, dtype=np.float64)
    rho = nave + amp * np.sin(2.0 * np.pi * x / length)
    means = np.outer(np.asarray(weights, dtype=np.float64), rho)
    return rng.poisson(means).astype(count_dtype(count_bytes))


# ---------------------------------------------------------------- named workloads

def workload_d1q2_l256() -> tuple[RunSpec, np.ndarray]:
    """D1Q2, L=256 periodic, uint32, rounded sine split evenly, omega=1.5, 1000 steps."""
    spec = RunSpec(q=2, length=256, count_bytes=4, omega=1.5, seed=1, realization=0, steps=1000)
    return spec, init_round_sine_split(256, count_bytes=4)


def workload_d1q3_big(length: int = 1 << 24, steps: int = 2000) -> tuple[RunSpec, np.ndarray]:
    """D1Q3, L=2^24 periodic, uint16, Poisson(50) i.i.d., omega=1.8, 2000 steps."""
    spec = RunSpec(q=3, length=length, count_bytes=2, omega=1.8, seed=1, realization=0, steps=steps)
    return spec, init_poisson_iid(3, length, 50.0, 2, init_seed=2)


@dataclasses.dataclass
class Ensemble:
    specs: List[RunSpec]
    inits: List[np.ndarray]

    @property
    def total_nodes(self) -> int:
        return sum(s.length for s in self.specs)


def ensemble_ragged_d1q2(nreal: int = 4096, steps: int = 5000, lmin: int = 64,
                         lmax: int = 8192, init_seed: int = 3) -> Ensemble:
    """Ragged D1Q2 ensemble: L log-uniform in [lmin, lmax], omega ~ U[1.0, 1.95],
    Philox seed 1000 + r, Poisson(30) per velocity, uint16."""
    rng = np.random.default_rng(init_seed)
    lens = np.rint(np.exp(rng.uniform(math.log(lmin), math.log(lmax), size=nreal))).astype(np.int64)
    omegas = rng.uniform(1.0, 1.95, size=nreal)
    specs, inits = [], []
    for r in range(nreal):
        L = int(lens[r])
        specs.append(RunSpec(q=2, length=L, count_bytes=2, omega=float(omegas[r]),
                             seed=1000 + r, realization=r, steps=steps))
        inits.append(rng.poisson(30.0, size=(2, L)).astype(np.uint16))
    return Ensemble(specs, inits)


DECAY_SWEEP_OMEGAS = (1.0, 1.25, 1.5, 1.75, 1.9, 1.98)


def ensemble_decay_sweep(nper: int = 1024, length: int = 4096, steps: int = 10000,
                         omegas: Sequence[float] = DECAY_SWEEP_OMEGAS, nave: float = 100.0,
                         amp: float = 40.0, count_bytes: int = 4,
                         init_seed: int = 4) -> Ensemble:
    """D1Q3 sine-mode decay sweep: nper realizations per omega, Poisson sine init
    with mean w_i (nave + amp sin(2 pi x/L)); seed = 10^6 * omega_index + r."""
    specs, inits = [], []
    rng = np.random.default_rng(init_seed)
    x = np.arange(length, dtype=np.float64)
    rho = nave + amp * np.sin(2.0 * np.pi * x / length)
    means = np.outer(np.asarray(D1Q3_WEIGHTS), rho)
    dt = count_dtype(count_bytes)
    for oi, om in enumerate(omegas):
        for r in range(nper):
            specs.append(RunSpec(q=3, length=length, count_bytes=count_bytes, omega=float(om),
                                 seed=1_000_000 * oi + r, realization=r, steps=steps))
            inits.append(rng.poisson(means).astype(dt))
    return Ensemble(specs, inits)


@dataclasses.dataclass(frozen=True)
class Request:
    arrival_s: float
    spec: RunSpec
    init_seed: int
    mean: float = 40.0

    def init(self) -> np.ndarray:
        return init_poisson_iid(self.spec.q, self.spec.length, self.mean,
                                self.spec.count_bytes, self.init_seed)


def request_stream(rate_per_s: float = 200.0, duration_s: float = 60.0, lmin_log2: int = 8,
                   lmax_log2: int = 20, tmin: int = 100, tmax: int = 10000,
                   seed: int = 5) -> List[Request]:
    """Poisson arrivals of D1Q2/D1Q3 runs (50/50), L log-uniform 2^8..2^20,
    steps uniform 100..10000, omega ~ U[1.0, 1.95], uint16, Poisson(40) init."""
    rng = np.random.default_rng(seed)
    out: List[Request] = []
    t = 0.0
    i = 0
    while True:
        t += rng.exponential(1.0 / rate_per_s)
        if t >= duration_s:
            break
        q = 2 if rng.random() < 0.5 else 3
        L = int(np.rint(2.0 ** rng.uniform(lmin_log2, lmax_log2)))
        steps = int(rng.integers(tmin, tmax + 1))
        om = float(rng.uniform(1.0, 1.95))
        spec = RunSpec(q=q, length=L, count_bytes=2, omega=om, seed=7_000_000 + i,
                       realization=i, steps=steps)
        out.append(Request(arrival_s=t, spec=spec, init_seed=10_000_000 + i))
        i += 1
    return out


class RequestInitPool:
    """Initial states for a request stream without drawing a fresh lattice per
    request: `npool` arrays of [3][2^lmax_log2] i.i.d. Poisson(mean) uint16
    counts; request i uses the first q rows and L columns of array i % npool
    (i.i.d. entries, so every slice is itself i.i.d. Poisson(mean))."""

    def __init__(self, npool: int = 8, lmax_log2: int = 20, mean: float = 40.0, seed: int = 6):
        rng = np.random.default_rng(seed)
        self.pool = [rng.poisson(mean, size=(3, 1 << lmax_log2)).astype(np.uint16)
                     for _ in range(npool)]

    def init(self, i: int, q: int, length: int) -> np.ndarray:
        return np.ascontiguousarray(self.pool[i % len(self.pool)][:q, :length])
