"""ctypes front end of the plain C oracle (ilg_oracle.c) plus its build step.

TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the
benchmark's CPU-baseline leg.  Nothing in the product package imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

from . import exact

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ilg_oracle.c")
_BUILD_DIR = os.path.join(_HERE, "_build")
# ILG_ORACLE_LIB names another build of ilg_oracle.c to load instead (the
# mutation tests load scratch copies with planted mistakes this way).
_LIB_PATH = os.environ.get("ILG_ORACLE_LIB") or os.path.join(_BUILD_DIR, "libilg_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (plain -O2, pthreads)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    os.makedirs(_BUILD_DIR, exist_ok=True)
    tmp = _LIB_PATH + ".tmp"
    subprocess.run(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared", "-pthread",
                    _SRC, "-o", tmp, "-lm"], check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        vp = ctypes.c_void_p
        L.oracle_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.oracle_philox4x32_10.restype = None
        L.oracle_philox4x32.argtypes = [u32p, u32p, ctypes.c_int, u32p]
        L.oracle_philox4x32.restype = None
        L.oracle_step.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                  ctypes.c_uint64, ctypes.c_int, ctypes.c_int, vp, vp, vp,
                                  ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, vp, vp,
                                  ctypes.c_int]
        L.oracle_step.restype = ctypes.c_int
        L.oracle_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_int, vp, vp,
                                 vp, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                                 ctypes.c_uint64, vp, vp, ctypes.c_int]
        L.oracle_run.restype = ctypes.c_int
        L.oracle_run_window.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                        ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, vp, vp, vp,
                                        ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                                        ctypes.c_uint64, vp, ctypes.c_int]
        L.oracle_run_window.restype = ctypes.c_int
        L.oracle_hash.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, vp]
        L.oracle_hash.restype = ctypes.c_uint64
        L.oracle_collide_node.argtypes = [ctypes.c_int, ctypes.c_int, vp, vp, vp, ctypes.c_uint64,
                                          ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, vp,
                                          vp]
        L.oracle_collide_node.restype = None
        L.oracle_collide_samples.argtypes = [ctypes.c_int, ctypes.c_int, vp, vp, vp,
                                             ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                             vp, ctypes.c_uint64, vp]
        L.oracle_collide_samples.restype = None
        L.oracle_binomial_samples.argtypes = [ctypes.c_uint64, vp, ctypes.c_uint64,
                                              ctypes.c_uint64, vp]
        L.oracle_binomial_samples.restype = None
        L.oracle_run2d.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int,
                                   vp, vp, vp, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                                   ctypes.c_uint64, vp, vp, ctypes.c_int]
        L.oracle_run2d.restype = ctypes.c_int
        L.oracle_sin2pi_frac.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.oracle_sin2pi_frac.restype = ctypes.c_double
        L.oracle_exp_neg.argtypes = [ctypes.c_double]
        L.oracle_exp_neg.restype = ctypes.c_double
        L.oracle_init_poisson_sine.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                               ctypes.c_uint64, ctypes.c_uint64,
                                               ctypes.c_uint64, vp,
                                               ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                               ctypes.c_uint32, vp]
        L.oracle_init_poisson_sine.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"]
    return ctypes.c_void_p(a.ctypes.data)


class Params:
    """Fixed-point collision parameters and their exact tables."""

    def __init__(self, q: int, omega: float, theta: float = 1.0 / 3.0, flip: str = "auto",
                 rounds: int = 10, exchange: bool = False):
        """rounds: Philox rounds of the step draws, 10 (draw specification
        v1) or 7 (v2).  exchange: the D1Q2 exchange form (specification v3):
        two crossing binomials with probability P_x = round(omega* 2^31),
        whose table replaces tab_p."""
        if rounds not in (7, 10):
            raise ValueError("rounds must be 10 or 7")
        if exchange and q != 2:
            raise ValueError("the exchange form is defined for D1Q2")
        self.q = q
        self.rounds = rounds
        self.exchange = exchange
        self.omega = omega
        self.theta = theta
        fp = exact.fixed_point_params(omega, theta, flip, q=q)
        self.flip = fp["flip"]
        self.omega_star = fp["omega_star"]
        self.P, self.P_half, self.P_rest = fp["P"], fp["P_half"], fp["P_rest"]
        self.P_x = fp["P_x"]
        self.tab_p = exact.binomial_table(self.P_x if exchange else self.P)
        self.tab_half = _cached_table(self.P_half)
        self.tab_rest = _cached_table(self.P_rest) if q in (3, 5) else None

    @property
    def flipword(self) -> int:
        """The C entry points' flip argument: bit 0 the flip, bit 1 the
        exchange form, bits 8..15 the Philox round count (0 for 10)."""
        return (int(self.flip) | (2 if self.exchange else 0)
                | (0 if self.rounds == 10 else self.rounds << 8))


_table_cache = {}


def _cached_table(P: int):
    if P not in _table_cache:
        _table_cache[P] = exact.binomial_table(P)
    return _table_cache[P]


def philox(ctr, key, rounds: int = 10) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    lib().oracle_philox4x32(c.ctypes.data_as(u32p), k.ctypes.data_as(u32p), rounds,
                            out.ctypes.data_as(u32p))
    return out


def state_hash(state: np.ndarray) -> int:
    """Hash of a [q][L] state, or of a D2Q5 [5][Ly][Lx] state with node
    index x + Lx y."""
    q = state.shape[0]
    s = np.ascontiguousarray(state)
    return int(lib().oracle_hash(q, s.dtype.itemsize, s.size // q, _ptr(s)))


def run(params: Params, state: np.ndarray, nsteps: int, seed: int, realization: int = 0,
        t0: int = 0, hashes: bool = False, nthreads: Optional[int] = None):
    """Advance a whole periodic lattice; returns (new_state, hashes or None, overflow)."""
    s = np.array(state, copy=True, order="C")
    q, L = s.shape
    assert q == params.q
    hs = np.zeros(max(nsteps, 1), dtype=np.uint64) if hashes else None
    ov = lib().oracle_run(q, s.dtype.itemsize, L, params.flipword, _ptr(params.tab_p),
                          _ptr(params.tab_half), _ptr(params.tab_rest), seed, realization, t0,
                          nsteps, _ptr(s), _ptr(hs), nthreads or default_threads())
    return s, (hs[:nsteps] if hashes else None), bool(ov)


def run2d(params: Params, state: np.ndarray, nsteps: int, seed: int, realization: int = 0,
          t0: int = 0, hashes: bool = False, nthreads: Optional[int] = None):
    """Advance a periodic D2Q5 lattice, state [5][Ly][Lx]; returns
    (new_state, hashes or None, overflow).  Node index x + Lx y."""
    s = np.array(state, copy=True, order="C")
    q, ly, lx = s.shape
    assert q == 5 and params.q == 5
    hs = np.zeros(max(nsteps, 1), dtype=np.uint64) if hashes else None
    ov = lib().oracle_run2d(s.dtype.itemsize, lx, ly, params.flipword, _ptr(params.tab_p),
                            _ptr(params.tab_half), _ptr(params.tab_rest), seed, realization, t0,
                            nsteps, _ptr(s), _ptr(hs), nthreads or default_threads())
    return s, (hs[:nsteps] if hashes else None), bool(ov)


def run_window(params: Params, window: np.ndarray, length: int, x0: int, nsteps: int, seed: int,
               realization: int = 0, t0: int = 0, nthreads: Optional[int] = None):
    """Light-cone run of the window [x0, x0+W) (global indices mod length);
    returns the window after nsteps, valid on [nsteps, W - nsteps)."""
    s = np.array(window, copy=True, order="C")
    q, W = s.shape
    ov = lib().oracle_run_window(q, s.dtype.itemsize, length, x0, W, params.flipword,
                                 _ptr(params.tab_p), _ptr(params.tab_half), _ptr(params.tab_rest),
                                 seed, realization, t0, nsteps, _ptr(s),
                                 nthreads or default_threads())
    return s, bool(ov)


def collide_samples(params: Params, n_in, nsamples: int, seed: int, realization: int = 0,
                    t: int = 0) -> np.ndarray:
    n = np.zeros(5, dtype=np.uint64)
    n[:params.q] = n_in
    out = np.zeros((nsamples, params.q), dtype=np.uint64)
    lib().oracle_collide_samples(params.q, params.flipword, _ptr(params.tab_p),
                                 _ptr(params.tab_half), _ptr(params.tab_rest), seed, realization,
                                 t, _ptr(n), nsamples, _ptr(out))
    return out


def binomial_samples(n: int, table: Optional[np.ndarray], nsamples: int, seed: int) -> np.ndarray:
    out = np.zeros(nsamples, dtype=np.uint64)
    lib().oracle_binomial_samples(n, _ptr(table), seed, nsamples, _ptr(out))
    return out


def init_weights(q: int, theta: float = 1.0 / 3.0) -> np.ndarray:
    """Velocity weights of the initial means: D1Q2 (1/2, 1/2); D1Q3
    (theta/2, 1 - theta, theta/2); D2Q5 (theta/2, theta/2, 1 - 2 theta,
    theta/2, theta/2), each one double operation."""
    if q == 2:
        return np.array([0.5, 0.5])
    if q == 5:
        h = theta * 0.5
        return np.array([h, h, 1.0 - 2.0 * theta, h, h])
    return np.array([theta * 0.5, 1.0 - theta, theta * 0.5])


def init_poisson_sine(q: int, count_bytes: int, length: int, nave: float, amp: float,
                      seed: int, realization: int = 0, theta: float = 1.0 / 3.0, x0: int = 0,
                      width: Optional[int] = None, height: int = 0):
    """Poisson sine initial state of nodes x0 .. x0+width-1 (mod the node
    count), as [q][width] counts, and the overflow flag (init v1, see
    ilg_oracle.c).  D2Q5: length = Lx, height = Ly, nodes x + Lx y, profile
    along x; with width None the result is the whole [5][Ly][Lx] state."""
    nodes = length * (height if q == 5 else 1)
    whole = width is None
    width = nodes if whole else width
    w = np.ascontiguousarray(init_weights(q, theta), dtype=np.float64)
    out = np.zeros((q, width), dtype=np.uint16 if count_bytes == 2 else np.uint32)
    ov = lib().oracle_init_poisson_sine(q, count_bytes, nodes, length, x0, width, _ptr(w),
                                        float(nave), float(amp), seed, realization, _ptr(out))
    if q == 5 and whole:
        out = out.reshape(5, height, length)
    return out, bool(ov)


def sin2pi_frac(x: int, length: int) -> float:
    return float(lib().oracle_sin2pi_frac(x, length))


def exp_neg(m: float) -> float:
    return float(lib().oracle_exp_neg(m))
