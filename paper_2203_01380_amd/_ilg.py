"""ctypes binding of libilg.so (include/ilg.h).

Argument marshalling only: every step of the lattice-gas path runs in the HIP
kernels of libilg.so.  PyTorch supplies device memory and streams.  If the
library is not built this module raises at import time; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libilg.so")

ABI_VERSION = 1
MAX_K = 64
TABLE_ENTRIES = 2080
FLIP_MODES = {"auto": 0, "off": 1, "on": 2}
DRAWS_PHILOX7 = 4  # draw specification v2 (7-round Philox)
DRAWS_EXCHANGE = 8  # draw specification v3 (D1Q2 exchange form)
STATUS = {0: "ILG_OK", -1: "ILG_E_INVALID", -2: "ILG_E_NOMEM", -3: "ILG_E_DEVICE",
          -4: "ILG_E_OVERFLOW", -5: "ILG_E_RANGE", -6: "ILG_E_BUSY"}


class IlgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class IlgConfig(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_uint32), ("q", ctypes.c_uint32),
                ("count_bytes", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("length", ctypes.c_uint64), ("omega", ctypes.c_double),
                ("theta", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("realization", ctypes.c_uint32), ("height", ctypes.c_uint32),
                ("t0", ctypes.c_uint64)]


class IlgFixed(ctypes.Structure):
    _fields_ = [("flip", ctypes.c_uint32), ("q", ctypes.c_uint32), ("p", ctypes.c_uint64),
                ("p_half", ctypes.c_uint64), ("p_rest", ctypes.c_uint64),
                ("omega_star", ctypes.c_double)]


class IlgSummary(ctypes.Structure):
    _fields_ = [("mass", ctypes.c_uint64), ("step", ctypes.c_uint64), ("hash", ctypes.c_uint64),
                ("amplitude", ctypes.c_double), ("nk", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("sk", ctypes.c_double * MAX_K)]


class IlgBatchDiag(ctypes.Structure):
    _fields_ = [("sk_every", ctypes.c_uint32), ("nk", ctypes.c_uint32),
                ("amp_every", ctypes.c_uint32), ("max_amp", ctypes.c_uint32)]


BATCH_MAX_K = 16


class IlgRequestInfo(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("state", ctypes.c_uint32), ("q", ctypes.c_uint32),
                ("length", ctypes.c_uint64), ("steps_total", ctypes.c_uint64),
                ("steps_done", ctypes.c_uint64), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


class IlgPollInfo(ctypes.Structure):
    _fields_ = [("admitted", ctypes.c_uint32), ("active", ctypes.c_uint32),
                ("queued", ctypes.c_uint32), ("finished", ctypes.c_uint32),
                ("quantum_steps", ctypes.c_uint32), ("failed", ctypes.c_uint32),
                ("bytes_in_use", ctypes.c_uint64), ("bytes_peak", ctypes.c_uint64)]


def _load():
    # torch ships a HIP runtime with the same SONAME as the system one; loading
    # torch first makes libilg.so bind to that single runtime instance, so
    # torch-allocated buffers and streams are valid in the library.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python paper_2203_01380_amd/build.py` "
                          "(the lattice-gas path has no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
    cfgp = ctypes.POINTER(IlgConfig)
    hp = ctypes.c_void_p
    sig = {
        "ilg_last_error": ([], ctypes.c_char_p),
        "ilg_fixed_point": ([cfgp, ctypes.POINTER(IlgFixed)], i32),
        "ilg_binomial_table": ([u64, vp], i32),
        "ilg_state_bytes": ([cfgp], u64),
        "ilg_state_pitch": ([cfgp], u64),
        "ilg_create": ([cfgp, vp, vp, ctypes.POINTER(hp)], i32),
        "ilg_create_on": ([cfgp, vp, vp, vp, ctypes.POINTER(hp)], i32),
        "ilg_state_device": ([hp], vp),
        "ilg_step": ([hp, u64], i32),
        "ilg_get_state": ([hp, vp], i32),
        "ilg_set_state": ([hp, vp, u64], i32),
        "ilg_init_poisson_sine": ([hp, ctypes.c_double, ctypes.c_double, u64], i32),
        "ilg_moments": ([hp, vp, vp, vp, u32, ctypes.POINTER(IlgSummary)], i32),
        "ilg_state_hash": ([hp, ctypes.POINTER(u64)], i32),
        "ilg_current_step": ([hp], u64),
        "ilg_destroy": ([hp], i32),
        "ilg_batch_create": ([cfgp, u32, ctypes.POINTER(ctypes.c_void_p),
                              ctypes.POINTER(IlgBatchDiag), vp, ctypes.POINTER(hp)], i32),
        "ilg_batch_run": ([hp, u64], i32),
        "ilg_batch_tune": ([hp, u32, ctypes.POINTER(u32)], i32),
        "ilg_batch_set_shape": ([hp, u32], i32),
        "ilg_batch_shape_count": ([], u32),
        "ilg_batch_get_state": ([hp, u32, vp], i32),
        "ilg_batch_structure_factor": ([hp, vp, vp], i32),
        "ilg_batch_amplitudes": ([hp, vp, vp], i32),
        "ilg_batch_destroy": ([hp], i32),
        "ilg_server_clock": ([], ctypes.c_double),
        "ilg_server_create": ([u64, u32, ctypes.POINTER(hp)], i32),
        "ilg_server_set_step_nodes": ([hp, u64], i32),
        "ilg_server_set_resident": ([hp, u64, u32], i32),
        "ilg_server_submit": ([hp, cfgp, vp, u64, ctypes.POINTER(u64)], i32),
        "ilg_server_submit_poisson_sine": ([hp, cfgp, ctypes.c_double, ctypes.c_double, u64, u64,
                                            ctypes.POINTER(u64)], i32),
        "ilg_server_poll": ([hp, ctypes.POINTER(IlgPollInfo)], i32),
        "ilg_server_info": ([hp, u64, ctypes.POINTER(IlgRequestInfo)], i32),
        "ilg_server_result": ([hp, u64, vp], i32),
        "ilg_server_cancel": ([hp, u64], i32),
        "ilg_server_destroy": ([hp], i32),
        "ilg_step_noalloc": ([cfgp, vp, vp, u64, vp, u32], i32),
        "ilg_probe_stream": ([u32, u64, vp, vp, vp], i32),
        "ilg_probe_philox": ([u64, u32, u32, u32, u64, vp, vp], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    return L


lib = _load()


def check(rc: int):
    if rc != 0:
        raise IlgError(rc, lib.ilg_last_error().decode())


def make_config(q: int, length: int, count_bytes: int, omega: float, seed: int,
                realization: int = 0, t0: int = 0, theta: float = 0.0,
                flip: str = "auto", height: int = 0, rounds: int = 10,
                exchange: bool = False) -> IlgConfig:
    """height: rows Ly of a D2Q5 lattice (q = 5, length = Lx); 0 otherwise.
    rounds: Philox rounds of the step draws, 10 (draw specification v1) or 7
    (v2).  exchange: the D1Q2 exchange form (v3)."""
    if rounds not in (7, 10):
        raise ValueError("rounds must be 10 or 7")
    flags = (FLIP_MODES[flip] | (DRAWS_PHILOX7 if rounds == 7 else 0)
             | (DRAWS_EXCHANGE if exchange else 0))
    return IlgConfig(ABI_VERSION, q, count_bytes, flags, length, omega, theta, seed,
                     realization, height, t0)


def fixed_point(cfg: IlgConfig) -> IlgFixed:
    out = IlgFixed()
    check(lib.ilg_fixed_point(ctypes.byref(cfg), ctypes.byref(out)))
    return out


def binomial_table(p: int) -> np.ndarray:
    out = np.zeros(TABLE_ENTRIES, dtype=np.uint32)
    check(lib.ilg_binomial_table(p, out.ctypes.data))
    return out


def _dtype(count_bytes: int):
    return np.uint16 if count_bytes == 2 else np.uint32


class Lattice:
    """One periodic lattice on the GPU.

    By default the two state buffers are torch CUDA tensors (ilg_create_on)
    and work is enqueued on torch's current stream; with use_torch=False the
    library allocates them itself (ilg_create)."""

    def __init__(self, q: int, length: int, count_bytes: int, omega: float, seed: int,
                 init: Optional[np.ndarray], realization: int = 0, t0: int = 0,
                 theta: float = 0.0, flip: str = "auto", use_torch: bool = True, stream=None,
                 height: int = 0, rounds: int = 10, exchange: bool = False):
        """init: [q][L] host counts (D2Q5: [5][height][length]), or None for an
        all-zero state (then call init_poisson_sine to draw the initial state
        on the device).  rounds: 10 or 7 Philox rounds for the step draws;
        exchange: the D1Q2 exchange form."""
        self.cfg = make_config(q, length, count_bytes, omega, seed, realization, t0, theta, flip,
                               height, rounds, exchange)
        self.q, self.length, self.count_bytes = q, length, count_bytes
        self.height = height
        self.shape = (q, height, length) if q == 5 else (q, length)
        nodes = length * (height if q == 5 else 1)
        if init is not None:
            init = np.ascontiguousarray(init, dtype=_dtype(count_bytes))
            if init.shape != self.shape:
                raise ValueError(f"init must have shape {self.shape}, got {init.shape}")
            init = init.reshape(q, nodes)
        self._h = ctypes.c_void_p()
        self._bufs = None
        if use_torch:
            import torch
            if stream is None:
                stream = torch.cuda.current_stream()
            self._stream = stream
            nbytes = int(lib.ilg_state_bytes(ctypes.byref(self.cfg)))
            pitch = int(lib.ilg_state_pitch(ctypes.byref(self.cfg)))
            b0 = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            b1 = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            with torch.cuda.stream(stream):
                if init is None:
                    b0.zero_()
                else:
                    padded = np.zeros((q, pitch), dtype=init.dtype)
                    padded[:, :nodes] = init
                    b0.copy_(torch.from_numpy(padded.view(np.uint8).reshape(-1)))
            stream.synchronize()
            self._bufs = (b0, b1)
            check(lib.ilg_create_on(ctypes.byref(self.cfg), ctypes.c_void_p(b0.data_ptr()),
                                    ctypes.c_void_p(b1.data_ptr()),
                                    ctypes.c_void_p(stream.cuda_stream), ctypes.byref(self._h)))
        else:
            self._stream = None
            sp = None if stream is None else ctypes.c_void_p(int(stream))
            check(lib.ilg_create(ctypes.byref(self.cfg),
                                 None if init is None else init.ctypes.data, sp,
                                 ctypes.byref(self._h)))

    @property
    def handle(self):
        return self._h

    def step(self, nsteps: int = 1):
        check(lib.ilg_step(self._h, nsteps))

    @property
    def t(self) -> int:
        return int(lib.ilg_current_step(self._h))

    def state(self) -> np.ndarray:
        out = np.empty(self.shape, dtype=_dtype(self.count_bytes))
        check(lib.ilg_get_state(self._h, out.ctypes.data))
        return out

    def set_state(self, state: np.ndarray, t: int):
        s = np.ascontiguousarray(state, dtype=_dtype(self.count_bytes))
        if s.shape != self.shape:
            raise ValueError(f"state must have shape {self.shape}, got {s.shape}")
        check(lib.ilg_set_state(self._h, s.ctypes.data, t))

    def init_poisson_sine(self, nave: float, amp: float, init_seed: int):
        """Draw the Poisson sine initial state on the device (init v1):
        n_i(x) ~ Poisson(w_i (nave + amp sin(2 pi x / L)))."""
        check(lib.ilg_init_poisson_sine(self._h, float(nave), float(amp), int(init_seed)))

    def hash(self) -> int:
        out = ctypes.c_uint64()
        check(lib.ilg_state_hash(self._h, ctypes.byref(out)))
        return int(out.value)

    def moments(self, per_node: bool = False, nk: int = 0) -> dict:
        s = IlgSummary()
        arrs = ([np.empty(self.shape[1:], dtype=np.int64) for _ in range(3)] if per_node
                else None)
        ptrs = [a.ctypes.data for a in arrs] if per_node else [None, None, None]
        check(lib.ilg_moments(self._h, *ptrs, nk, ctypes.byref(s)))
        out = dict(mass=int(s.mass), step=int(s.step), hash=int(s.hash),
                   amplitude=float(s.amplitude), sk=np.array(s.sk[:nk], dtype=np.float64))
        if per_node:
            out.update(rho=arrs[0], j=arrs[1], e=arrs[2])
        return out

    def close(self):
        if self._h:
            h, self._h = self._h, ctypes.c_void_p()
            check(lib.ilg_destroy(h))
        self._bufs = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            if self._h:
                lib.ilg_destroy(self._h)
        except Exception:
            pass


def _member_shape(m: dict) -> tuple:
    """Host layout of a member's counts: [q][L], or [5][height][length]."""
    if m["q"] == 5:
        return (5, m["height"], m["length"])
    return (m["q"], m["length"])


class Batch:
    """An ensemble of independent lattices advanced by one persistent launch.

    members: sequence of dicts with keys q, length, count_bytes, omega, seed
    and optionally realization, t0, theta, flip, rounds, exchange and (D2Q5)
    height; inits: matching [q][L] arrays ([5][height][length] for D2Q5).
    Work goes to torch's current stream unless `stream` is given."""

    def __init__(self, members, inits, sk_every: int = 0, nk: int = 0, amp_every: int = 0,
                 max_amp: int = 0, stream=None):
        n = len(members)
        if n == 0 or len(inits) != n:
            raise ValueError("need one initial state per member")
        cfgs = (IlgConfig * n)()
        keep = []
        ptrs = (ctypes.c_void_p * n)()
        for r, (m, init) in enumerate(zip(members, inits)):
            cfgs[r] = make_config(m["q"], m["length"], m["count_bytes"], m["omega"], m["seed"],
                                  m.get("realization", 0), m.get("t0", 0), m.get("theta", 0.0),
                                  m.get("flip", "auto"), m.get("height", 0),
                                  m.get("rounds", 10), m.get("exchange", False))
            a = np.ascontiguousarray(init, dtype=_dtype(m["count_bytes"]))
            if a.shape != _member_shape(m):
                raise ValueError(f"member {r}: init shape {a.shape}")
            keep.append(a)
            ptrs[r] = a.ctypes.data
        self.members = [dict(m) for m in members]
        self.nreal = n
        self.q, self.count_bytes = members[0]["q"], members[0]["count_bytes"]
        self.nk = nk if sk_every else 0
        self.max_amp = max_amp if amp_every else 0
        diag = IlgBatchDiag(sk_every, nk, amp_every, max_amp)
        if stream is None:
            import torch
            stream = torch.cuda.current_stream()
        self._stream = stream
        self._h = ctypes.c_void_p()
        check(lib.ilg_batch_create(cfgs, n, ptrs, ctypes.byref(diag),
                                   ctypes.c_void_p(stream.cuda_stream), ctypes.byref(self._h)))

    def run(self, nsteps: int):
        check(lib.ilg_batch_run(self._h, nsteps))

    def tune(self, steps: int = 20) -> int:
        out = ctypes.c_uint32()
        check(lib.ilg_batch_tune(self._h, steps, ctypes.byref(out)))
        return int(out.value)

    def set_shape(self, shape: int):
        check(lib.ilg_batch_set_shape(self._h, shape))

    @staticmethod
    def shape_count() -> int:
        return int(lib.ilg_batch_shape_count())

    def state(self, r: int) -> np.ndarray:
        m = self.members[r]
        out = np.empty(_member_shape(m), dtype=_dtype(m["count_bytes"]))
        check(lib.ilg_batch_get_state(self._h, r, out.ctypes.data))
        return out

    def structure_factor(self):
        sums = np.zeros((self.nreal, max(self.nk, 1)), dtype=np.float64)
        cnt = np.zeros(self.nreal, dtype=np.uint64)
        check(lib.ilg_batch_structure_factor(self._h, sums.ctypes.data, cnt.ctypes.data))
        return sums[:, :self.nk], cnt

    def amplitudes(self):
        amp = np.zeros((self.nreal, max(self.max_amp, 1)), dtype=np.float64)
        cnt = np.zeros(self.nreal, dtype=np.uint32)
        check(lib.ilg_batch_amplitudes(self._h, amp.ctypes.data, cnt.ctypes.data))
        return amp[:, :self.max_amp], cnt

    def close(self):
        if self._h:
            h, self._h = self._h, ctypes.c_void_p()
            check(lib.ilg_batch_destroy(h))

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            if self._h:
                lib.ilg_batch_destroy(self._h)
        except Exception:
            pass


REQ_STATES = {0: "queued", 1: "active", 2: "done", 3: "cancelled", 4: "failed"}


class Server:
    """Continuous-batching request server (ilg_server_*)."""

    def __init__(self, budget_bytes: int, quantum_steps: int = 100, step_nodes: int = 0,
                 resident: Optional[tuple] = None):
        """resident: (max_nodes, max_steps) for ilg_server_set_resident, or
        None for the library's default (small requests of up to 4096 nodes,
        up to 16 quanta per poll)."""
        self._h = ctypes.c_void_p()
        check(lib.ilg_server_create(budget_bytes, quantum_steps, ctypes.byref(self._h)))
        if step_nodes:
            self.set_step_nodes(step_nodes)
        if resident is not None:
            self.set_resident(*resident)
        self._shapes = {}

    def set_resident(self, max_nodes: int, max_steps: int = 0):
        """Requests of at most max_nodes nodes advance inside one workgroup,
        by up to max_steps steps per poll (at least the quantum); 0: none."""
        check(lib.ilg_server_set_resident(self._h, max_nodes, max_steps))

    def set_step_nodes(self, max_nodes: int):
        """Advance at most max_nodes nodes per quantum, least remaining work
        first (0: every active request)."""
        check(lib.ilg_server_set_step_nodes(self._h, max_nodes))

    @staticmethod
    def clock() -> float:
        return float(lib.ilg_server_clock())

    def submit(self, member: dict, init: np.ndarray, nsteps: int) -> int:
        cfg = make_config(member["q"], member["length"], member["count_bytes"], member["omega"],
                          member["seed"], member.get("realization", 0), member.get("t0", 0),
                          member.get("theta", 0.0), member.get("flip", "auto"),
                          member.get("height", 0), member.get("rounds", 10),
                          member.get("exchange", False))
        a = np.ascontiguousarray(init, dtype=_dtype(member["count_bytes"]))
        if a.shape != _member_shape(member):
            raise ValueError(f"init shape {a.shape}")
        rid = ctypes.c_uint64()
        check(lib.ilg_server_submit(self._h, ctypes.byref(cfg), a.ctypes.data, nsteps,
                                    ctypes.byref(rid)))
        self._shapes[int(rid.value)] = (_member_shape(member), member["count_bytes"])
        return int(rid.value)

    def submit_poisson_sine(self, member: dict, nave: float, amp: float, init_seed: int,
                            nsteps: int) -> int:
        """Queue a request whose initial state is drawn on the device at
        admission (Poisson sine condition, init v1)."""
        cfg = make_config(member["q"], member["length"], member["count_bytes"], member["omega"],
                          member["seed"], member.get("realization", 0), member.get("t0", 0),
                          member.get("theta", 0.0), member.get("flip", "auto"),
                          member.get("height", 0), member.get("rounds", 10),
                          member.get("exchange", False))
        rid = ctypes.c_uint64()
        check(lib.ilg_server_submit_poisson_sine(self._h, ctypes.byref(cfg), float(nave),
                                                 float(amp), int(init_seed), nsteps,
                                                 ctypes.byref(rid)))
        self._shapes[int(rid.value)] = (_member_shape(member), member["count_bytes"])
        return int(rid.value)

    def poll(self) -> dict:
        info = IlgPollInfo()
        check(lib.ilg_server_poll(self._h, ctypes.byref(info)))
        return {f: int(getattr(info, f)) for f, _ in IlgPollInfo._fields_}

    def info(self, rid: int) -> dict:
        out = IlgRequestInfo()
        check(lib.ilg_server_info(self._h, rid, ctypes.byref(out)))
        d = {f: getattr(out, f) for f, _ in IlgRequestInfo._fields_}
        d["state"] = REQ_STATES[int(d["state"])]
        return d

    def result(self, rid: int) -> np.ndarray:
        shape, cb = self._shapes[rid]
        out = np.empty(shape, dtype=_dtype(cb))
        check(lib.ilg_server_result(self._h, rid, out.ctypes.data))
        del self._shapes[rid]
        return out

    def cancel(self, rid: int):
        check(lib.ilg_server_cancel(self._h, rid))
        self._shapes.pop(rid, None)

    def close(self):
        if self._h:
            h, self._h = self._h, ctypes.c_void_p()
            check(lib.ilg_server_destroy(h))

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            if self._h:
                lib.ilg_server_destroy(self._h)
        except Exception:
            pass


def probe_stream(q: int, length: int, src, dst, stream=None):
    """Streaming-only probe (ilg_probe_stream): src and dst are torch uint16
    CUDA tensors of at least q * pitch elements; enqueued on `stream` (torch's
    current stream by default)."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream()
    check(lib.ilg_probe_stream(q, length, src.data_ptr(), dst.data_ptr(), st.cuda_stream))


def probe_philox(length: int, blocks: int, out, rounds: int = 10, t: int = 0, seed: int = 1,
                 stream=None):
    """Draws-only probe (ilg_probe_philox): out is a torch uint32 (or int32)
    CUDA tensor of at least `length` elements."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream()
    check(lib.ilg_probe_philox(length, blocks, rounds, t, seed, out.data_ptr(), st.cuda_stream))
