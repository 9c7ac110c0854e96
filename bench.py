"""Benchmark of the lattice-gas step with flip (flip -> sampling collision -> stream).

Headline workload (the JSON line's value): D1Q3, L = 2^24 periodic nodes,
uint16 counts, Poisson(50) i.i.d. initial state, omega = 1.8 (flip on,
omega* = 0.2), Philox seed 1.  A "step" is one full lattice time step; the
state is resident in HBM before timing; timing uses HIP events on the stream
the kernels run on.

Also reported (extra JSON objects): the same step on a 2^26-node lattice
(state larger than the MALL), the same step with 7-round Philox draws, D1Q2
on 2^24 nodes with three binomials and in the exchange form, the D2Q5
extension on 4096 x 4096 nodes, the
batched ensemble form on the ragged
D1Q2 ensemble (4096 members, L log-uniform in [64, 8192], 5000 steps, S(k)
every 10 steps) against the plain per-realization loop on a sample of the same
members, the batched D1Q3 decay sweep (6 x 1024 members, L = 4096, uint32,
10^4 steps), the continuous-batching server on a Poisson request stream
(q in {2, 3}, L log-uniform 2^8..2^20, 100..10000 steps, uint16) at 1, 1/2 and
1/4 of 200 requests/s with p50/p99 latency, and the CPU oracle timed on a
bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz: VALU lane-instruction slots per
# second (a SIMD issues one wave64 VALU instruction every 4 cycles; a
# half-rate instruction such as the 32x32->64 multiply takes two slots).
VALU_PEAK_T_LANE_INSTS = 256 * 4 * 16 * 2.4e9 / 1e12
ALG_BYTES_PER_NODE_UPDATE = 12    # D1Q3 uint16: 3 counts read + 3 written


def traffic_file(length: int) -> str:
    return os.path.join(ROOT, "profiles", f"traffic_step_d1q3_u16_l2p{length.bit_length() - 1}.json")


SQ_FILE = os.path.join(ROOT, "profiles", "sq_step_d1q3_u16_l2p24.json")


MALL_FREE_LENGTH = 1 << 26   # 768 MiB of double-buffered state, beyond the 256 MB MALL
STEP_SOURCES = [os.path.join(ROOT, "paper_2203_01380_amd", "csrc", f)
                for f in ("step.hip", "sampler.h")]


def step_source_digest() -> str:
    h = hashlib.sha256()
    for p in STEP_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _current_record(path):
    """A committed counter record, or None if absent or taken on a different
    version of the step kernel."""
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("step_source_sha256_16") != step_source_digest():
        return None
    return rec


def counter_traffic(length: int):
    """HBM bytes per launch of the step kernel from the committed counter
    summary for this lattice length (None if absent or stale)."""
    rec = _current_record(traffic_file(length))
    return rec.get("bytes_per_launch") if rec else None


def alu_roofline(ms_per_launch: float, length: int):
    """The step's VALU issue against the chip's VALU issue slots: wave
    instructions per launch (SQ_INSTS_VALU, from the committed counter record
    of the current kernel) x 64 lanes / the launch time measured here."""
    rec = _current_record(SQ_FILE)
    if not rec or rec.get("length") != length:
        return None
    insts = rec["valu_wave_insts_per_launch"]
    achieved = insts * 64 / (ms_per_launch / 1e3) / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_T_LANE_INSTS,
            "unit": "T VALU lane-instructions/s", "frac": achieved / VALU_PEAK_T_LANE_INSTS,
            "valu_lane_insts_per_node_update": insts * 64 / length,
            "source": os.path.relpath(SQ_FILE, ROOT),
            "note": "instruction issue; 32x32->64 multiplies (two per Philox round) "
                    "take two issue slots each, so cycle use is higher than this fraction"}


def say(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


def timed(stream, fn):
    import torch
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3


def cpu_baseline(init, spec, seconds: float):
    """The oracle as it stands, on all host threads (capped at 16), on the same
    lattice, stepping until `seconds` have passed (at least one step)."""
    from oracle import oracle
    threads = oracle.default_threads()
    p = oracle.Params(spec.q, spec.omega)
    state = init
    steps = 0
    t0 = time.perf_counter()
    while True:
        state, _, _ = oracle.run(p, state, 1, seed=spec.seed, t0=steps, nthreads=threads)
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return {"value": spec.length * steps / el, "unit": "node-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{steps} full steps of the same D1Q3 L={spec.length} lattice "
                      f"({spec.length * steps} node-updates, {el:.1f} s)"}


def cpu_other_configs(W, seconds: float):
    """The oracle on bounded samples of the other workloads (each about
    `seconds` of host time): the D1Q2 L = 256 case in full, and members or
    requests of the batched, decay and serving workloads at their real
    lengths for a few steps each."""
    from oracle import oracle
    threads = oracle.default_threads()

    def run_members(items):
        """items: (q, omega, seed, realization, init) lattices, 20 steps each,
        one single-threaded oracle run per host thread at a time (the calls
        release the interpreter lock), rounds over the items until `seconds`
        have passed."""
        from concurrent.futures import ThreadPoolExecutor
        steps_each = 20

        params = {}
        for q, omega, _, _, _ in items:      # tables built once, outside the timing
            params.setdefault((q, omega), oracle.Params(q, omega))

        def one(item):
            q, omega, seed, r, init = item
            oracle.run(params[(q, omega)], init, steps_each, seed=seed, realization=r,
                       nthreads=1)
            return init.shape[1] * steps_each

        work, k = 0, 0
        with ThreadPoolExecutor(threads) as ex:
            t0 = time.perf_counter()
            while True:
                work += sum(ex.map(one, items))
                k += len(items)
                el = time.perf_counter() - t0
                if el >= seconds:
                    return work / el, k, el

    out = {}
    spec, init = W.workload_d1q2_l256()
    p1 = oracle.Params(spec.q, spec.omega)
    t0 = time.perf_counter()
    oracle.run(p1, init, spec.steps, seed=spec.seed, nthreads=1)
    el = time.perf_counter() - t0
    out["d1q2_l256"] = {"node_updates_per_s": spec.length * spec.steps / el, "cores": 1,
                        "sample": f"the full run: {spec.steps} steps of L = 256 in {el:.2f} s"}
    ens = W.ensemble_ragged_d1q2(steps=20)
    order = np.argsort([s.length for s in ens.specs])
    pick = order[np.linspace(0, len(order) - 1, 64).astype(int)]
    rate, k, el = run_members([(2, ens.specs[r].omega, ens.specs[r].seed,
                                ens.specs[r].realization, ens.inits[r]) for r in pick])
    out["batched_ragged"] = {"node_updates_per_s": rate, "cores": threads,
                             "sample": f"{k} member runs of 20 steps over 64 members spread "
                                       f"by length ({el:.1f} s; no S(k))"}
    ens = W.ensemble_decay_sweep(nper=1, steps=20)
    rate, k, el = run_members([(3, s.omega, s.seed, s.realization, ens.inits[i])
                               for i, s in enumerate(ens.specs)])
    out["batched_decay"] = {"node_updates_per_s": rate, "cores": threads,
                            "sample": f"{k} runs of 20 steps, one L = 4096 uint32 member per "
                                      f"omega ({el:.1f} s; no A^LG)"}
    reqs = W.request_stream(rate_per_s=200, duration_s=0.2)
    pool = W.RequestInitPool(npool=2)
    rate, k, el = run_members([(rq.spec.q, rq.spec.omega, rq.spec.seed, rq.spec.realization,
                                pool.init(i, rq.spec.q, rq.spec.length))
                               for i, rq in enumerate(reqs)])
    out["serving_requests"] = {"node_updates_per_s": rate, "cores": threads,
                               "sample": f"{k} runs of 20 steps over {len(reqs)} requests of the "
                                         f"stream ({el:.1f} s)"}
    return out


def bench_probes(ilg, stream, warmup: int, launches: int = 200):
    """The two costs of the headline step apart, in its launch shape: the
    streaming-only probe (the step's memory traffic, no collision) at 2^24 and
    2^26 nodes, and the draws-only probe (two Philox4x32 blocks per node, 10
    and 7 rounds) at 2^24 nodes."""
    import torch
    out = {"workload": "D1Q3 uint16 step pattern, one launch per step; draws: 2 Philox "
                       "blocks per node (counter (x, t, 0, b)), xor-folded to 4 B per node",
           "launches": launches}
    # ~0.25 s of streaming launches first, untimed, so that the clock has
    # ramped up before any timed launch
    L = 1 << 24
    pitch = (L + 63) // 64 * 64
    a = torch.zeros(3 * pitch, dtype=torch.int16, device="cuda")
    b = torch.zeros_like(a)
    t_end = time.perf_counter() + 0.25
    while time.perf_counter() < t_end:
        for _ in range(100):
            ilg.probe_stream(3, L, a, b, stream)
        torch.cuda.synchronize()
    del a, b
    for L in (1 << 24, 1 << 26):
        pitch = (L + 63) // 64 * 64
        a = torch.zeros(3 * pitch, dtype=torch.int16, device="cuda")
        b = torch.zeros_like(a)
        for _ in range(warmup):
            ilg.probe_stream(3, L, a, b, stream)
        sec = timed(stream, lambda: [ilg.probe_stream(3, L, a, b, stream)
                                     for _ in range(launches)])
        ms = sec * 1e3 / launches
        gbs = 12 * L / (ms / 1e3) / 1e9
        out[f"stream_only_l2p{L.bit_length() - 1}"] = {
            "ms_per_launch": ms, "alg_gbs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
            "node_updates_per_s": L / (ms / 1e3)}
        del a, b
    L = 1 << 24
    o = torch.zeros(L, dtype=torch.int32, device="cuda")
    for rounds in (10, 7):
        for _ in range(warmup):
            ilg.probe_philox(L, 2, o, rounds=rounds, stream=stream)
        sec = timed(stream, lambda: [ilg.probe_philox(L, 2, o, rounds=rounds, t=k, stream=stream)
                                     for k in range(launches)])
        ms = sec * 1e3 / launches
        out[f"draws_only_{rounds}_rounds"] = {
            "ms_per_launch": ms, "philox_blocks_per_s": 2 * L / (ms / 1e3),
            "node_updates_per_s_bound": L / (ms / 1e3),
            "hbm_frac_bound": 12 * L / (ms / 1e3) / 1e9 / HBM_PEAK_GBS}
    return out


def bench_plain_mall_free(ilg, W, stream, warmup: int, steps: int = 500):
    """The headline kernel on a lattice whose double-buffered state (768 MiB)
    does not fit the 256 MB MALL, so every step really streams from HBM."""
    spec, init = W.workload_d1q3_big(length=MALL_FREE_LENGTH, steps=steps)
    lat = ilg.Lattice(spec.q, spec.length, spec.count_bytes, spec.omega, spec.seed, init)
    lat.step(warmup)
    sec = timed(stream, lambda: lat.step(steps))
    lat.close()
    ms = sec * 1e3 / steps
    alg_bytes = 2 * spec.q * spec.count_bytes * spec.length
    return {"workload": "same step, D1Q3 L=2^26 periodic, uint16, Poisson(50), omega=1.8",
            "steps": steps, "ms_per_step": ms, "node_updates_per_s": spec.length / (ms / 1e3),
            "alg_gbs": alg_bytes / (ms / 1e3) / 1e9,
            "traffic": counter_traffic(spec.length)}


def bench_philox7(ilg, W, stream, warmup: int, steps: int = 1000):
    """Draw specification v2 (7-round Philox) on the headline lattice: the
    same step with a different, equally valid random stream."""
    spec, init = W.workload_d1q3_big(steps=steps)
    lat = ilg.Lattice(spec.q, spec.length, spec.count_bytes, spec.omega, spec.seed, init,
                      rounds=7)
    mass0 = int(init.astype(np.int64).sum())
    lat.step(warmup)
    sec = timed(stream, lambda: lat.step(steps))
    if lat.moments()["mass"] != mass0:
        raise SystemExit("Philox-7: mass not conserved")
    lat.close()
    ms = sec * 1e3 / steps
    alg_bytes = 2 * spec.q * spec.count_bytes * spec.length
    return {"workload": "same step with 7-round Philox draws (draw specification v2), D1Q3 "
                        "L=2^24 periodic, uint16, Poisson(50), omega=1.8",
            "steps": steps, "ms_per_step": ms, "node_updates_per_s": spec.length / (ms / 1e3),
            "alg_gbs": alg_bytes / (ms / 1e3) / 1e9}


def bench_dense(ilg, W, stream, warmup: int, steps: int = 500):
    """A dense D1Q3 lattice whose moving populations exceed one 64-trial
    chunk: L = 2^24, uint16, Poisson(90) per velocity, theta = 2/3 (equal
    weights, so every count stays near 90), omega = 1.8."""
    L = 1 << 24
    init = W.init_poisson_iid(3, L, 90.0, 2, init_seed=8)
    lat = ilg.Lattice(3, L, 2, 1.8, 4, init, theta=2.0 / 3.0)
    mass0 = int(init.astype(np.int64).sum())
    lat.step(warmup)
    sec = timed(stream, lambda: lat.step(steps))
    if lat.moments()["mass"] != mass0:
        raise SystemExit("dense D1Q3: mass not conserved")
    lat.close()
    ms = sec * 1e3 / steps
    return {"workload": "D1Q3 with flip, L=2^24 periodic, uint16, Poisson(90) per velocity, "
                        "theta=2/3, omega=1.8",
            "steps": steps, "ms_per_step": ms, "node_updates_per_s": L / (ms / 1e3),
            "alg_gbs": 12 * L / (ms / 1e3) / 1e9}


def bench_exchange(ilg, W, stream, warmup: int, steps: int = 1000):
    """D1Q2, L = 2^24, uint16, Poisson(40), omega = 1.5: the three-binomial
    collision against the exchange form (draw specification v3, two
    crossing binomials per node)."""
    L = 1 << 24
    init = W.init_poisson_iid(2, L, 40.0, 2, init_seed=7)
    mass0 = int(init.astype(np.int64).sum())
    out = {"workload": "D1Q2 with flip, L=2^24 periodic, uint16, Poisson(40), omega=1.5",
           "steps": steps}
    for name, ex in (("three_binomials", False), ("exchange", True)):
        lat = ilg.Lattice(2, L, 2, 1.5, 1, init, exchange=ex)
        lat.step(warmup)
        sec = timed(stream, lambda: lat.step(steps))
        if lat.moments()["mass"] != mass0:
            raise SystemExit("D1Q2: mass not conserved")
        lat.close()
        ms = sec * 1e3 / steps
        out[name] = {"ms_per_step": ms, "node_updates_per_s": L / (ms / 1e3),
                     "alg_gbs": 2 * 2 * 2 * L / (ms / 1e3) / 1e9}
    return out


def bench_d2q5(ilg, stream, warmup: int, steps: int = 500):
    """The D2Q5 extension: 4096 x 4096 periodic nodes, uint16, Poisson
    occupations drawn on the device (means 25, 25, 50, 25, 25), omega = 1.8."""
    lx = ly = 4096
    lat = ilg.Lattice(5, lx, 2, 1.8, 1, None, height=ly)
    lat.init_poisson_sine(150.0, 0.0, 2)
    mass0 = lat.moments()["mass"]
    lat.step(warmup)
    sec = timed(stream, lambda: lat.step(steps))
    if lat.moments()["mass"] != mass0:
        raise SystemExit("D2Q5: mass not conserved")
    lat.close()
    ms = sec * 1e3 / steps
    nodes = lx * ly
    alg_bytes = 2 * 5 * 2 * nodes
    return {"workload": "D2Q5 with flip, 4096 x 4096 periodic, uint16, Poisson means "
                        "(25, 25, 50, 25, 25) drawn on the device, omega=1.8",
            "steps": steps, "ms_per_step": ms, "node_updates_per_s": nodes / (ms / 1e3),
            "alg_bytes_per_node_update": 20, "alg_gbs": alg_bytes / (ms / 1e3) / 1e9,
            "hbm_frac": alg_bytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS}


def bench_batched_ragged(ilg, W, stream, steps: int, loop_members: int):
    ens = W.ensemble_ragged_d1q2(steps=steps)
    members = [dict(q=s.q, length=s.length, count_bytes=s.count_bytes, omega=s.omega,
                    seed=s.seed, realization=s.realization) for s in ens.specs]
    b = ilg.Batch(members, ens.inits, sk_every=10, nk=16)
    shape = b.tune(40)
    sec = timed(stream, lambda: b.run(steps))
    nu = ens.total_nodes * steps
    b.close()
    # plain form, one member after another, on an evenly spaced sample by length
    lens = np.array([s.length for s in ens.specs])
    order = np.argsort(-lens, kind="stable")
    pick = order[np.linspace(0, len(order) - 1, loop_members).astype(int)]
    lats = [ilg.Lattice(s.q, s.length, s.count_bytes, s.omega, s.seed, ens.inits[r],
                        realization=s.realization) for r, s in ((r, ens.specs[r]) for r in pick)]

    def loop():
        for lat in lats:
            lat.step(steps)

    sec_loop = timed(stream, loop)
    nu_loop = int(lens[pick].sum()) * steps
    for lat in lats:
        lat.close()
    rate, rate_loop = nu / sec, nu_loop / sec_loop
    return {
        "workload": f"4096 independent D1Q2 lattices, L log-uniform in [64, 8192] "
                    f"(sum {ens.total_nodes}), omega ~ U[1, 1.95], own seeds, uint16, "
                    f"Poisson(30), {steps} steps, S(k) k=1..16 every 10 steps",
        "node_updates_per_s": rate, "seconds": sec, "node_updates": nu, "shape": shape,
        "plain_loop": {"node_updates_per_s": rate_loop, "seconds": sec_loop,
                       "members": int(loop_members), "node_updates": nu_loop,
                       "note": "same members one after another through the plain API "
                               "(no diagnostics), evenly spaced by length"},
        "batched_over_plain_loop": rate / rate_loop,
    }


def bench_batched_specs(ilg, W, stream, steps: int):
    """The ragged D1Q2 ensemble (with its S(k) sampling) under draw
    specifications v2 (7-round draws) and v3 (the exchange form), each with
    its own autotuned shape."""
    ens = W.ensemble_ragged_d1q2(steps=steps)
    nu = ens.total_nodes * steps
    out = {}
    for key, rounds, exchange in (("v2_philox7", 7, False), ("v3_exchange", 10, True)):
        members = [dict(q=s.q, length=s.length, count_bytes=s.count_bytes, omega=s.omega,
                        seed=s.seed, realization=s.realization, rounds=rounds,
                        exchange=exchange) for s in ens.specs]
        b = ilg.Batch(members, ens.inits, sk_every=10, nk=16)
        shape = b.tune(40)
        sec = timed(stream, lambda: b.run(steps))
        b.close()
        out[key] = {"node_updates_per_s": nu / sec, "seconds": sec, "shape": shape}
    out["workload"] = ("the batched ragged ensemble's members and S(k) sampling, "
                       f"{steps} steps, under draw specifications v2 and v3")
    return out


def bench_batched_d2q5(ilg, stream, steps: int = 2000, n: int = 2048, side: int = 64):
    """An ensemble of small D2Q5 lattices: n members of side x side nodes,
    uint16, Poisson means (25, 25, 50, 25, 25), omega ~ U[1, 1.95], own seeds."""
    rng = np.random.default_rng(12)
    means = np.array([25.0, 25.0, 50.0, 25.0, 25.0])[:, None, None]
    members, inits = [], []
    for r in range(n):
        members.append(dict(q=5, length=side, height=side, count_bytes=2,
                            omega=float(rng.uniform(1.0, 1.95)), seed=20_000 + r, realization=r))
        inits.append(rng.poisson(means, size=(5, side, side)).astype(np.uint16))
    b = ilg.Batch(members, inits)
    shape = b.tune(20)
    sec = timed(stream, lambda: b.run(steps))
    b.close()
    nu = n * side * side * steps
    # The cost of a node grows steeply with the collision fraction omega*
    # (more than 64 collided particles take the chunked redistribution), so
    # the plain form is timed at the same rates: one 1024 x 1024 lattice at
    # each of 16 evenly spaced quantiles of the members' omega, 100 steps.
    oms = np.sort([m["omega"] for m in members])
    tot, work, side_p = 0.0, 0, 1024
    per_omega = []
    for q in np.linspace(0, len(oms) - 1, 16).astype(int):
        init = rng.poisson(means, size=(5, side_p, side_p)).astype(np.uint16)
        lat = ilg.Lattice(5, side_p, 2, float(oms[q]), 7, init, height=side_p)
        lat.step(10)
        sec_q = timed(stream, lambda: lat.step(100))
        tot += sec_q
        work += side_p * side_p * 100
        per_omega.append([round(float(oms[q]), 4), side_p * side_p * 100 / sec_q])
        lat.close()
    plain = work / tot
    return {"workload": f"{n} D2Q5 lattices of {side} x {side}, uint16, Poisson means "
                        f"(25, 25, 50, 25, 25), omega ~ U[1, 1.95], own seeds, {steps} steps",
            "node_updates_per_s": nu / sec, "seconds": sec, "node_updates": nu, "shape": shape,
            "plain_same_rates": {"node_updates_per_s": plain, "lattices": 16,
                                 "side": side_p, "steps": 100,
                                 "omega_and_node_updates_per_s": per_omega},
            "batched_over_plain_same_rates": (nu / sec) / plain}


def bench_batched_decay(ilg, W, stream, steps: int):
    ens = W.ensemble_decay_sweep(steps=steps)
    members = [dict(q=s.q, length=s.length, count_bytes=s.count_bytes, omega=s.omega,
                    seed=s.seed, realization=s.realization) for s in ens.specs]
    b = ilg.Batch(members, ens.inits, amp_every=100, max_amp=steps // 100 + 1)
    shape = b.tune(40)
    sec = timed(stream, lambda: b.run(steps))
    b.close()
    nu = ens.total_nodes * steps
    return {"workload": f"6 omega x 1024 D1Q3 lattices, L=4096, uint32, Poisson sine init "
                        f"(100 + 40 sin), {steps} steps, A^LG every 100 steps",
            "node_updates_per_s": nu / sec, "seconds": sec, "node_updates": nu, "shape": shape}


def bench_serving_saturated(ilg, W, stream, steps: int = 1000, nreq: int = 64):
    """Serving capacity: nreq requests of 2^20 nodes submitted at once (the
    first nreq requests of the stream's rates and seeds), all D1Q2, all D1Q3,
    then mixed, against plain 2^22-node lattices stepped at each of the same
    rates (the comparison the server's per-tile overhead is read from).  Each
    server run is timed end to end (admission with its host-to-device copies,
    the quanta, and the results copied back), at `steps` and at 3 x `steps`
    steps; the difference of the two is the marginal rate of the quanta
    alone, which is what the plain lattices' rate compares with."""
    import torch
    base = W.request_stream(rate_per_s=200, duration_s=2.0)[:nreq]
    pool = W.RequestInitPool()
    out = {"workload": f"{nreq} requests of 2^20 nodes, uint16, Poisson(40), omega ~ U[1, 1.95], "
                       f"{steps} steps each (and {3 * steps} for the marginal rate), submitted "
                       f"at once; plain: one lattice of 2^22 at each of the same rates"}

    def run(qfun, nsteps):
        srv = ilg.Server(16 << 30, 100)
        for i, rq in enumerate(base):
            q = qfun(rq)
            m = dict(q=q, length=1 << 20, count_bytes=2, omega=rq.spec.omega, seed=rq.spec.seed,
                     realization=rq.spec.realization)
            srv.submit(m, pool.init(i, q, m["length"]), nsteps)
        t0 = time.perf_counter()
        while True:
            st = srv.poll()
            if st["active"] == 0 and st["queued"] == 0:
                break
        sec = time.perf_counter() - t0
        srv.close()
        return sec

    for label, qfun in (("d1q2", lambda rq: 2), ("d1q3", lambda rq: 3),
                        ("mixed", lambda rq: rq.spec.q)):
        sec = run(qfun, steps)
        sec3 = run(qfun, 3 * steps)
        nu = len(base) * (1 << 20) * steps
        out[label] = {"node_updates_per_s": nu / sec, "seconds": sec,
                      "marginal_node_updates_per_s": 2 * nu / (sec3 - sec),
                      "seconds_3x": sec3}
    # The plain form at every one of the same rates (the work per node
    # depends strongly on the collision fraction), one 2^22-node lattice per
    # rate, 100 timed steps each.
    for q in (2, 3):
        tot, work, L = 0.0, 0, 1 << 22
        init = W.init_poisson_iid(q, L, 40.0, 2, init_seed=5)
        for i, rq in enumerate(base):
            lat = ilg.Lattice(q, L, 2, rq.spec.omega, rq.spec.seed, init)
            lat.step(10)
            tot += timed(stream, lambda: lat.step(100))
            work += L * 100
            lat.close()
        out[f"plain_d1q{q}_same_rates"] = {"node_updates_per_s": work / tot,
                                           "lattices": len(base), "length": L, "steps": 100}
        out[f"serving_over_plain_d1q{q}"] = (out[f"d1q{q}"]["marginal_node_updates_per_s"] /
                                             out[f"plain_d1q{q}_same_rates"]["node_updates_per_s"])
    return out


def bench_serving(ilg, W, rate: float, duration: float, budget: int, quantum: int,
                  step_nodes: int = 0):
    """Replay a Poisson request stream in real time through the server: each
    request is submitted once its arrival time has passed, every loop iteration
    polls once (admit, one quantum of shared launches, retire).  Latency is
    completion minus arrival."""
    reqs = W.request_stream(rate_per_s=rate, duration_s=duration)
    pool = W.RequestInitPool()
    srv = ilg.Server(budget, quantum, step_nodes=step_nodes)
    clock = ilg.Server.clock
    t0 = clock()
    i = 0
    pending = {}
    lat, work = [], 0
    polls = 0
    peak = 0
    while i < len(reqs) or pending:
        now = clock() - t0
        while i < len(reqs) and reqs[i].arrival_s <= now:
            rq = reqs[i]
            m = dict(q=rq.spec.q, length=rq.spec.length, count_bytes=2, omega=rq.spec.omega,
                     seed=rq.spec.seed, realization=rq.spec.realization)
            rid = srv.submit(m, pool.init(i, m["q"], m["length"]), rq.spec.steps)
            pending[rid] = (t0 + rq.arrival_s, rq.spec.length * rq.spec.steps)
            i += 1
        st = srv.poll()
        polls += 1
        peak = max(peak, st["bytes_peak"])
        if st["finished"]:
            for rid in list(pending):
                info = srv.info(rid)
                if info["state"] == "done":
                    arr, nu = pending.pop(rid)
                    lat.append(info["t_done"] - arr)
                    work += nu
                    srv.result(rid)
        if not pending and i < len(reqs):
            wait = t0 + reqs[i].arrival_s - clock()
            if wait > 0:
                time.sleep(wait)
    t_end = clock()
    srv.close()
    lat = np.array(lat)
    return {"rate_per_s": rate, "requests": len(reqs), "duration_s": duration,
            "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_latency_s": float(lat.mean()),
            "node_updates_per_s": work / (t_end - t0), "wall_s": t_end - t0, "polls": polls,
            "peak_bytes": int(peak), "budget_bytes": budget, "quantum_steps": quantum}


def summarize_counters(fetch_csv: str, write_csv: str, length: int):
    """Turn two rocprofv3 --pmc runs of `bench.py --forms plain --copy-probe`
    (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch) into HBM bytes per step
    launch.  Each counter is scaled by what it reads for the probe copy of
    768 MiB (the largest copy dispatch), so the record is in true bytes."""
    import csv

    def per_kernel(path, counter):
        rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
        step = [float(r["Counter_Value"]) for r in rows if "step_kernel" in r["Kernel_Name"]]
        copies = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]
                  or "copy" in r["Kernel_Name"].lower()]
        return float(np.mean(step)), max(copies)

    probe_kib = (768 << 20) / 1024.0
    f_step, f_copy = per_kernel(fetch_csv, "FETCH_SIZE")
    w_step, w_copy = per_kernel(write_csv, "WRITE_SIZE")
    f_scale, w_scale = probe_kib / f_copy, probe_kib / w_copy
    rec = {"step_source_sha256_16": step_source_digest(),
           "fetch_kib_raw": f_step, "write_kib_raw": w_step,
           "copy_probe_fetch_kib_raw": f_copy, "copy_probe_write_kib_raw": w_copy,
           "fetch_scale": f_scale, "write_scale": w_scale,
           "fetch_bytes_per_launch": f_step * f_scale * 1024,
           "write_bytes_per_launch": w_step * w_scale * 1024,
           "bytes_per_launch": (f_step * f_scale + w_step * w_scale) * 1024,
           "length": length, "alg_bytes_per_launch": 12 * length}
    with open(traffic_file(length), "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


def summarize_sq(csv_path: str, length: int, skip: int):
    """Turn a rocprofv3 --pmc run of the SQ counters (SQ_INSTS_VALU,
    SQ_INSTS_SALU, SQ_INSTS_LDS, SQ_LDS_BANK_CONFLICT, SQ_WAVE_CYCLES,
    SQ_WAIT_ANY, SQ_WAIT_INST_ANY, SQ_ACTIVE_INST_ANY) of `bench.py --forms
    plain` into a per-launch record of the step kernel (dispatches after the
    first `skip`, when the state has relaxed), kept with the kernel digest."""
    import csv
    vals = {}
    for r in csv.DictReader(open(csv_path)):
        if "step_kernel" not in r["Kernel_Name"]:
            continue
        vals.setdefault(r["Counter_Name"], {})[int(r["Dispatch_Id"])] = float(r["Counter_Value"])
    rec = {"step_source_sha256_16": step_source_digest(), "length": length, "skipped": skip}
    for name, per in vals.items():
        ids = sorted(per)[skip:]
        rec[name.lower() + "_per_launch"] = float(np.mean([per[i] for i in ids]))
        rec["dispatches"] = len(ids)
    rec["valu_wave_insts_per_launch"] = rec.get("sq_insts_valu_per_launch")
    with open(SQ_FILE, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--length", type=int, default=1 << 24)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="plain,probes,mallfree,philox7,dense,exchange,d2q5,batched,batched_specs,batched_d2q5,decay,serving_saturated,serving",
                    help="comma list of plain (always), probes, mallfree, philox7, exchange, "
                         "d2q5, batched, batched_specs, batched_d2q5, decay, serving_saturated, "
                         "serving")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-step-nodes", type=int, default=0,
                    help="server policy: at most this many nodes advanced per quantum, least "
                         "remaining work first (0: every active request)")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-budget-gib", type=float, default=16.0)
    ap.add_argument("--serve-quantum", type=int, default=100)
    ap.add_argument("--batched-steps", type=int, default=5000)
    ap.add_argument("--decay-steps", type=int, default=10000)
    ap.add_argument("--loop-members", type=int, default=32)
    ap.add_argument("--copy-probe", action="store_true",
                    help="after timing, one plain device copy of 768 MiB (counter scale)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the counter traffic record from two rocprofv3 --pmc runs and exit")
    ap.add_argument("--summarize-sq", metavar="SQ_CSV",
                    help="write the SQ counter record of the step kernel from a rocprofv3 --pmc "
                         "run and exit")
    ap.add_argument("--sq-skip", type=int, default=100,
                    help="with --summarize-sq: step dispatches to leave out at the start")
    args = ap.parse_args()
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters, args.length)
        return
    if args.summarize_sq:
        summarize_sq(args.summarize_sq, args.length, args.sq_skip)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(ensembles would shard by realization, one lattice along x).", file=sys.stderr)
        sys.exit(2)
    forms = set(args.forms.split(","))

    import torch

    import ilg_workloads as W
    import paper_2203_01380_amd as ilg

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    spec, init = W.workload_d1q3_big(length=args.length, steps=args.steps)
    mass0 = int(init.astype(np.int64).sum())
    lat = ilg.Lattice(spec.q, spec.length, spec.count_bytes, spec.omega, spec.seed, init)
    # The probes run between the upload of the headline lattice and its
    # warm-up steps, back to back: after host-side set-up the GPU clock ramps
    # up over tens of launches (2.3 -> 2.5 GHz, profiles/
    # step_d1q3_u16_l2p24_clock_ramp.md), so the timed steps follow
    # continuous GPU work as they would in a long run.  Without the probes
    # form the timed steps follow the upload directly.
    probes = None
    if "probes" in forms:
        say("probes: streaming only, draws only")
        probes = bench_probes(ilg, stream, args.warmup)
    say(f"warmup {args.warmup} steps")
    lat.step(args.warmup)
    say(f"timing {args.steps} steps")
    sec = timed(stream, lambda: lat.step(args.steps))
    if lat.moments()["mass"] != mass0:
        raise SystemExit("mass not conserved")
    lat.close()
    if args.copy_probe:
        a = torch.empty(768 << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    ms_per_step = sec * 1e3 / args.steps       # one step kernel launch per step
    value = spec.length * args.steps / sec
    alg_bytes = 2 * spec.q * spec.count_bytes * spec.length   # per launch
    assert alg_bytes == ALG_BYTES_PER_NODE_UPDATE * spec.length
    gbs = alg_bytes / (ms_per_step / 1e3) / 1e9
    out = {
        "metric": "node-updates/s",
        "value": value,
        "unit": "node-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16",
        "data": "synthetic",
        "config": {"workload": f"1D diffusive ILG with flip, D1Q3, L=2^{spec.length.bit_length() - 1} "
                               "periodic, uint16 counts, Poisson(50) per velocity, omega=1.8, "
                               "Philox seed 1",
                   "q": spec.q, "length": spec.length, "count_bytes": spec.count_bytes,
                   "omega": spec.omega, "form": "plain"},
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "traffic": counter_traffic(spec.length),
                     "alg_bytes_per_node_update": ALG_BYTES_PER_NODE_UPDATE,
                     "traffic_source": (os.path.relpath(traffic_file(spec.length), ROOT)
                                        + " (step sources digest " + step_source_digest() + ")"),
                     "limiter": "integer VALU (alu_roofline; probes)"},
        "alu_roofline": alu_roofline(ms_per_step, spec.length),
    }
    if "probes" in forms:
        out["probes"] = probes
    if "mallfree" in forms and spec.length != MALL_FREE_LENGTH:
        say("plain step at 2^26 nodes")
        out["plain_l2p26"] = bench_plain_mall_free(ilg, W, stream, args.warmup)
    if "philox7" in forms:
        say("plain step with 7-round draws")
        out["philox7"] = bench_philox7(ilg, W, stream, args.warmup)
    if "dense" in forms:
        say("dense D1Q3 lattice")
        out["d1q3_dense"] = bench_dense(ilg, W, stream, args.warmup)
    if "exchange" in forms:
        say("D1Q2: three binomials against the exchange form")
        out["d1q2_exchange"] = bench_exchange(ilg, W, stream, args.warmup)
    if "d2q5" in forms:
        say("D2Q5 4096 x 4096")
        out["d2q5"] = bench_d2q5(ilg, stream, args.warmup)
    if "batched" in forms:
        say("batched ragged ensemble")
        out["batched"] = bench_batched_ragged(ilg, W, stream, args.batched_steps,
                                              args.loop_members)
    if "batched_specs" in forms:
        say("batched ragged ensemble under draw specifications v2 and v3")
        out["batched_specs"] = bench_batched_specs(ilg, W, stream, args.batched_steps)
    if "batched_d2q5" in forms:
        say("batched D2Q5 ensemble")
        out["batched_d2q5"] = bench_batched_d2q5(ilg, stream)
    if "decay" in forms:
        say("batched decay sweep")
        out["batched_decay"] = bench_batched_decay(ilg, W, stream, args.decay_steps)
    if "serving_saturated" in forms:
        say("serving capacity: 64 requests of 2^20 nodes at once")
        out["serving_saturated"] = bench_serving_saturated(ilg, W, stream)
    if "serving" in forms:
        out["serving"] = []
        for frac in (1.0, 0.5, 0.25):
            say(f"serving at {frac:g} x {args.serve_rate:g} req/s for {args.serve_seconds:g} s")
            out["serving"].append(bench_serving(ilg, W, args.serve_rate * frac, args.serve_seconds,
                                                int(args.serve_budget_gib * (1 << 30)),
                                                args.serve_quantum, args.serve_step_nodes))
    if not args.no_cpu_baseline:
        say(f"cpu baseline (~{args.cpu_seconds:.0f} s)")
        out["cpu_baseline"] = cpu_baseline(init, spec, args.cpu_seconds)
        say("cpu baseline on the other workloads")
        out["cpu_baseline"]["other_workloads"] = cpu_other_configs(W, args.cpu_seconds / 4)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
