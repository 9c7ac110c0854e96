"""Benchmark of the fused lattice-gas step (flip -> sampling collision -> stream).

Workload: D1Q3, L = 2^24 periodic nodes, uint16 counts, Poisson(50) i.i.d.
initial state, omega = 1.8 (flip on, omega* = 0.2), Philox seed 1.  A "step"
is one full lattice time step; the state is resident in HBM before timing.
Prints one JSON line: node-updates/s, the HBM roofline of the step kernel
(algorithmic 12 bytes per node-update: 3 uint16 counts read and written), and
the CPU oracle timed on a bounded sample on the host cores.
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_step_d1q3_u16_l2p24.json")
STEP_SOURCE = os.path.join(ROOT, "paper_2203_01380_amd", "csrc", "step.hip")


def step_source_digest() -> str:
    with open(STEP_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def counter_traffic():
    """HBM bytes per launch from the committed PMC summary, or None if absent or
    taken on a different version of the step kernel."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("step_source_sha256_16") != step_source_digest():
        return None
    return rec.get("bytes_per_launch")


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--length", type=int, default=1 << 24)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after timing, run one plain device copy of 768 MiB (counter scale)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(ensembles and lattices would shard by realization or along x).", file=sys.stderr)
        sys.exit(2)

    import torch

    import ilg_workloads as W
    import paper_2203_01380_amd as ilg

    torch.cuda.set_device(0)
    spec, init = W.workload_d1q3_big(length=args.length, steps=args.steps)
    mass0 = int(init.astype(np.int64).sum())
    lat = ilg.Lattice(spec.q, spec.length, spec.count_bytes, spec.omega, spec.seed, init)
    stream = torch.cuda.current_stream()

    print(f"# warmup {args.warmup} steps", file=sys.stderr, flush=True)
    lat.step(args.warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    print(f"# timing {args.steps} steps", file=sys.stderr, flush=True)
    ev0.record(stream)
    lat.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    mass1 = lat.moments()["mass"]
    if mass1 != mass0:
        raise SystemExit(f"mass not conserved: {mass0} -> {mass1}")

    if args.copy_probe:
        a = torch.empty(768 << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    sec = ms / 1e3
    ms_per_step = ms / args.steps
    value = spec.length * args.steps / sec
    alg_bytes = 2 * spec.q * spec.count_bytes * spec.length   # per launch
    achieved = alg_bytes / (ms_per_step / 1e3) / 1e9
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
        "config": {"workload": "1D diffusive ILG with flip, D1Q3, L=2^24 periodic, uint16 counts, "
                               "Poisson(50) per velocity, omega=1.8, Philox seed 1",
                   "q": spec.q, "length": spec.length, "count_bytes": spec.count_bytes,
                   "omega": spec.omega, "form": "plain"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": counter_traffic()},
    }
    if not args.no_cpu_baseline:
        print(f"# cpu baseline (~{args.cpu_seconds:.0f} s)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(init, spec, args.cpu_seconds)
    lat.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
