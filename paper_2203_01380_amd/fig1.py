"""Amplitude-decay sweep of the paper's Fig. 1 (Results section).

D1Q3, L = 320 periodic nodes, N^ave = 100, sine profile with amplitude
A_0 = N^ave, occupations drawn as Poisson variates on the device
(ilg_init_poisson_sine), several realizations per omega^j; the no-flip
operator for omega^j <= 1 and the flip for omega^j > 1 (chosen by the
library from omega^j).  Every realization runs in one batched launch per
omega^j, recording A^LG(t) = sum_x sin(2 pi x / L) N(x) / sum_x sin^2(2 pi x / L)
on the device every `every` steps.  The mean over realizations is compared
with A^th(t) = N^ave exp(-4 pi^2 D t / L^2), D = theta (1/omega^j - 1/2)
(Eq. ampdecay).

    python -m paper_2203_01380_amd.fig1 --out fig1.tsv

writes one row per recorded time: t, then for each omega^j the mean A^LG, its
standard error and A^th.
"""
from __future__ import annotations

import argparse
import math
import sys
from typing import Dict, Sequence

import numpy as np

DEFAULT_OMEGAS = (0.5, 0.75, 1.0, 1.25, 1.5, 1.75, 1.9, 2.0)


def amplitude(n: np.ndarray) -> float:
    """A^LG of one state [q][L] (host)."""
    L = n.shape[-1]
    s = np.sin(2.0 * math.pi * np.arange(L) / L)
    return float(np.dot(s, n.astype(np.float64).sum(axis=0)) / np.dot(s, s))


def theory(t, omega_j: float, nave: float, length: int, theta: float = 1.0 / 3.0):
    D = theta * (1.0 / omega_j - 0.5)
    return nave * np.exp(-4.0 * math.pi ** 2 * D * np.asarray(t, dtype=np.float64) / length ** 2)


def run_sweep(omegas: Sequence[float] = DEFAULT_OMEGAS, nreal: int = 500, length: int = 320,
              nave: float = 100.0, amp: float | None = None, steps: int = 40000,
              every: int = 200, seed: int = 1, count_bytes: int = 2) -> Dict:
    """Run the sweep; returns times, and per omega^j the mean A^LG(t), its
    standard error and A^th(t)."""
    from . import Batch, Lattice
    amp = nave if amp is None else amp
    nrec = steps // every
    t = np.arange(nrec + 1) * every
    out = {"t": t, "omegas": list(omegas), "mean": {}, "sem": {}, "theory": {}}
    for oi, om in enumerate(omegas):
        members, inits = [], []
        # initial states drawn on the device, one init seed per realization
        lat = Lattice(3, length, count_bytes, float(om), 1, None)
        for r in range(nreal):
            lat.init_poisson_sine(nave, amp, (seed << 40) + (oi << 20) + r)
            inits.append(lat.state())
            members.append(dict(q=3, length=length, count_bytes=count_bytes, omega=float(om),
                                seed=(seed << 20) + oi * nreal + r, realization=r))
        lat.close()
        b = Batch(members, inits, amp_every=every, max_amp=nrec)
        b.run(steps)
        series, cnt = b.amplitudes()
        b.close()
        if not (cnt == nrec).all():
            raise RuntimeError("amplitude series incomplete")
        a = np.empty((nreal, nrec + 1))
        a[:, 0] = [amplitude(x) for x in inits]
        a[:, 1:] = series
        out["mean"][om] = a.mean(axis=0)
        out["sem"][om] = a.std(axis=0, ddof=1) / math.sqrt(nreal)
        out["theory"][om] = theory(t, om, nave, length)
    return out


def write_table(res: Dict, path: str):
    with open(path, "w") as f:
        cols = ["t"]
        for om in res["omegas"]:
            cols += [f"A_mean(w={om:g})", f"A_sem(w={om:g})", f"A_th(w={om:g})"]
        f.write("\t".join(cols) + "\n")
        for i, t in enumerate(res["t"]):
            row = [str(int(t))]
            for om in res["omegas"]:
                row += [f"{res['mean'][om][i]:.4f}", f"{res['sem'][om][i]:.4f}",
                        f"{res['theory'][om][i]:.4f}"]
            f.write("\t".join(row) + "\n")


def summary(res: Dict) -> Dict:
    """Per omega^j: the largest |mean - theory| in standard errors, and the
    amplitude at the last time (measured, theory)."""
    out = {}
    for om in res["omegas"]:
        z = np.abs(res["mean"][om] - res["theory"][om]) / np.maximum(res["sem"][om], 1e-12)
        out[om] = {"max_z": float(z.max()), "A_end": float(res["mean"][om][-1]),
                   "A_th_end": float(res["theory"][om][-1])}
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", default="fig1.tsv")
    ap.add_argument("--nreal", type=int, default=500)
    ap.add_argument("--steps", type=int, default=40000)
    ap.add_argument("--every", type=int, default=200)
    ap.add_argument("--omegas", default=",".join(f"{o:g}" for o in DEFAULT_OMEGAS))
    args = ap.parse_args(argv)
    omegas = [float(o) for o in args.omegas.split(",")]
    res = run_sweep(omegas, nreal=args.nreal, steps=args.steps, every=args.every)
    write_table(res, args.out)
    for om, s in summary(res).items():
        print(f"omega^j={om:g}: max |mean - A_th| = {s['max_z']:.2f} standard errors; "
              f"A({res['t'][-1]}) = {s['A_end']:.3f} (theory {s['A_th_end']:.3f})", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
