"""Convergence-error sweep on the GPU: error of an order-p composed method at time T
as a function of the step, against the same-scheme order-8 Suzuki run with a step
eight times smaller (the paper measures |psi_dt(t) - psi_dt/2(t)|, Sec. III; here the
reference is order 8 at dt/8), in the grid L2 norm and in the phase at the
wavefunction's peak (Sec. III, Fig. 5).

All runs of one scheme go into one batched launch with a per-item step: the
dt_k = dt0 * 2^-k run and its reference at dt_k / 8 = dt_(k+3) are items of the same
batch.  Long sweeps are issued in chunks of steps so progress can be printed.

    python -m paper_1902_04661_amd.convergence --n 2048 --T 4000 --kmax 3
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time
from typing import Dict, List

import numpy as np
import torch

from . import gqd, inputs


def grid_norm(dq: float, a: np.ndarray) -> float:
    return math.sqrt(dq * float(np.sum(np.abs(a) ** 2)))


def phase_at_peak(psi: np.ndarray) -> float:
    """arg psi at the grid point of largest amplitude (Sec. III's phase measure).  For a
    two-surface state the peak is taken over surfaces and points together, the first in
    memory order on ties."""
    flat = np.asarray(psi).reshape(-1)
    return float(np.angle(flat[int(np.argmax(np.abs(flat)))]))


def phase_error(psi: np.ndarray, ref: np.ndarray) -> float:
    """|phi - phi_ref| with phi = phase_at_peak of each state (each at its own peak, as
    the paper defines it), folded into [0, pi]."""
    d = phase_at_peak(psi) - phase_at_peak(ref)
    return abs(math.remainder(d, 2.0 * math.pi))


def run_batch(item, scheme: str, order: int, dts: List[float], T: float, opts: gqd.SolverOpts,
              chunk: int = 64, log=print) -> Dict[float, np.ndarray]:
    """Propagate copies of `item` to time T, copy b with step dts[b]; return the states."""
    items = [item] * len(dts)
    prop = gqd.from_items(items)
    psi = prop.pack([item.psi0] * len(dts))
    nsteps = np.array([int(round(T / dt)) for dt in dts], dtype=np.int64)
    for dt, ns in zip(dts, nsteps):
        if abs(ns * dt - T) > 1e-9 * T:
            raise ValueError(f"T = {T} is not a whole number of steps of {dt}")
    done = np.zeros_like(nsteps)
    t0 = time.time()
    while np.any(done < nsteps):
        step = np.minimum(nsteps - done, chunk)
        st = prop.propagate_items(psi, "midp", scheme, order, dt=np.asarray(dts), nsteps=step, opts=opts)
        done += step
        log(f"  {scheme}-{order}: {int(done.min())}..{int(done.max())} of {int(nsteps.max())} steps, "
            f"{time.time() - t0:.1f} s, mean GMRES iterations {st.iterations / max(st.solves, 1):.2f}")
    return {dt: s for dt, s in zip(dts, prop.unpack(psi))}


def sweep(item, T: float = 4000.0, dt0: float = 40.0, kmax: int = 3, order: int = 8,
          schemes=("suzuki", "triple_jump"), tol: float = 1e-14, restart: int = 48,
          chunk: int = 64, log=print) -> dict:
    opts = gqd.SolverOpts(tol=tol, restart=restart, maxit=2000)
    dts = [dt0 * 2.0 ** (-k) for k in range(kmax + 4)]
    ref_runs = run_batch(item, "suzuki", 8, dts, T, opts, chunk, log)
    result = {"T": T, "n": item.n, "order": order, "tol": tol, "dt": dts[:kmax + 1], "errors": {}}
    for scheme in schemes:
        if scheme == "suzuki" and order == 8:
            runs = ref_runs
        else:
            runs = run_batch(item, scheme, order, dts[:kmax + 1], T, opts, chunk, log)
        errs = [grid_norm(item.dq, runs[dts[k]] - ref_runs[dts[k + 3]]) for k in range(kmax + 1)]
        result["errors"][scheme] = errs
        result.setdefault("phase_errors", {})[scheme] = [
            phase_error(runs[dts[k]], ref_runs[dts[k + 3]]) for k in range(kmax + 1)]
        ok = [dts[k] for k in range(kmax + 1) if errs[k] <= 1e-10]
        result.setdefault("dt_star", {})[scheme] = max(ok) if ok else None
    return result


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--T", type=float, default=4000.0)
    ap.add_argument("--dt0", type=float, default=40.0)
    ap.add_argument("--kmax", type=int, default=3)
    ap.add_argument("--order", type=int, default=8)
    ap.add_argument("--tol", type=float, default=1e-14)
    ap.add_argument("--chunk", type=int, default=64)
    ap.add_argument("--json", type=str, default="")
    args = ap.parse_args(argv)
    item = inputs.nai_like_item(args.n)
    res = sweep(item, args.T, args.dt0, args.kmax, args.order, tol=args.tol, chunk=args.chunk,
                log=lambda m: print(m, flush=True))
    print(json.dumps(res), flush=True)
    if args.json:
        with open(args.json, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    sys.exit(main())
