"""Convergence of the wavefunction with grid density (App. B, Fig. 8): grids of
N = N0 * 2^k points whose ranges and densities both grow by sqrt(2) per doubling (so the
position and momentum grids stay balanced), all propagated in one ragged launch on the
GPU, each compared with the densest by trigonometric interpolation of its own state.

    python -m paper_1902_04661_amd.gridconv --tf 200 --dt 2
"""
from __future__ import annotations

import argparse
import json
import math
import sys
from typing import List, Sequence

import numpy as np

from . import gqd, inputs


def trig_interpolate(psi: np.ndarray, qmin: float, qmax: float, x: np.ndarray) -> np.ndarray:
    """Band-limited trigonometric interpolant of grid values psi (..., n) on the periodic
    grid [qmin, qmax), evaluated at points x: the DFT modes k' = -n/2+1 .. n/2-1 as plane
    waves exp(2 pi i k' (x - qmin) / L) and the Nyquist mode as its cosine, so that the
    interpolant takes the grid values at the grid points."""
    n = psi.shape[-1]
    L = qmax - qmin
    coef = np.fft.fft(psi, axis=-1) / n
    k = np.fft.fftfreq(n, d=1.0 / n)  # 0 .. n/2-1, -n/2 .. -1
    phase = 2.0 * np.pi * np.outer(x - qmin, k) / L  # (len(x), n)
    basis = np.exp(1j * phase)
    nyq = n // 2
    basis[:, nyq] = np.cos(phase[:, nyq])
    return coef @ basis.T


def study_items(sizes: Sequence[int] = (256, 512, 1024, 2048, 4096), center: float = 7.0,
                length0: float = 0.5, q0: float = 7.0, p0: float = 0.0, width: float = 0.05,
                amp: float = 0.4) -> List[inputs.Item1D]:
    """The NaI-like surfaces and coupling on grids centred at `center`; grid k has
    sizes[k] points and length length0 * sqrt(2)^k.  A narrow packet (width 0.05) makes
    the smallest ranges cut into its tails, which is what the study resolves."""
    items = []
    for k, n in enumerate(sizes):
        L = length0 * math.sqrt(2.0) ** k
        items.append(inputs.nai_like_item(n, center - 0.5 * L, center + 0.5 * L, q0=q0, p0=p0,
                                          width=width, amp=amp))
    return items


def compare_to_densest(items: Sequence[inputs.Item1D], states: Sequence[np.ndarray]) -> List[float]:
    """L2 error of each state's interpolant against the densest state, on the densest grid:
    inside a sparser grid's range its interpolant, outside it zero."""
    fine, ref = items[-1], states[-1]
    x = fine.q
    dq = fine.dq
    errs = []
    for it, st in zip(items[:-1], states[:-1]):
        inside = (x >= it.qmin) & (x < it.qmax)
        approx = np.zeros_like(ref)
        approx[:, inside] = trig_interpolate(st, it.qmin, it.qmax, x[inside])
        errs.append(math.sqrt(dq * float(np.sum(np.abs(ref - approx) ** 2))))
    return errs


def grid_study(tf: float = 200.0, dt: float = 2.0, order: int = 8, tol: float = 1e-14,
               sizes: Sequence[int] = (256, 512, 1024, 2048, 4096), **kw) -> dict:
    """Errors at t = 0 and t = tf of every grid against the densest (Suzuki composition of
    the trapezoidal rule; the paper's Fig. 8 uses an optimal 10th-order one)."""
    items = study_items(sizes, **kw)
    prop = gqd.from_items(items)
    psi = prop.pack([it.psi0 for it in items])
    init = prop.unpack(psi)
    nsteps = int(round(tf / dt))
    st = prop.propagate(psi, "trap", "suzuki", order, dt, nsteps, gqd.SolverOpts(tol=tol, restart=48))
    final = prop.unpack(psi)
    return {"sizes": list(sizes)[:-1], "lengths": [it.qmax - it.qmin for it in items[:-1]],
            "error_t0": compare_to_densest(items, init), "error_tf": compare_to_densest(items, final),
            "tf": tf, "dt": dt, "order": order, "mean_gmres_iterations": st.iterations / max(st.solves, 1)}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--tf", type=float, default=200.0)
    ap.add_argument("--dt", type=float, default=2.0)
    ap.add_argument("--order", type=int, default=8)
    args = ap.parse_args(argv)
    print(json.dumps(grid_study(args.tf, args.dt, args.order)), flush=True)


if __name__ == "__main__":
    sys.exit(main())
