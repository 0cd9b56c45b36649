"""Seeded synthetic workloads for the two-surface adiabatic model.

This module builds *inputs only*: position grids, the adiabatic potential
surfaces V_s(q), the nonadiabatic coupling component F12(q) and the initial
Gaussian wavepacket.  It holds none of the propagation method's arithmetic
(no Hamiltonian action, no solver, no composition), so both the HIP path and
the CPU oracle can be fed from it without sharing any of the method.

The paper's own NaI model (Sec. III) cites Engel and Metiu for its potential
parameters and does not print them, so a "NaI-like" model with the same
shapes stands in: a bound Morse surface and a repulsive surface, a Gaussian
coupling peak between them, a reduced mass of NaI scale (3.5e4 a.u.) and an
initial Gaussian of width ~0.12 bohr (the paper's is 0.110436 bohr).

Conventions (atomic units, hbar = 1):
  * uniform periodic grid q_j = qmin + j*(qmax - qmin)/n, j = 0..n-1 (right end excluded);
  * surface index 0 is "surface 1" (Morse), index 1 is "surface 2" (repulsive);
  * wavefunction arrays have shape (S=2, *n) and dtype complex128;
  * the Gaussian width w is the standard deviation of |psi|^2, i.e.
    psi ~ exp(-(q-q0)^2/(4 w^2) + i p0 (q-q0)), renormalised on the grid so that
    dq * sum |psi|^2 = 1.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

MASS = 3.5e4  # reduced mass (a.u.)
QMIN, QMAX = 3.0, 16.0

# Surface and coupling parameters of the 1D NaI-like model.
MORSE_D, MORSE_A, MORSE_Q0 = 0.02, 1.0, 5.0
REP_A, REP_B, REP_Q = 0.08, 0.6, 3.0
COUP_AMP, COUP_CENTER, COUP_WIDTH = 0.4, 7.0, 0.5
PACKET_Q0, PACKET_P0, PACKET_W = 5.0, 0.0, 0.12

BATCH_SIZES = (256, 512, 1024, 2048, 4096)


def uniform_grid(n: int, qmin: float, qmax: float) -> np.ndarray:
    """Periodic uniform grid of n points on [qmin, qmax) (right end excluded)."""
    return qmin + np.arange(n, dtype=np.float64) * ((qmax - qmin) / n)


def morse(q, d=MORSE_D, a=MORSE_A, q0=MORSE_Q0):
    """Morse well, zero at its minimum: d (1 - exp(-a (q - q0)))^2."""
    return d * (1.0 - np.exp(-a * (q - q0))) ** 2


def repulsive(q, amp=REP_A, b=REP_B, q0=REP_Q):
    """Repulsive exponential wall amp * exp(-b (q - q0))."""
    return amp * np.exp(-b * (q - q0))


def coupling(q, amp=COUP_AMP, center=COUP_CENTER, width=COUP_WIDTH):
    """Gaussian coupling peak F12(q) = amp * exp(-((q - center)/width)^2)."""
    return amp * np.exp(-(((q - center) / width) ** 2))


def gaussian_packet_1d(q: np.ndarray, q0: float, p0: float, width: float,
                       surface: int = 0, nsurf: int = 2) -> np.ndarray:
    """Normalised Gaussian on one surface, zero on the others; shape (nsurf, n)."""
    dq = q[1] - q[0]
    g = np.exp(-((q - q0) ** 2) / (4.0 * width * width) + 1j * p0 * (q - q0))
    g = g / np.sqrt(dq * np.sum(np.abs(g) ** 2))
    psi = np.zeros((nsurf, q.size), dtype=np.complex128)
    psi[surface] = g
    return psi


@dataclass
class Item1D:
    """One 1D two-surface wavepacket problem: grid, surfaces, coupling, initial state."""
    n: int
    qmin: float
    qmax: float
    mass: float
    V: np.ndarray      # (2, n) float64
    F: np.ndarray      # (1, n) float64, F12 (F21 = -F12)
    psi0: np.ndarray   # (2, n) complex128
    params: dict = field(default_factory=dict)

    @property
    def q(self) -> np.ndarray:
        return uniform_grid(self.n, self.qmin, self.qmax)

    @property
    def dq(self) -> float:
        return (self.qmax - self.qmin) / self.n


def nai_like_item(n: int = 512, qmin: float = QMIN, qmax: float = QMAX,
                  q0: float = PACKET_Q0, p0: float = PACKET_P0, width: float = PACKET_W,
                  amp: float = COUP_AMP, center: float = COUP_CENTER,
                  cwidth: float = COUP_WIDTH, mass: float = MASS) -> Item1D:
    """The 1D NaI-like model on n points with a Gaussian on surface index 0."""
    q = uniform_grid(n, qmin, qmax)
    V = np.stack([morse(q), repulsive(q)])
    F = coupling(q, amp, center, cwidth)[None, :]
    psi0 = gaussian_packet_1d(q, q0, p0, width)
    return Item1D(n, qmin, qmax, mass, V, F, psi0,
                  dict(q0=q0, p0=p0, width=width, amp=amp, center=center, cwidth=cwidth))


def crank_nicolson_config() -> dict:
    """Trapezoidal-rule run: N=512 on [3,16), dt=10 a.u., 2000 steps, GMRES tol 1e-13."""
    return dict(item=nai_like_item(512), method="trap", order=2, dt=10.0, nsteps=2000, tol=1e-13)


def convergence_sweep_config(kmax: int = 10) -> dict:
    """Implicit-midpoint sweep at N=2048: dt_k = 40 * 2^-k to T = 4000 a.u."""
    return dict(item=nai_like_item(2048), method="midp", T=4000.0,
                dts=[40.0 * 2.0 ** (-k) for k in range(kmax + 1)])


def ragged_batch_draws(batch: int = 4096, seed: int = 0,
                       sizes: Sequence[int] = BATCH_SIZES) -> dict:
    """Draws for the ragged batch, in a fixed order from numpy's default_rng(seed):
    grid size, packet centre q0 ~ U[4.5, 6], momentum p0 ~ U[-5, 5],
    coupling amplitude ~ U[0.1, 0.8]."""
    rng = np.random.default_rng(seed)
    n = rng.choice(np.asarray(sizes), size=batch)
    q0 = rng.uniform(4.5, 6.0, size=batch)
    p0 = rng.uniform(-5.0, 5.0, size=batch)
    amp = rng.uniform(0.1, 0.8, size=batch)
    return dict(n=n.astype(np.int64), q0=q0, p0=p0, amp=amp)


def ragged_batch(batch: int = 4096, seed: int = 0, sizes: Sequence[int] = BATCH_SIZES,
                 fixed_n: int | None = None) -> List[Item1D]:
    """Items of the ragged batch (or, with fixed_n, the same draws on one grid size)."""
    d = ragged_batch_draws(batch, seed, sizes)
    items = []
    for b in range(batch):
        n = int(fixed_n if fixed_n is not None else d["n"][b])
        items.append(nai_like_item(n, q0=float(d["q0"][b]), p0=float(d["p0"][b]),
                                   amp=float(d["amp"][b])))
    return items


def adjoint_batch(batch: int = 256, seed: int = 1, n: int = 1024) -> List[Item1D]:
    """Batch for the gradient workload: same draws as the ragged batch, N fixed."""
    rng = np.random.default_rng(seed)
    q0 = rng.uniform(4.5, 6.0, size=batch)
    p0 = rng.uniform(-5.0, 5.0, size=batch)
    amp = rng.uniform(0.1, 0.8, size=batch)
    return [nai_like_item(n, q0=float(q0[b]), p0=float(p0[b]), amp=float(amp[b]))
            for b in range(batch)]


# ------------------------------------------------------------------ diabatic model

@dataclass
class DiabaticItem:
    """A two-state diabatic model on a 1D grid: H_diab = p^2 / 2m + W(q) with the real
    symmetric W of Sec. II.F, its first derivatives, and a packet on diabatic state 1."""
    n: int
    qmin: float
    qmax: float
    mass: float
    W: np.ndarray    # (3, n): W11, W22, W12
    dW: np.ndarray   # (3, n): their derivatives in q
    psi0: np.ndarray  # (2, n) diabatic components

    @property
    def q(self) -> np.ndarray:
        return uniform_grid(self.n, self.qmin, self.qmax)

    @property
    def dq(self) -> float:
        return (self.qmax - self.qmin) / self.n


def diabatic_crossing_item(n: int = 2048, qmin: float = QMIN, qmax: float = QMAX,
                           k: float = 0.035, centers=(5.0, 7.0), c12: float = 0.003,
                           x12: float = 6.0, w12: float = 1.0, q0: float = 5.0, p0: float = 40.0,
                           width: float = 0.12, mass: float = MASS) -> DiabaticItem:
    """Two shifted harmonic diabats W_ii = k (q - c_i)^2 / 2 crossing once (at 6 bohr),
    coupled by W12 = c12 exp(-((q - x12) / w12)^2); a Gaussian on diabat 1 whose
    momentum carries it through the crossing.  k = 0.035 gives the packet's width 0.12
    as the harmonic ground state of diabat 1 at m = 3.5e4."""
    q = uniform_grid(n, qmin, qmax)
    W11 = 0.5 * k * (q - centers[0]) ** 2
    W22 = 0.5 * k * (q - centers[1]) ** 2
    g = np.exp(-(((q - x12) / w12) ** 2))
    W12 = c12 * g
    dW = np.stack([k * (q - centers[0]), k * (q - centers[1]), -2.0 * (q - x12) / (w12 * w12) * W12])
    return DiabaticItem(n, qmin, qmax, mass, np.stack([W11, W22, W12]), dW,
                        gaussian_packet_1d(q, q0, p0, width))


# --------------------------------------------------------------------------- 2D model

@dataclass
class Item2D:
    n: Tuple[int, int]
    qmin: Tuple[float, float]
    qmax: Tuple[float, float]
    mass: Tuple[float, float]
    V: np.ndarray      # (2, n1, n2)
    F: np.ndarray      # (2, n1, n2): F12 along q1 and along q2
    psi0: np.ndarray   # (2, n1, n2)
    params: dict = field(default_factory=dict)

    def grids(self):
        q1 = uniform_grid(self.n[0], self.qmin[0], self.qmax[0])
        q2 = uniform_grid(self.n[1], self.qmin[1], self.qmax[1])
        return np.meshgrid(q1, q2, indexing="ij")


def coupling_2d(q1, q2, amp=0.4, c1=7.0, c2=5.0, w=0.5, direction=(0.8, 0.6)):
    """Vector coupling F12^(d) = amp * exp(-((q1-c1)^2 + (q2-c2)^2)/w^2) * direction_d."""
    g = amp * np.exp(-((q1 - c1) ** 2 + (q2 - c2) ** 2) / (w * w))
    return np.stack([direction[0] * g, direction[1] * g])


def two_dim_item(n1: int = 256, n2: int = 256, seed: int = 2,
                 cparams=(0.4, 7.0, 5.0, 0.5), q0=(5.8, 5.0), p0=(0.0, 0.0),
                 width=(0.12, 0.12)) -> Item2D:
    """2D two-surface model on [3,16) x [1.5,8.5): anharmonic surfaces, a seeded
    Gaussian ridge R on surface 2 and a Gaussian vector coupling."""
    rng = np.random.default_rng(seed)
    alpha = rng.uniform(-0.5, 0.5)
    beta = rng.uniform(5.5, 7.0)
    qmin, qmax = (3.0, 1.5), (16.0, 8.5)
    q1 = uniform_grid(n1, qmin[0], qmax[0])
    q2 = uniform_grid(n2, qmin[1], qmax[1])
    Q1, Q2 = np.meshgrid(q1, q2, indexing="ij")
    ridge = 0.01 * np.exp(-((Q1 - alpha * Q2 - beta) ** 2) / (2 * 0.3 ** 2))
    v1 = morse(Q1) + 0.02 * (Q2 - 5.0) ** 2 + 0.002 * (Q1 - 5.0) * (Q2 - 5.0) ** 2
    v2 = repulsive(Q1) + 0.02 * (Q2 - 5.0) ** 2 + ridge
    F = coupling_2d(Q1, Q2, *cparams)
    dq1, dq2 = q1[1] - q1[0], q2[1] - q2[0]
    g = np.exp(-((Q1 - q0[0]) ** 2) / (4 * width[0] ** 2) - ((Q2 - q0[1]) ** 2) / (4 * width[1] ** 2)
               + 1j * (p0[0] * (Q1 - q0[0]) + p0[1] * (Q2 - q0[1])))
    g = g / np.sqrt(dq1 * dq2 * np.sum(np.abs(g) ** 2))
    psi0 = np.zeros((2, n1, n2), dtype=np.complex128)
    psi0[0] = g
    return Item2D((n1, n2), qmin, qmax, (MASS, MASS), np.stack([v1, v2]), F, psi0,
                  dict(alpha=alpha, beta=beta, cparams=cparams))


def random_state(shape, seed: int) -> np.ndarray:
    """Seeded complex Gaussian noise of the given shape (for parity tests)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
