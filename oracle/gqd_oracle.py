"""Plain FP64 CPU oracle for the implicit geometric integrators of Choi & Vanicek,
"Efficient geometric integrators for nonadiabatic quantum dynamics. I. The adiabatic
representation" (J. Chem. Phys. 150, 204112 (2019), arXiv:1902.04661).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke entry point and the
benchmark's CPU-baseline leg may import or call this module.  It imports nothing
from the HIP package and the HIP package never imports it.

What it computes, in the paper's order and notation (hbar = 1, as in App. A):
  * the dynamic Fourier action of p on a uniform periodic grid (Sec. II.E);
  * the adiabatic molecular Hamiltonian H = (1/2) [p 1 - i F]^dag m^-1 [p 1 - i F] + V,
    Eq. (22), for S = 2 surfaces, applied in that factored form;
  * explicit Euler (Eq. 13) and implicit Euler (Eq. 14), the latter solved by GMRES
    with the explicit-Euler initial guess (Sec. II.C), and second-order differencing
    (Eq. 16) started by a second-order Runge-Kutta step (Sec. III);
  * the two-state diabatic -> adiabatic transformation (Sec. II.F, Eqs. 24-28) and, in
    the diabatic representation, the composed second-order split-operator method of
    Table I, as an independent check of the adiabatic propagation;
  * trapezoidal rule (Eq. 18) and implicit midpoint (Eq. 19);
  * triple-jump (Eq. 20) and Suzuki-fractal (Eq. 21) recursive symmetric compositions
    (Sec. II.D);
  * the invariants of Sec. II.A: norm, inner product, symplectic two-form (Eq. 5),
    energy (Eq. 6), populations; and the adjoint (reverse) sweep that the exact
    time reversibility of App. A (Eq. A40) makes checkpoint-free.

Numpy primitives (FFT, vdot, norm) serve as steps; there is no blocking, fusion or
reordering beyond the definitions.  GMRES is Saad & Schultz's method: Arnoldi with
modified Gram-Schmidt, complex Givens rotations, restart after m iterations.

Readings where the paper is silent (the same readings bind the HIP path):
  * grid: periodic, right end excluded, dq = L/n; momentum p_k = 2 pi k'/L with
    k' = k for k < n/2 and k - n otherwise (the Nyquist entry is -n/2);
  * forward DFT X_k = sum_j x_j exp(-2 pi i j k/n), inverse with 1/n;
  * GMRES stops when the Givens residual estimate |g_{j+1}| <= tol * ||b||
    (Euclidean norms); after m iterations without that it restarts from the current
    x with a freshly computed true residual; it fails after maxit iterations;
  * composition: U_{p+2}(dt) = U_p(g_M dt) ... U_p(g_1 dt) applies g_1 first; the
    flattened list is built level by level, tau <- gamma * tau;
  * substep of length h has half-step a = h/2 computed as 0.5 * (tau * dt);
  * "economy" mode uses exact identities of the Cayley map instead of one explicit
    half-step per substep: midpoint psi' = 2x - psi (since (1 + iaH)x = psi implies
    (1 - iaH)x = 2x - psi), trapezoid reuses H psi' = (b - psi')/(i a) from the
    previous solve.  "literal" mode performs every half-step, so it costs the 3 + I
    H-applications per substep that Table I counts.

Every function here is pinned by a test under tests/ against a closed form, a dense
brute-force computation, an invariant or a value the paper prints.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

TRAP, MIDP = "trap", "midp"
TRIPLE_JUMP, SUZUKI, OPTIMAL = "triple_jump", "suzuki", "optimal"


# ----------------------------------------------------------------------------- grid


def momentum_grid(n: int, length: float) -> np.ndarray:
    """Momentum grid conjugate to a uniform periodic position grid of n points over a
    period `length` (dynamic Fourier method, Sec. II.E): p_k = 2 pi k'/L."""
    k = np.arange(n)
    kp = np.where(k < n // 2, k, k - n).astype(np.float64)
    return 2.0 * np.pi * kp / length


@dataclass
class Model:
    """Grid, masses, adiabatic potentials and coupling of an S = 2 problem.

    V has shape (2, *n): the diagonal of the potential matrix (Eq. 22).
    F has shape (D, *n): F12 along each nuclear dof; F21 = -F12, F11 = F22 = 0 (Eq. 28).
    """
    n: Tuple[int, ...]
    qmin: Tuple[float, ...]
    qmax: Tuple[float, ...]
    mass: Tuple[float, ...]
    V: np.ndarray
    F: np.ndarray

    def __post_init__(self):
        self.n = tuple(int(x) for x in np.atleast_1d(self.n))
        self.qmin = tuple(float(x) for x in np.atleast_1d(self.qmin))
        self.qmax = tuple(float(x) for x in np.atleast_1d(self.qmax))
        self.mass = tuple(float(x) for x in np.atleast_1d(self.mass))
        D = len(self.n)
        assert len(self.qmin) == D and len(self.qmax) == D and len(self.mass) == D
        self.V = np.asarray(self.V, dtype=np.float64).reshape((2,) + self.n)
        self.F = np.asarray(self.F, dtype=np.float64).reshape((D,) + self.n)
        self._p = [momentum_grid(self.n[d], self.qmax[d] - self.qmin[d]) for d in range(D)]

    @property
    def D(self) -> int:
        return len(self.n)

    @property
    def shape(self) -> Tuple[int, ...]:
        return (2,) + self.n

    @property
    def dq(self) -> Tuple[float, ...]:
        return tuple((self.qmax[d] - self.qmin[d]) / self.n[d] for d in range(self.D))

    @property
    def dv(self) -> float:
        """Volume element of the grid quadrature: prod_d dq_d."""
        return float(np.prod(self.dq))

    def momentum(self, d: int) -> np.ndarray:
        return self._p[d]


def model_from_item(item) -> Model:
    """Build a Model from an input item (an object with n, qmin, qmax, mass, V, F)."""
    return Model(item.n, item.qmin, item.qmax, item.mass, item.V, item.F)


# ----------------------------------------------------------------- Hamiltonian action


class Counter:
    """Counts Hamiltonian applications (the paper's cost unit is 4D Fourier
    transforms per H-application, Sec. II.F)."""

    def __init__(self):
        self.h_applies = 0


def apply_P(model: Model, psi: np.ndarray, d: int) -> np.ndarray:
    """p_d acting on every surface: Fourier transform along dof d, multiply by the
    momentum grid, transform back (Sec. II.E)."""
    ax = 1 + d
    shape = [1] * psi.ndim
    shape[ax] = model.n[d]
    p = model.momentum(d).reshape(shape)
    return np.fft.ifft(p * np.fft.fft(psi, axis=ax), axis=ax)


def apply_F(model: Model, psi: np.ndarray, d: int) -> np.ndarray:
    """Electronic matrix F^(d) acting pointwise: (F psi)_1 = F12 psi_2,
    (F psi)_2 = F21 psi_1 = -F12 psi_1 (Eq. 28)."""
    f = model.F[d]
    return np.stack([f * psi[1], -f * psi[0]])


def apply_A(model: Model, psi: np.ndarray, d: int) -> np.ndarray:
    """[p_d 1 - i F^(d)] psi, the factor of Eq. (22) (hbar = 1).  With F real and
    antisymmetric, -iF is Hermitian, so this factor equals its own adjoint."""
    return apply_P(model, psi, d) - 1j * apply_F(model, psi, d)


def apply_H(model: Model, psi: np.ndarray, counter: Optional[Counter] = None) -> np.ndarray:
    """H psi = sum_d (1/2 m_d) A_d^dag A_d psi + V psi, Eq. (22), with A_d^dag = A_d."""
    if counter is not None:
        counter.h_applies += 1
    out = model.V * psi
    for d in range(model.D):
        out = out + apply_A(model, apply_A(model, psi, d), d) / (2.0 * model.mass[d])
    return out


def dense_H(model: Model) -> np.ndarray:
    """The Hamiltonian as a dense matrix, column by column (small grids only)."""
    size = int(np.prod(model.shape))
    H = np.zeros((size, size), dtype=np.complex128)
    for c in range(size):
        e = np.zeros(size, dtype=np.complex128)
        e[c] = 1.0
        H[:, c] = apply_H(model, e.reshape(model.shape)).ravel()
    return H


# ------------------------------------------------------------------------- invariants


def inner(model: Model, psi: np.ndarray, phi: np.ndarray) -> complex:
    """<psi|phi> on the grid: dv * sum conj(psi) phi (Sec. II.A)."""
    return complex(model.dv * np.vdot(psi.ravel(), phi.ravel()))


def norm(model: Model, psi: np.ndarray) -> float:
    """||psi|| = <psi|psi>^(1/2) (Sec. II.A)."""
    return math.sqrt(inner(model, psi, psi).real)


def energy(model: Model, psi: np.ndarray) -> float:
    """E = <psi|H|psi> (Eq. 6); real for Hermitian H, the real part is returned."""
    return inner(model, psi, apply_H(model, psi)).real


def populations(model: Model, psi: np.ndarray) -> np.ndarray:
    """P_s = dv * sum_j |psi_s,j|^2 for s = 1, 2."""
    return model.dv * np.sum(np.abs(psi.reshape(2, -1)) ** 2, axis=1)


def symplectic_form(model: Model, psi: np.ndarray, phi: np.ndarray) -> float:
    """omega(psi, phi) = -2 hbar Im <psi|phi> (Eq. 5), hbar = 1."""
    return -2.0 * inner(model, psi, phi).imag


# ------------------------------------------------------------------------------ GMRES


@dataclass
class SolverOpts:
    tol: float = 1e-13     # relative residual target |r| <= tol * |b|
    restart: int = 64      # Krylov dimension m before a restart
    maxit: int = 1000      # total Arnoldi iterations allowed per solve
    literal: bool = False  # True: perform every explicit half-step (3 + I applies)
    verify: bool = False   # True: confirm convergence on the true residual (restart if not met)
    precond: bool = False  # True: right-precondition by the exact inverse of 1 + i a T


@dataclass
class SolveInfo:
    iterations: int
    converged: bool
    true_resid: float = float("nan")  # |b - A x| / |b| when the solve ended on it


@dataclass
class Stats:
    h_applies: int = 0
    solves: int = 0
    iterations: int = 0
    max_iters: int = 0
    failures: int = 0
    max_true_resid: float = 0.0
    per_solve: List[int] = field(default_factory=list)

    def record(self, info: SolveInfo):
        self.solves += 1
        self.iterations += info.iterations
        self.max_iters = max(self.max_iters, info.iterations)
        self.per_solve.append(info.iterations)
        if info.converged and not math.isnan(info.true_resid):
            self.max_true_resid = max(self.max_true_resid, info.true_resid)
        if not info.converged:
            self.failures += 1


def givens(a: complex, b: float) -> Tuple[float, complex, complex]:
    """Complex Givens rotation G = [[c, s], [-conj(s), c]] (c real) with
    G [a, b]^T = [r, 0]^T for real b >= 0."""
    if b == 0.0:
        return 1.0, 0j, complex(a)
    if a == 0:
        return 0.0, 1.0 + 0j, complex(b)
    absa = abs(a)
    rho = math.sqrt(absa * absa + b * b)
    phase = a / absa
    return absa / rho, phase * (b / rho), phase * rho


def gmres(matvec: Callable[[np.ndarray], np.ndarray], b: np.ndarray, x0: np.ndarray,
          tol: float, m: int, maxit: int, verify: bool = False,
          prec: Optional[Callable[[np.ndarray], np.ndarray]] = None) -> Tuple[np.ndarray, SolveInfo]:
    """Restarted GMRES(m) (Saad & Schultz) for A x = b from x0 (Sec. II.C).

    Arnoldi with modified Gram-Schmidt, least squares by Givens rotations; the stop
    rule is the residual estimate |g_{j+1}| <= tol * ||b||.  With verify, a solve that
    meets it forms x and ends only if the true residual |b - A x| meets the tolerance
    as well; otherwise GMRES restarts from that x.  With prec (x -> M^-1 x), GMRES is
    right-preconditioned: the Arnoldi process runs on A M^-1 and the cycle's update is
    M^-1 V y, so the residual it minimises and tests is still that of A x = b."""
    P = prec if prec is not None else (lambda v: v)
    bnorm = float(np.linalg.norm(b))
    x = x0.copy()
    iters = 0
    while True:
        r = b - matvec(x)
        beta = float(np.linalg.norm(r))
        if beta <= tol * bnorm:
            return x, SolveInfo(iters, True, beta / bnorm if bnorm > 0.0 else 0.0)
        if iters >= maxit:
            return x, SolveInfo(iters, False)
        basis = np.zeros((m + 1, b.size), dtype=np.complex128)
        R = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        basis[0] = r / beta
        k = 0
        converged = False
        for j in range(m):
            w = matvec(P(basis[j]))
            iters += 1
            for i in range(j + 1):                      # modified Gram-Schmidt
                R[i, j] = np.vdot(basis[i], w)
                w = w - R[i, j] * basis[i]
            hn = float(np.linalg.norm(w))
            for i in range(j):                          # earlier rotations on column j
                t = cs[i] * R[i, j] + sn[i] * R[i + 1, j]
                R[i + 1, j] = -np.conj(sn[i]) * R[i, j] + cs[i] * R[i + 1, j]
                R[i, j] = t
            c, s, rr = givens(R[j, j], hn)
            cs[j], sn[j] = c, s
            R[j, j] = rr
            g[j + 1] = -np.conj(s) * g[j]
            g[j] = c * g[j]
            k = j + 1
            if abs(g[j + 1]) <= tol * bnorm:
                converged = True
                break
            if hn == 0.0 or iters >= maxit:
                break
            basis[j + 1] = w / hn
        y = np.zeros(k, dtype=np.complex128)
        for i in range(k - 1, -1, -1):                  # back substitution R y = g
            y[i] = (g[i] - np.dot(R[i, i + 1:k], y[i + 1:k])) / R[i, i]
        x = x + P(basis[:k].T @ y)
        if converged and not verify:
            return x, SolveInfo(iters, True)


# ------------------------------------------------------------- elementary propagators


def explicit_euler(model: Model, psi: np.ndarray, eps: float,
                   counter: Optional[Counter] = None, hpsi: Optional[np.ndarray] = None) -> np.ndarray:
    """U_expl(eps) psi = (1 - i eps H) psi, Eq. (13)."""
    if hpsi is None:
        hpsi = apply_H(model, psi, counter)
    return psi - 1j * eps * hpsi


def kinetic_inverse(model: Model, eps: float) -> Callable[[np.ndarray], np.ndarray]:
    """x -> (1 + i eps T)^-1 x with T = sum_d p_d^2 / 2 m_d, exactly, in momentum space
    (forward DFT along every nuclear axis, division, inverse DFT), the same operator on
    both surfaces: a right preconditioner for 1 + i eps H, whose kinetic part it inverts
    (the coupling and the potential are left to GMRES)."""
    T = np.zeros(model.shape[1:], dtype=np.float64)
    for d in range(model.D):
        p = momentum_grid(model.n[d], model.qmax[d] - model.qmin[d])
        sh = [1] * model.D
        sh[d] = model.n[d]
        T = T + (p.reshape(sh) ** 2) / (2.0 * model.mass[d])
    den = 1.0 + 1j * eps * T
    axes = tuple(range(1, model.D + 1))

    def apply(x: np.ndarray) -> np.ndarray:
        return np.fft.ifftn(np.fft.fftn(x, axes=axes) / den[None], axes=axes)

    return apply


def implicit_euler(model: Model, psi: np.ndarray, eps: float, opts: SolverOpts,
                   stats: Optional[Stats] = None) -> np.ndarray:
    """U_impl(eps) psi = (1 + i eps H)^-1 psi, Eq. (14), by GMRES with the explicit-Euler
    initial guess (1 - i eps H) psi (Sec. II.C)."""
    stats = stats if stats is not None else Stats()
    counter = Counter()
    shape = psi.shape

    def matvec(v):
        return v + 1j * eps * apply_H(model, v.reshape(shape), counter).ravel()

    x0 = explicit_euler(model, psi, eps, counter)
    prec = kinetic_inverse(model, eps) if opts.precond else None
    x, info = gmres(matvec, psi.ravel(), x0.ravel(), opts.tol, opts.restart, opts.maxit, opts.verify,
                    None if prec is None else (lambda v: prec(v.reshape(shape)).ravel()))
    stats.record(info)
    stats.h_applies += counter.h_applies
    return x.reshape(shape)


def trapezoidal_step(model: Model, psi: np.ndarray, h: float, opts: SolverOpts,
                     stats: Optional[Stats] = None, hpsi: Optional[np.ndarray] = None):
    """U_trap(h) = U_impl(h/2) U_expl(h/2), Eq. (18).

    Returns (psi', H psi') where the second item is the economy-mode reuse of the solve,
    H psi' = (b - psi')/(i a), or None in literal mode."""
    stats = stats if stats is not None else Stats()
    a = 0.5 * h
    counter = Counter()
    if opts.literal:
        hpsi = None
    b = explicit_euler(model, psi, a, counter, hpsi)
    stats.h_applies += counter.h_applies
    out = implicit_euler(model, b, a, opts, stats)
    h_out = None if opts.literal else (b - out) / (1j * a)
    return out, h_out


def midpoint_step(model: Model, psi: np.ndarray, h: float, opts: SolverOpts,
                  stats: Optional[Stats] = None) -> np.ndarray:
    """U_midp(h) = U_expl(h/2) U_impl(h/2), Eq. (19)."""
    stats = stats if stats is not None else Stats()
    a = 0.5 * h
    x = implicit_euler(model, psi, a, opts, stats)
    if opts.literal:
        counter = Counter()
        out = explicit_euler(model, x, a, counter)
        stats.h_applies += counter.h_applies
        return out
    return 2.0 * x - psi


# ------------------------------------------------------------------------ composition


def composition_gammas(scheme: str, p: int) -> List[float]:
    """Coefficients that raise a symmetric method of order p to order p + 2:
    triple jump (M = 3, Eq. 20) or Suzuki's fractal (M = 5, Eq. 21), completed by
    the symmetry gamma_{M+1-n} = gamma_n."""
    if scheme == TRIPLE_JUMP:
        s = 2.0 ** (1.0 / (p + 1))
        g1 = 1.0 / (2.0 - s)
        g2 = -s / (2.0 - s)
        return [g1, g2, g1]
    if scheme == SUZUKI:
        s = 4.0 ** (1.0 / (p + 1))
        g1 = 1.0 / (4.0 - s)
        g3 = -s / (4.0 - s)
        return [g1, g1, g3, g1, g1]
    raise ValueError(f"unknown composition scheme {scheme!r}")


# The non-recursive "optimal" compositions Sec. II.D uses, as published: the first
# (M + 1)/2 coefficients g_1 .. g_(M+1)/2, the rest given by g_(M+1-n) = g_n.
#   order 6, M = 9 and order 8, M = 17: Kahan and Li (1997), the largest |g_n| smallest;
#   order 10, M = 35: Sofroniou and Spaletta (2005), the sum of |g_n| smallest.
# At fourth order the section states that Suzuki's fractal is the optimal scheme.
OPTIMAL_HALVES = {
    6: [0.39216144400731413928, 0.33259913678935943860, -0.70624617255763935981,
        0.08221359629355080023, 0.79854399093482996340],
    8: [0.13020248308889008088, 0.56116298177510838456, -0.38947496264484728641,
        0.15884190655515560090, -0.39590389413323757734, 0.18453964097831570709,
        0.25837438768632204729, 0.29501172360931029887, -0.60550853383003451170],
    10: [0.07879572252168641926, 0.31309610341510852776, 0.02791838323507806611,
         -0.22959284159390709415, 0.13096206107716486317, -0.26973340565451071434,
         0.07497334315589143567, 0.11199342399981020489, 0.36613344954622675119,
         -0.39910563013603589788, 0.10308739852747107732, 0.41143087395589023782,
         -0.00486636058313526176, -0.39203335370863990645, 0.05194250296244964704,
         0.05066509075992449634, 0.04967437063972987905, 0.04931773575959453792],
}


def optimal_gammas(order: int) -> List[float]:
    """g_1 .. g_M of the non-recursive composition of the given order (4, 6, 8, 10)."""
    if order == 4:
        return composition_gammas(SUZUKI, 2)
    if order not in OPTIMAL_HALVES:
        raise ValueError(f"no non-recursive composition of order {order}")
    half = OPTIMAL_HALVES[order]
    return half + half[-2::-1]


def substep_fractions(scheme: str, order: int) -> List[float]:
    """Flattened fractions tau_c of the time step, in order of application, for the
    composition of a second-order method up to `order` (Sec. II.D): recursive triple
    jump or Suzuki fractal, 3^(order/2 - 1) or 5^(order/2 - 1) of them, or the
    non-recursive optimal one (5, 9, 17, 35 of them at orders 4, 6, 8, 10)."""
    if order < 2 or order % 2:
        raise ValueError("order must be even and >= 2")
    if scheme == OPTIMAL:
        return [1.0] if order == 2 else optimal_gammas(order)
    taus = [1.0]
    for p in range(2, order, 2):
        gam = composition_gammas(scheme, p)
        taus = [g * t for g in gam for t in taus]
    return taus


# ------------------------------------------------------------------------ propagation


def propagate(model: Model, psi0: np.ndarray, method: str, scheme: str, order: int,
              dt: float, nsteps: int, opts: SolverOpts,
              stats: Optional[Stats] = None) -> np.ndarray:
    """nsteps steps of the composed trapezoidal rule or implicit midpoint method."""
    stats = stats if stats is not None else Stats()
    taus = substep_fractions(scheme, order)
    psi = np.array(psi0, dtype=np.complex128, copy=True)
    hpsi = None
    for _ in range(nsteps):
        for tau in taus:
            h = tau * dt
            if method == TRAP:
                psi, hpsi = trapezoidal_step(model, psi, h, opts, stats, hpsi)
            elif method == MIDP:
                psi = midpoint_step(model, psi, h, opts, stats)
            else:
                raise ValueError(f"unknown method {method!r}")
    return psi


def explicit_euler_propagate(model: Model, psi0: np.ndarray, dt: float, nsteps: int) -> np.ndarray:
    """Repeated explicit Euler steps (Eq. 13): a non-geometric control."""
    psi = np.array(psi0, dtype=np.complex128, copy=True)
    for _ in range(nsteps):
        psi = explicit_euler(model, psi, dt)
    return psi


def implicit_euler_propagate(model: Model, psi0: np.ndarray, dt: float, nsteps: int,
                             opts: SolverOpts) -> np.ndarray:
    """Repeated implicit Euler steps (Eq. 14): a non-geometric control."""
    psi = np.array(psi0, dtype=np.complex128, copy=True)
    for _ in range(nsteps):
        psi = implicit_euler(model, psi, dt, opts)
    return psi


def sod_start(model: Model, psi0: np.ndarray, dt: float) -> np.ndarray:
    """psi(-dt) from psi(0) by one second-order Runge-Kutta step of length -dt (Sec. III,
    discussion of Fig. 7).  For the linear equation d psi/dt = -i H psi every two-stage
    second-order scheme gives the same step, the second-order Taylor polynomial:
    psi(-dt) = (1 + i dt H - dt^2 H^2 / 2) psi(0)."""
    h1 = apply_H(model, psi0)
    h2 = apply_H(model, h1)
    return psi0 + 1j * dt * h1 - 0.5 * dt * dt * h2


def sod_propagate(model: Model, psi0: np.ndarray, dt: float, nsteps: int,
                  return_previous: bool = False):
    """Second-order differencing, Eq. (16): psi(t + dt) = psi(t - dt) - 2 i dt H psi(t),
    started from psi(0) and psi(-dt) = sod_start(psi(0)).  With return_previous, also
    psi(t_f - dt), the second state the two-step recurrence carries."""
    prev = sod_start(model, psi0, dt)
    cur = np.array(psi0, dtype=np.complex128, copy=True)
    for _ in range(nsteps):
        nxt = prev - 2j * dt * apply_H(model, cur)
        prev, cur = cur, nxt
    return (cur, prev) if return_previous else cur


# --------------------------------------------------------------- diabatic representation


def diabatic_to_adiabatic(W: np.ndarray, dW: np.ndarray):
    """Two-state diabatic -> adiabatic (Sec. II.F, Eqs. 24-28) for W = (W11, W22, W12)
    and its derivatives dW on a grid.  Returns (V, F12, cos, sin):
      V = (V_1, V_2) = Wbar +- sqrt((Delta W / 2)^2 + W12^2), Delta W = W22 - W11;
      O(q) of Eq. (26) is the rotation by theta with cos = W12 / n, sin = Delta / n,
      Delta = V_1 - W11, i.e. tan(theta) = Delta / W12, equivalently
      tan(2 theta) = 2 W12 / (W11 - W22) (theta in (0, pi/2) where W12 > 0);
      F = O^T O' (Eq. 27) gives F12 = -theta' = (Delta W W12' - W12 Delta W') /
      (Delta W^2 + 4 W12^2), which is Eq. (28) rewritten without the cancellation in
      Delta = V_1 - W11 far from the crossing.
    The adiabatic state is psi = O^T psi_diab (Eq. 25): psi_1 = cos d1 + sin d2,
    psi_2 = -sin d1 + cos d2."""
    W11, W22, W12 = W
    dW11, dW22, dW12 = dW
    wbar = 0.5 * (W11 + W22)
    dw = W22 - W11
    r = np.sqrt((0.5 * dw) ** 2 + W12 ** 2)
    V = np.stack([wbar + r, wbar - r])
    theta = 0.5 * np.arctan2(2.0 * W12, W11 - W22)
    ddw = dW22 - dW11
    F12 = (dw * dW12 - W12 * ddw) / (dw * dw + 4.0 * W12 * W12)
    return V, F12, np.cos(theta), np.sin(theta)


def to_adiabatic(psi_diab: np.ndarray, c: np.ndarray, s: np.ndarray) -> np.ndarray:
    """psi = O(q)^T psi_diab pointwise (Eq. 25)."""
    d1, d2 = psi_diab
    return np.stack([c * d1 + s * d2, -s * d1 + c * d2])


def apply_H_diabatic(n: int, qmin: float, qmax: float, mass: float, W: np.ndarray,
                     psi: np.ndarray) -> np.ndarray:
    """H_diab psi = p^2/(2m) psi + W psi (the diabatic Hamiltonian of Sec. II.F)."""
    p = momentum_grid(n, qmax - qmin)
    kin = np.fft.ifft((p * p / (2.0 * mass)) * np.fft.fft(psi, axis=-1), axis=-1)
    W11, W22, W12 = W
    return kin + np.stack([W11 * psi[0] + W12 * psi[1], W12 * psi[0] + W22 * psi[1]])


def exp_W(W: np.ndarray, psi: np.ndarray, tau: float) -> np.ndarray:
    """exp(-i W(q) tau) applied pointwise, from the eigendecomposition of each 2 x 2
    W(q) (a library eigensolver as a step)."""
    W11, W22, W12 = W
    M = np.stack([np.stack([W11, W12], -1), np.stack([W12, W22], -1)], -2)  # (n, 2, 2)
    lam, U = np.linalg.eigh(M)
    E = U @ (np.exp(-1j * tau * lam)[..., None] * np.swapaxes(U, -1, -2))
    return np.einsum("nij,jn->in", E, psi)


def exp_T(n: int, qmin: float, qmax: float, mass: float, psi: np.ndarray, tau: float) -> np.ndarray:
    """exp(-i p^2 tau / 2m) on both components, diagonal in the Fourier basis."""
    p = momentum_grid(n, qmax - qmin)
    return np.fft.ifft(np.exp(-1j * tau * p * p / (2.0 * mass)) * np.fft.fft(psi, axis=-1), axis=-1)


def split_operator_step(n, qmin, qmax, mass, W, psi, h: float) -> np.ndarray:
    """The standard second-order (Strang) splitting the paper lists among its reference
    methods (Table I): exp(-i W h/2) exp(-i T h) exp(-i W h/2)."""
    psi = exp_W(W, psi, 0.5 * h)
    psi = exp_T(n, qmin, qmax, mass, psi, h)
    return exp_W(W, psi, 0.5 * h)


def split_operator_propagate(n, qmin, qmax, mass, W, psi0: np.ndarray, scheme: str, order: int,
                             dt: float, nsteps: int) -> np.ndarray:
    """nsteps steps of the split-operator step composed like the implicit methods
    (Sec. II.D): substep c has length tau_c dt, in list order."""
    psi = np.array(psi0, dtype=np.complex128, copy=True)
    taus = substep_fractions(scheme, order)
    for _ in range(nsteps):
        for t in taus:
            psi = split_operator_step(n, qmin, qmax, mass, W, psi, t * dt)
    return psi


# ---------------------------------------------------------------------------- adjoint


def adjoint(model: Model, psi_T: np.ndarray, lam_T: np.ndarray, scheme: str, order: int,
            dt: float, nsteps: int, opts: SolverOpts, stats: Optional[Stats] = None):
    """Reverse sweep for a real loss L(psi(T)).

    Input lam_T = dL/dpsi*(T) in the Euclidean sense (dL = 2 Re sum conj(lam) dpsi).
    Returns (psi(0) reconstructed, lam(0) = dL/dpsi*(0), dL/dF12 on the grid, shape (D, *n)).

    Each substep of length h (a = h/2) is the Cayley map C = (1 + iaH)^-1 (1 - iaH)
    = 2 (1 + iaH)^-1 - 1, shared by the trapezoidal rule and the implicit midpoint
    method (Sec. II.C).  Its inverse and its adjoint are both 2 (1 - iaH)^-1 - 1
    (unitarity, Eq. A13-A14; time reversibility, Eq. A40), so with
    phi = (1 - iaH)^-1 psi_after and mu = (1 - iaH)^-1 lam_after:
        psi_before = 2 phi - psi_after,  lam_before = 2 mu - lam_after,
    and, from dC = -2 i a (1 + iaH)^-1 dH (1 + iaH)^-1 with dH = (1/2m)(dA A + A dA),
    dA = -i dF, the F12 gradient at grid point j gains
        -(2 a / m_d) Re[conj(mu_1)(A phi)_2 - conj(mu_2)(A phi)_1
                        + conj(A mu)_1 phi_2 - conj(A mu)_2 phi_1]_j.
    Both solves use GMRES with the explicit-Euler guess for step -a."""
    stats = stats if stats is not None else Stats()
    taus = substep_fractions(scheme, order)
    psi = np.array(psi_T, dtype=np.complex128, copy=True)
    lam = np.array(lam_T, dtype=np.complex128, copy=True)
    gF = np.zeros((model.D,) + model.n)
    for _ in range(nsteps):
        for tau in reversed(taus):
            a = 0.5 * (tau * dt)
            phi = implicit_euler(model, psi, -a, opts, stats)
            mu = implicit_euler(model, lam, -a, opts, stats)
            for d in range(model.D):
                Aphi = apply_A(model, phi, d)
                Amu = apply_A(model, mu, d)
                term = (np.conj(mu[0]) * Aphi[1] - np.conj(mu[1]) * Aphi[0]
                        + np.conj(Amu[0]) * phi[1] - np.conj(Amu[1]) * phi[0])
                gF[d] += -(2.0 * a / model.mass[d]) * term.real
            psi = 2.0 * phi - psi
            lam = 2.0 * mu - lam
    return psi, lam, gF


def population_loss(model: Model, psi: np.ndarray, surface: int = 1) -> Tuple[float, np.ndarray]:
    """L = P_surface(psi) and its Euclidean gradient dL/dpsi* = dv * Pi_surface psi."""
    lam = np.zeros_like(psi)
    lam[surface] = model.dv * psi[surface]
    return float(populations(model, psi)[surface]), lam
