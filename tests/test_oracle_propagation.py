"""Pins for the oracle's GMRES solve, the trapezoidal/midpoint steps and composed
propagation: dense linear algebra, exact solutions, and the invariants the paper
proves (Sec. II.A-C, Theorem of Sec. II.D, App. A) with the bound it prints."""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_1902_04661_amd import inputs as I

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def small_model(n=16, L=6.0, M=10.0):
    q = np.arange(n) * L / n
    V = np.stack([0.5 * np.cos(2 * math.pi * q / L), 0.3 * np.sin(2 * math.pi * q / L) + 0.2])
    F = 0.4 * np.exp(-((q - 3) / 1.0) ** 2)
    m = O.Model((n,), (0.0,), (L,), (M,), V, F[None])
    psi0 = np.stack([np.exp(-(q - 3) ** 2), 0 * q]).astype(complex)
    return m, psi0 / np.linalg.norm(psi0)


# ------------------------------------------------------------------------------ GMRES

def test_givens_rotation_zeroes_second_component():
    for a, b in [(1 + 2j, 0.5), (-0.3j, 3.0), (0j, 2.0), (1.5, 0.0)]:
        c, s, r = O.givens(a, b)
        assert abs(c * c + abs(s) ** 2 - 1) < 1e-15
        assert abs(c * a + s * b - r) < 1e-15
        assert abs(-np.conj(s) * a + c * b) < 1e-15


@pytest.mark.parametrize("m", [64, 3])
def test_gmres_matches_dense_solve(m):
    rng = np.random.default_rng(11)
    n = 40
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    Hm = (A + A.conj().T) / 2
    a = 0.37
    X = np.eye(n) + 1j * a * Hm
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, info = O.gmres(lambda v: X @ v, b, b - 1j * a * (Hm @ b), 1e-14, m, 2000)
    assert info.converged
    ref = np.linalg.solve(X, b)
    assert np.linalg.norm(x - ref) <= 1e-13 * np.linalg.norm(ref)
    assert np.linalg.norm(b - X @ x) <= 2e-14 * np.linalg.norm(b)


def test_gmres_nonnormal_and_failure_flag():
    rng = np.random.default_rng(12)
    n = 30
    X = np.eye(n) * 3 + rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    b = rng.standard_normal(n) + 0j
    x, info = O.gmres(lambda v: X @ v, b, np.zeros(n, complex), 1e-13, 64, 200)
    assert info.converged and np.linalg.norm(x - np.linalg.solve(X, b)) < 1e-11
    x, info = O.gmres(lambda v: X @ v, b, np.zeros(n, complex), 1e-13, 64, 1)
    assert not info.converged and info.iterations == 1


def test_gmres_zero_rhs_returns_zero_without_iterations():
    x, info = O.gmres(lambda v: 2 * v, np.zeros(5, complex), np.zeros(5, complex), 1e-13, 8, 10)
    assert info.converged and info.iterations == 0 and not np.any(x)


def test_implicit_euler_is_the_inverse_of_one_plus_i_eps_h():
    m, psi0 = small_model()
    H = O.dense_H(m)
    for eps in [0.5, -2.0, 30.0]:
        x = O.implicit_euler(m, psi0, eps, O.SolverOpts(tol=1e-15))
        ref = np.linalg.solve(np.eye(H.shape[0]) + 1j * eps * H, psi0.ravel())
        assert np.linalg.norm(x.ravel() - ref) < 1e-13


# ---------------------------------------------------------------------- single steps

@pytest.mark.parametrize("method", [O.TRAP, O.MIDP])
@pytest.mark.parametrize("literal", [False, True])
def test_step_is_the_cayley_transform(method, literal):
    # Sec. II.C: both methods are the Cayley transform (1 + iaH)^-1 (1 - iaH), a = h/2.
    m, psi0 = small_model()
    H = O.dense_H(m)
    w, Q = np.linalg.eigh(H)
    for h in [0.3, 7.0, -4.0]:
        a = 0.5 * h
        ref = Q @ ((1 - 1j * a * w) / (1 + 1j * a * w) * (Q.conj().T @ psi0.ravel()))
        opts = O.SolverOpts(tol=1e-15, literal=literal)
        out = (O.trapezoidal_step(m, psi0, h, opts)[0] if method == O.TRAP
               else O.midpoint_step(m, psi0, h, opts))
        assert np.linalg.norm(out.ravel() - ref) < 1e-13


def test_trapezoid_and_midpoint_agree_to_solver_tolerance():
    it = I.nai_like_item(256, p0=2.5)
    m = O.model_from_item(it)
    opts = O.SolverOpts(tol=1e-15)
    a = O.propagate(m, it.psi0, O.TRAP, O.SUZUKI, 4, 10.0, 5, opts)
    b = O.propagate(m, it.psi0, O.MIDP, O.SUZUKI, 4, 10.0, 5, opts)
    assert np.linalg.norm(a - b) < 1e-13


@pytest.mark.parametrize("method", [O.TRAP, O.MIDP])
def test_literal_mode_costs_three_plus_I_applies_per_substep(method):
    # Table I: 4D(3 + I)C Fourier transforms per step, i.e. 3 + I H-applications per substep.
    assert GOLDEN["cost_per_step"]["h_applies_per_substep_literal"] == "3 + I"
    it = I.nai_like_item(256, p0=1.0)
    m = O.model_from_item(it)
    st = O.Stats()
    O.propagate(m, it.psi0, method, O.TRIPLE_JUMP, 4, 8.0, 2, O.SolverOpts(tol=1e-13, literal=True), st)
    assert st.solves == 6
    assert st.h_applies == sum(3 + i for i in st.per_solve)
    st2 = O.Stats()
    O.propagate(m, it.psi0, method, O.TRIPLE_JUMP, 4, 8.0, 2, O.SolverOpts(tol=1e-13), st2)
    # economy mode saves the explicit half-step (midpoint) or reuses H psi (trapezoid)
    assert st2.h_applies == sum(2 + i for i in st2.per_solve) + (1 if method == O.TRAP else 0)


# ----------------------------------------------------------------- composed propagation

ORDER_CASES = [(O.TRIPLE_JUMP, 2, range(5, 9)), (O.TRIPLE_JUMP, 4, range(5, 9)),
               (O.TRIPLE_JUMP, 6, range(5, 9)), (O.SUZUKI, 4, range(2, 6)),
               (O.SUZUKI, 6, range(2, 6)), (O.SUZUKI, 8, range(0, 4)),
               (O.OPTIMAL, 4, range(2, 6)), (O.OPTIMAL, 6, range(3, 8)), (O.OPTIMAL, 8, range(2, 6)),
               (O.OPTIMAL, 10, range(1, 6))]
# smallest acceptable largest slope: at eighth and tenth order the error reaches the
# rounding floor before the slope reaches its asymptotic value
MIN_SLOPE = {2: 1.5, 4: 3.5, 6: 5.5, 8: 7.0, 10: 8.5}


@pytest.mark.parametrize("scheme,order,ks", ORDER_CASES)
def test_global_order_against_exact_evolution(scheme, order, ks):
    m, psi0 = small_model()
    H = O.dense_H(m)
    w, Q = np.linalg.eigh(H)
    T = 8.0
    ex = Q @ (np.exp(-1j * w * T) * (Q.conj().T @ psi0.ravel()))
    errs = []
    for k in ks:
        out = O.propagate(m, psi0, O.MIDP, scheme, order, T / 2 ** k, 2 ** k, O.SolverOpts(tol=1e-15))
        errs.append(np.linalg.norm(out.ravel() - ex))
    slopes = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)
              if errs[i + 1] > 2e-11]
    assert max(slopes) >= MIN_SLOPE[order], (errs, slopes)
    assert max(slopes) <= order + 0.5, (errs, slopes)


def test_free_particle_grid_exact_and_continuum_spreading():
    n, qmin, qmax, M = 256, -40.0, 40.0, 1.0
    q = I.uniform_grid(n, qmin, qmax)
    m = O.Model((n,), (qmin,), (qmax,), (M,), np.zeros((2, n)), np.zeros((1, n)))
    q0, p0, s = -5.0, 1.5, 0.8
    psi0 = I.gaussian_packet_1d(q, q0, p0, s)
    dt, nsteps, order = 0.25, 32, 6
    out = O.propagate(m, psi0, O.MIDP, O.SUZUKI, order, dt, nsteps, O.SolverOpts(tol=1e-15))
    # grid-exact: each k-mode picks up prod_c (1 - i a_c E_k)/(1 + i a_c E_k)
    E = O.momentum_grid(n, qmax - qmin) ** 2 / (2 * M)
    fac = np.ones(n, complex)
    for _ in range(nsteps):
        for t in O.substep_fractions(O.SUZUKI, order):
            a = 0.5 * t * dt
            fac *= (1 - 1j * a * E) / (1 + 1j * a * E)
    ref = np.fft.ifft(fac * np.fft.fft(psi0[0]))
    assert np.linalg.norm(out[0] - ref) < 1e-12 * np.linalg.norm(ref)
    # continuum: <q> = q0 + p0 t/M, var q = s^2 (1 + (t/(2 M s^2))^2)
    t = dt * nsteps
    dq = q[1] - q[0]
    rho = np.abs(out[0]) ** 2 * dq
    mean = np.sum(q * rho)
    var = np.sum((q - mean) ** 2 * rho)
    # (limited by the time-step error of the packet's own modes, ~1e-5 here)
    assert abs(mean - (q0 + p0 * t / M)) < 1e-4
    assert abs(var - s * s * (1 + (t / (2 * M * s * s)) ** 2)) < 1e-3


def test_harmonic_coherent_state_follows_classical_trajectory():
    n, qmin, qmax, M, w, qc = 256, -10.0, 10.0, 1.0, 1.0, 0.0
    q = I.uniform_grid(n, qmin, qmax)
    V = 0.5 * M * w * w * (q - qc) ** 2
    m = O.Model((n,), (qmin,), (qmax,), (M,), np.stack([V, V]), np.zeros((1, n)))
    q0, p0 = 1.5, 0.7
    s = math.sqrt(1 / (2 * M * w))           # ground-state width: a coherent state
    psi0 = I.gaussian_packet_1d(q, q0, p0, s)
    dt, nsteps = 0.1, 40
    out = O.propagate(m, psi0, O.MIDP, O.SUZUKI, 6, dt, nsteps, O.SolverOpts(tol=1e-15))
    t = dt * nsteps
    rho = np.abs(out[0]) ** 2 * (q[1] - q[0])
    mean = np.sum(q * rho)
    # (time-step error of the sixth-order scheme at dt = 0.1 is ~1e-8)
    assert abs(mean - (qc + (q0 - qc) * math.cos(w * t) + p0 / (M * w) * math.sin(w * t))) < 1e-7
    # the width of a coherent state does not change
    assert abs(np.sum((q - mean) ** 2 * rho) - s * s) < 1e-7


# ------------------------------------------------------------------------ invariants

@pytest.mark.parametrize("method", [O.TRAP, O.MIDP])
@pytest.mark.parametrize("scheme,order", [(O.SUZUKI, 2), (O.TRIPLE_JUMP, 4), (O.SUZUKI, 4)])
def test_geometric_invariants_within_paper_bound(method, scheme, order):
    # Fig. 7 set-up: phi(0) with q0 = 5.05, p0 = 2.5 and the width of psi(0); dt = 5 a.u.
    g = GOLDEN["fig7_second_state"]
    bound = GOLDEN["invariant_residual_bound"]["bound"]
    it = I.nai_like_item(256)
    m = O.model_from_item(it)
    phi0 = I.gaussian_packet_1d(it.q, g["q0"], g["p0"], it.params["width"])
    dt, nsteps = g["dt_geometric"], 40
    opts = O.SolverOpts(tol=1e-15)
    psi = O.propagate(m, it.psi0, method, scheme, order, dt, nsteps, opts)
    phi = O.propagate(m, phi0, method, scheme, order, dt, nsteps, opts)
    assert abs(O.norm(m, psi) - O.norm(m, it.psi0)) < bound
    assert abs(O.energy(m, psi) - O.energy(m, it.psi0)) < bound
    assert abs(O.symplectic_form(m, psi, phi) - O.symplectic_form(m, it.psi0, phi0)) < bound
    back = O.propagate(m, psi, method, scheme, order, -dt, nsteps, opts)
    assert math.sqrt(abs(O.inner(m, back - it.psi0, back - it.psi0))) < bound


def test_euler_methods_fail_norm_conservation_as_the_paper_derives():
    it = I.nai_like_item(256, p0=2.5)
    m = O.model_from_item(it)
    eps = GOLDEN["fig7_second_state"]["dt_euler"]
    H2 = O.inner(m, O.apply_H(m, it.psi0), O.apply_H(m, it.psi0)).real   # <H^2>
    n0 = O.norm(m, it.psi0) ** 2
    e1 = O.explicit_euler(m, it.psi0, eps)
    # Eq. (A19) holds exactly: ||(1 - i eps H) psi||^2 = ||psi||^2 + eps^2 <H^2>
    assert abs(O.norm(m, e1) ** 2 - (n0 + eps * eps * H2)) < 1e-15
    i1 = O.implicit_euler(m, it.psi0, eps, O.SolverOpts(tol=1e-15))
    # Eq. (A20): decrease by eps^2 <H^2> to leading order
    d = O.norm(m, i1) ** 2 - n0
    assert GOLDEN["euler_norm_change"]["implicit_sign"] * d > 0
    assert abs(d + eps * eps * H2) < 0.05 * eps * eps * H2
    # long runs: explicit Euler's norm grows without bound, implicit Euler's decays
    ex = O.explicit_euler_propagate(m, it.psi0, 5.0, 200)
    im = O.implicit_euler_propagate(m, it.psi0, 5.0, 200, O.SolverOpts(tol=1e-13))
    assert O.norm(m, ex) > 1.0 + 1e-3 and O.norm(m, im) < 1.0 - 1e-3


def test_two_dimensional_propagation_against_exact_evolution():
    n1, n2 = 8, 8
    L1, L2 = 6.0, 5.0
    q1 = np.arange(n1) * L1 / n1
    q2 = np.arange(n2) * L2 / n2
    Q1, Q2 = np.meshgrid(q1, q2, indexing="ij")
    V = np.stack([0.1 * np.cos(2 * math.pi * Q1 / L1) + 0.05 * np.sin(2 * math.pi * Q2 / L2),
                  0.2 + 0.03 * np.cos(2 * math.pi * (Q1 / L1 + Q2 / L2))])
    g = 0.3 * np.exp(-((Q1 - 3) ** 2 + (Q2 - 2.5) ** 2))
    F = np.stack([0.8 * g, 0.6 * g])
    m = O.Model((n1, n2), (0.0, 0.0), (L1, L2), (10.0, 12.0), V, F)
    psi0 = np.zeros((2, n1, n2), complex)
    psi0[0] = np.exp(-((Q1 - 3) ** 2 + (Q2 - 2.5) ** 2))
    psi0 /= np.linalg.norm(psi0)
    H = O.dense_H(m)
    w, Q = np.linalg.eigh(H)
    T = 4.0
    ex = Q @ (np.exp(-1j * w * T) * (Q.conj().T @ psi0.ravel()))
    errs = []
    for k in [3, 4, 5]:
        out = O.propagate(m, psi0, O.MIDP, O.SUZUKI, 4, T / 2 ** k, 2 ** k, O.SolverOpts(tol=1e-15))
        errs.append(np.linalg.norm(out.ravel() - ex))
    assert errs[-1] < 1e-7
    assert math.log2(errs[-2] / errs[-1]) > 3.5
