"""Pins of the oracle's second-order differencing (Eq. 16) and its Runge-Kutta start
(Sec. III): a closed form on spinor eigenstates, the two quantities App. A proves exactly
conserved (Eqs. A21 and A32), the second-order global error against exact evolution, the
fourth-order norm and energy errors (Propositions 5 and 6), and the stability bound of
Eq. (A48)."""
import math

import numpy as np
import scipy.linalg

import oracle as O
from paper_1902_04661_amd import inputs as I


def constant_coupling_model(n=64, qmin=0.0, qmax=10.0, M=2.0, f=0.3, v=0.01):
    m = O.Model((n,), (qmin,), (qmax,), (M,), v * np.ones((2, n)), f * np.ones((1, n)))
    return m, I.uniform_grid(n, qmin, qmax), qmax - qmin, M, f, v


def test_sod_on_spinor_eigenstates_closed_form():
    # with constant F and V, the spinors (e^{ipq}, +-i e^{ipq}) are eigenstates with
    # E = (p +- f)^2 / 2M + v; on each, SOD is the scalar recurrence
    # c_{n+1} = c_{n-1} - 2 i dt E c_n with c_0 = 1 and c_{-1} = 1 + i dt E - (dt E)^2 / 2
    # M = 20 keeps E_max ~ 2.5 on this grid, so dt = 0.1 is inside the stable range (A48)
    m, q, L, M, f, v = constant_coupling_model(n=32, M=20.0)
    rng = np.random.default_rng(5)
    psi = np.zeros((2, q.size), complex)
    comps = []
    for mode in [-4, -1, 0, 3]:
        for sign in [+1, -1]:
            cf = rng.standard_normal() + 1j * rng.standard_normal()
            p = 2 * math.pi * mode / L
            vec = np.stack([np.exp(1j * p * q), sign * 1j * np.exp(1j * p * q)])
            comps.append((cf, vec, (p + sign * f) ** 2 / (2 * M) + v))
            psi += cf * vec
    dt, nsteps = 0.1, 60
    out, prev = O.sod_propagate(m, psi, dt, nsteps, return_previous=True)
    ref = np.zeros_like(psi)
    ref_prev = np.zeros_like(psi)
    for cf, vec, E in comps:
        c_prev, c = 1 + 1j * dt * E - 0.5 * (dt * E) ** 2, 1.0 + 0j
        for _ in range(nsteps):
            c_prev, c = c, c_prev - 2j * dt * E * c
        ref += cf * c * vec
        ref_prev += cf * c_prev * vec
    scale = np.linalg.norm(ref)
    assert np.linalg.norm(out - ref) < 1e-13 * scale
    assert np.linalg.norm(prev - ref_prev) < 1e-13 * scale


def test_sod_start_is_the_second_order_taylor_step_backwards():
    m, q, L, M, f, v = constant_coupling_model(n=32, M=20.0)
    rng = np.random.default_rng(6)
    psi = rng.standard_normal((2, 32)) + 1j * rng.standard_normal((2, 32))
    H = O.dense_H(m)
    dt = 0.3
    ref = psi.ravel() + 1j * dt * (H @ psi.ravel()) - 0.5 * dt * dt * (H @ (H @ psi.ravel()))
    assert np.allclose(O.sod_start(m, psi, dt).ravel(), ref, rtol=0, atol=1e-14 * np.linalg.norm(ref))
    # and it approximates exact backward evolution to third order in dt
    for d in (0.04, 0.02):
        ex = scipy.linalg.expm(1j * d * H) @ psi.ravel()
        err = np.linalg.norm(O.sod_start(m, psi, d).ravel() - ex)
        if d == 0.04:
            e1 = err
    assert 6.0 < e1 / err < 10.0


def test_sod_conserves_the_inner_product_and_energy_analogues():
    # Eq. (A21): (<psi(t)|phi(t - dt)> + <psi(t - dt)|phi(t)>) / 2 is conserved, and with
    # phi = psi, Re <psi(t)|psi(t - dt)>; Eq. (A32): Re <psi(t)|H|psi(t + dt)> is conserved
    it = I.nai_like_item(256, p0=2.5)
    m = O.model_from_item(it)
    phi0 = I.gaussian_packet_1d(it.q, 5.05, 2.5, 0.12)
    dt = 0.2
    seq_psi = [(O.sod_start(m, it.psi0, dt)), it.psi0]
    seq_phi = [(O.sod_start(m, phi0, dt)), phi0]
    for _ in range(60):
        seq_psi.append(seq_psi[-2] - 2j * dt * O.apply_H(m, seq_psi[-1]))
        seq_phi.append(seq_phi[-2] - 2j * dt * O.apply_H(m, seq_phi[-1]))
    # the recurrence above is Eq. (16) retyped; pin sod_propagate to it first
    assert np.array_equal(O.sod_propagate(m, it.psi0, dt, 60), seq_psi[-1])
    a21 = [0.5 * (O.inner(m, seq_psi[k], seq_phi[k - 1]) + O.inner(m, seq_psi[k - 1], seq_phi[k]))
           for k in range(1, len(seq_psi))]
    norm_like = [O.inner(m, seq_psi[k], seq_psi[k - 1]).real for k in range(1, len(seq_psi))]
    a32 = [O.inner(m, seq_psi[k], O.apply_H(m, seq_psi[k + 1])).real for k in range(1, len(seq_psi) - 1)]
    assert max(abs(x - a21[0]) for x in a21) < 1e-13 * abs(a21[0])
    assert max(abs(x - norm_like[0]) for x in norm_like) < 1e-13
    assert max(abs(x - a32[0]) for x in a32) < 1e-13 * abs(a32[0])


def test_sod_global_errors_have_the_orders_of_propositions_5_and_6():
    # small dense problem: the state error is second order, norm and energy fourth order
    n = 32
    m, q, L, M, f, v = constant_coupling_model(n=n, M=5.0)
    m.V[1] += 0.05 * np.cos(2 * math.pi * q / L)
    m.F[0] = 0.3 * np.exp(-((q - 5.0) / 1.5) ** 2)
    psi0 = np.stack([np.exp(-((q - 4.0) ** 2) / 2 + 1j * 0.8 * q), np.zeros(n)])
    psi0 /= O.norm(m, psi0)
    H = O.dense_H(m)
    T = 4.0
    ex = (scipy.linalg.expm(-1j * T * H) @ psi0.ravel()).reshape(2, n)
    E0 = O.energy(m, psi0)
    errs = []
    for k in (0, 1):
        dt = 0.05 / 2 ** k
        out = O.sod_propagate(m, psi0, dt, int(round(T / dt)))
        errs.append((np.linalg.norm(out - ex), abs(O.norm(m, out) - 1.0), abs(O.energy(m, out) - E0)))
    r_state = errs[0][0] / errs[1][0]
    r_norm = errs[0][1] / errs[1][1]
    r_energy = errs[0][2] / errs[1][2]
    assert 3.5 < r_state < 4.5
    assert 12.0 < r_norm < 20.0
    assert 12.0 < r_energy < 20.0


def test_sod_is_stable_only_below_the_critical_step():
    # Eq. (A48): stable for dt < 1 / E_max, E_max the largest |eigenvalue| of H
    m, q, L, M, f, v = constant_coupling_model(n=32, M=1.0)
    H = O.dense_H(m)
    emax = np.abs(np.linalg.eigvalsh(H)).max()
    rng = np.random.default_rng(7)
    psi = rng.standard_normal((2, 32)) + 1j * rng.standard_normal((2, 32))
    psi /= O.norm(m, psi)
    below = O.sod_propagate(m, psi, 0.95 / emax, 400)
    above = O.sod_propagate(m, psi, 1.05 / emax, 400)
    assert O.norm(m, below) < 2.0
    assert O.norm(m, above) > 1e6
