"""Pins for the oracle's reverse (adjoint) sweep: central finite differences of the
surface-2 population and exact reconstruction of psi(0) by time reversibility (Eq. A40)."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1902_04661_amd import inputs as I

N, QMIN, QMAX, MASS = 128, 3.0, 16.0, 200.0
BASE = dict(q0=6.0, p0=8.0, w=0.3, amp=0.4, center=7.0)
OPTS = O.SolverOpts(tol=1e-15)
DT, NSTEPS, SCHEME, ORDER = 4.0, 10, O.SUZUKI, 4


def build(q0, p0, w, amp, center):
    q = I.uniform_grid(N, QMIN, QMAX)
    V = np.stack([I.morse(q), I.repulsive(q)])
    F = I.coupling(q, amp, center, 0.5)[None]
    return O.Model((N,), (QMIN,), (QMAX,), (MASS,), V, F), I.gaussian_packet_1d(q, q0, p0, w)


def loss(**kw):
    p = dict(BASE, **kw)
    m, psi0 = build(**p)
    psi = O.propagate(m, psi0, O.MIDP, SCHEME, ORDER, DT, NSTEPS, OPTS)
    return O.population_loss(m, psi)[0]


@pytest.fixture(scope="module")
def sweep():
    m, psi0 = build(**BASE)
    psiT = O.propagate(m, psi0, O.MIDP, SCHEME, ORDER, DT, NSTEPS, OPTS)
    _, lam = O.population_loss(m, psiT)
    psiR, lam0, gF = O.adjoint(m, psiT, lam, SCHEME, ORDER, DT, NSTEPS, OPTS)
    return m, psi0, psiR, lam0, gF


def test_reverse_sweep_reconstructs_initial_state(sweep):
    m, psi0, psiR, _, _ = sweep
    assert math.sqrt(abs(O.inner(m, psiR - psi0, psiR - psi0))) < 2e-12


@pytest.mark.parametrize("name", ["amp", "center"])
def test_coupling_parameter_gradients_match_central_differences(sweep, name):
    m, _, _, _, gF = sweep
    q = I.uniform_grid(N, QMIN, QMAX)
    F = I.coupling(q, BASE["amp"], BASE["center"], 0.5)
    dF = F / BASE["amp"] if name == "amp" else F * 2 * (q - BASE["center"]) / 0.25
    g = float(np.sum(gF[0] * dF))
    h = 1e-5
    fd = (loss(**{name: BASE[name] + h}) - loss(**{name: BASE[name] - h})) / (2 * h)
    assert abs(g - fd) < 1e-6 * abs(fd)


@pytest.mark.parametrize("name", ["q0", "p0", "w"])
def test_initial_state_parameter_gradients_match_central_differences(sweep, name):
    _, _, _, lam0, _ = sweep
    e = 1e-6
    dpsi = (build(**dict(BASE, **{name: BASE[name] + e}))[1]
            - build(**dict(BASE, **{name: BASE[name] - e}))[1]) / (2 * e)
    g = 2 * np.real(np.vdot(lam0.ravel(), dpsi.ravel()))
    h = 1e-5
    fd = (loss(**{name: BASE[name] + h}) - loss(**{name: BASE[name] - h})) / (2 * h)
    assert abs(g - fd) < 1e-6 * abs(fd)


def test_pointwise_coupling_gradient_matches_central_differences(sweep):
    m, psi0, _, _, gF = sweep
    j = int(np.argmax(np.abs(gF[0])))
    h = 1e-6
    def L_with(delta):
        F = m.F.copy()
        F[0, j] += delta
        mm = O.Model(m.n, m.qmin, m.qmax, m.mass, m.V, F)
        psi = O.propagate(mm, psi0, O.MIDP, SCHEME, ORDER, DT, NSTEPS, OPTS)
        return O.population_loss(mm, psi)[0]
    fd = (L_with(h) - L_with(-h)) / (2 * h)
    assert abs(gF[0, j] - fd) < 1e-5 * abs(fd)


def test_adjoint_is_the_same_for_trapezoid_forward_sweep():
    # both base methods share the Cayley map, so the reverse sweep is method independent
    m, psi0 = build(**BASE)
    psiT = O.propagate(m, psi0, O.TRAP, SCHEME, ORDER, DT, NSTEPS, OPTS)
    _, lam = O.population_loss(m, psiT)
    psiR, lam0, gF = O.adjoint(m, psiT, lam, SCHEME, ORDER, DT, NSTEPS, OPTS)
    assert math.sqrt(abs(O.inner(m, psiR - psi0, psiR - psi0))) < 2e-12
    d = np.random.default_rng(5).standard_normal(psi0.shape) * (1 + 0j)
    h = 1e-6
    fd = (O.population_loss(m, O.propagate(m, psi0 + h * d, O.TRAP, SCHEME, ORDER, DT, NSTEPS, OPTS))[0]
          - O.population_loss(m, O.propagate(m, psi0 - h * d, O.TRAP, SCHEME, ORDER, DT, NSTEPS, OPTS))[0]) / (2 * h)
    g = 2 * np.real(np.vdot(lam0.ravel(), d.ravel()))
    assert abs(g - fd) < 1e-6 * max(abs(fd), 1e-8)


def test_two_dimensional_coupling_gradients_match_central_differences():
    # 16 x 16 grid, distinct coupling components along q1 and q2: the sweep's dL/dF^(d)
    # against central differences, pointwise for each component and along a random
    # direction of both at once
    n, L1, L2 = 16, 6.0, 5.0
    q1 = np.arange(n) * L1 / n
    q2 = np.arange(n) * L2 / n
    Q1, Q2 = np.meshgrid(q1, q2, indexing="ij")
    V = np.stack([0.2 * (Q1 - 3) ** 2 + 0.1 * (Q2 - 2.5) ** 2,
                  0.3 + 0.1 * np.cos(2 * math.pi * Q1 / L1)])
    g = np.exp(-((Q1 - 3.2) ** 2 + (Q2 - 2.4) ** 2))
    F = np.stack([0.9 * g, -0.5 * g * (Q2 - 2.0)])
    m = O.Model((n, n), (0.0, 0.0), (L1, L2), (3.0, 4.0), V, F)
    psi0 = np.zeros((2, n, n), complex)
    psi0[0] = np.exp(-((Q1 - 2.8) ** 2 + (Q2 - 2.5) ** 2) + 0.7j * Q1)
    psi0 /= math.sqrt(m.dv * np.sum(np.abs(psi0) ** 2))
    dt, nsteps = 0.5, 6

    def L_of(Fx):
        mm = O.Model(m.n, m.qmin, m.qmax, m.mass, m.V, Fx)
        return O.population_loss(mm, O.propagate(mm, psi0, O.MIDP, SCHEME, ORDER, dt, nsteps, OPTS))[0]

    psiT = O.propagate(m, psi0, O.MIDP, SCHEME, ORDER, dt, nsteps, OPTS)
    _, lam = O.population_loss(m, psiT)
    psiR, _, gF = O.adjoint(m, psiT, lam, SCHEME, ORDER, dt, nsteps, OPTS)
    assert math.sqrt(abs(O.inner(m, psiR - psi0, psiR - psi0))) < 2e-12
    h = 1e-6
    for d in range(2):
        j = np.unravel_index(int(np.argmax(np.abs(gF[d]))), gF[d].shape)
        Fp, Fm = F.copy(), F.copy()
        Fp[(d,) + j] += h
        Fm[(d,) + j] -= h
        fd = (L_of(Fp) - L_of(Fm)) / (2 * h)
        assert abs(gF[(d,) + j] - fd) < 1e-5 * abs(fd)
    D = np.random.default_rng(11).standard_normal(F.shape)
    fd = (L_of(F + h * D) - L_of(F - h * D)) / (2 * h)
    assert abs(float(np.sum(gF * D)) - fd) < 1e-5 * abs(fd)
