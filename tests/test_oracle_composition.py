"""Pins for the composition schemes (Sec. II.D, Eqs. 20-21) and the elementary steps'
Taylor expansions (App. A, Eqs. A5-A7), against values the paper prints."""
import json
import math
import os

import mpmath
import numpy as np
import pytest

import oracle as O
from paper_1902_04661_amd import inputs as I

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def cplx(v):
    return complex(v[0], v[1])


@pytest.mark.parametrize("scheme,key", [(O.TRIPLE_JUMP, "triple_jump"), (O.SUZUKI, "suzuki")])
def test_substep_counts_match_paper(scheme, key):
    g = GOLDEN["substep_counts"]
    for order, count in zip(g["orders"], g[key]):
        assert len(O.substep_fractions(scheme, order)) == count


def test_suzuki_to_triple_jump_cost_ratio():
    g = GOLDEN["suzuki_vs_triple_jump_cost"]
    for order, ratio in zip(g["ratio_orders"], g["ratio"]):
        r = len(O.substep_fractions(O.SUZUKI, order)) / len(O.substep_fractions(O.TRIPLE_JUMP, order))
        assert abs(r - ratio) < 1e-12


@pytest.mark.parametrize("scheme", [O.TRIPLE_JUMP, O.SUZUKI])
@pytest.mark.parametrize("p", [2, 4, 6, 8])
def test_gammas_sum_symmetry_and_order_condition(scheme, p):
    gam = O.composition_gammas(scheme, p)
    assert abs(sum(gam) - GOLDEN["composition_sum"]["sum"]) < 1e-14
    assert gam == gam[::-1]
    # a symmetric composition of an order-p symmetric method gains two orders iff the
    # leading error terms cancel: sum_n gamma_n^(p+1) = 0 (Yoshida 1990; Suzuki 1990)
    assert abs(sum(g ** (p + 1) for g in gam)) < 1e-13


@pytest.mark.parametrize("scheme", [O.TRIPLE_JUMP, O.SUZUKI])
@pytest.mark.parametrize("order", [2, 4, 6, 8])
def test_flattened_fractions_sum_to_one_and_are_palindromic(scheme, order):
    taus = O.substep_fractions(scheme, order)
    assert abs(math.fsum(taus) - 1.0) < 1e-13
    assert np.allclose(taus, taus[::-1], rtol=0, atol=1e-15)


SCHEME_ORDERS = ([(s, o) for s in (O.TRIPLE_JUMP, O.SUZUKI) for o in (2, 4, 6, 8)]
                 + [(O.OPTIMAL, o) for o in (4, 6, 8, 10)])


@pytest.mark.parametrize("scheme,order", SCHEME_ORDERS)
def test_scalar_phase_error_has_the_composed_order(scheme, order):
    # On an eigenvector of H with eigenvalue E, each Cayley substep multiplies by
    # (1 - i a E)/(1 + i a E) = exp(-2 i atan(a E)); the composed step's phase error
    # sum_c 2 atan(tau_c x / 2) - x must vanish like x^(order+1), x = E dt.
    mpmath.mp.dps = 50
    taus = [mpmath.mpf(t) for t in O.substep_fractions(scheme, order)]
    def err(x):
        x = mpmath.mpf(x)
        return abs(sum(2 * mpmath.atan(t * x / 2) for t in taus) - x)
    # start where the error clears the fp64 rounding of the tau list (~1e-16) by 1000x
    x = 0.0125
    while err(x) < 1e-13:
        x *= 2
    slope = float(mpmath.log(err(2 * x) / err(x)) / mpmath.log(2))
    assert abs(slope - (order + 1)) < 0.35, slope


def constant_coupling_eigenstate(n=64, mode=5, sign=+1, M=2.0, f=0.3, v=0.01):
    qmin, qmax = 0.0, 10.0
    q = I.uniform_grid(n, qmin, qmax)
    p = 2 * math.pi * mode / (qmax - qmin)
    psi = np.stack([np.exp(1j * p * q), sign * 1j * np.exp(1j * p * q)]) / math.sqrt(2 * (qmax - qmin))
    m = O.Model((n,), (qmin,), (qmax,), (M,), v * np.ones((2, n)), f * np.ones((1, n)))
    E = (p + sign * f) ** 2 / (2 * M) + v
    return m, psi, E


@pytest.mark.parametrize("method", [O.TRAP, O.MIDP])
@pytest.mark.parametrize("literal", [False, True])
def test_step_taylor_expansion_matches_paper(method, literal):
    m, psi, E = constant_coupling_eigenstate()
    coef = [cplx(c) for c in GOLDEN["trap_midp_taylor"]["coefficients"]]
    lerr = cplx(GOLDEN["trap_midp_local_error"]["coefficient"])
    opts = O.SolverOpts(tol=1e-15, literal=literal)
    ratios = []
    for x in [0.2, 0.1, 0.05]:
        h = x / E
        if method == O.TRAP:
            out, _ = O.trapezoidal_step(m, psi, h, opts)
        else:
            out = O.midpoint_step(m, psi, h, opts)
        c = np.vdot(psi.ravel(), out.ravel()) / np.vdot(psi.ravel(), psi.ravel())
        poly = sum(coef[k] * x ** k for k in range(4))
        assert abs(c - poly) < 0.2 * x ** 4
        # local error vs exact evolution: i x^3/12 to leading order (Eq. A7 and text)
        ratios.append((c - complex(math.cos(x), -math.sin(x))) / x ** 3)
    assert abs(ratios[-1] - lerr) < 0.01


def test_implicit_euler_taylor_expansion_matches_paper():
    m, psi, E = constant_coupling_eigenstate()
    coef = [cplx(c) for c in GOLDEN["implicit_euler_taylor"]["coefficients"]]
    for x in [0.1, 0.05]:
        out = O.implicit_euler(m, psi, x / E, O.SolverOpts(tol=1e-15))
        c = np.vdot(psi.ravel(), out.ravel()) / np.vdot(psi.ravel(), psi.ravel())
        assert abs(c - sum(coef[k] * x ** k for k in range(4))) < 2 * x ** 4


@pytest.mark.parametrize("scheme,order", SCHEME_ORDERS)
def test_composed_propagation_on_constant_coupling_closed_form(scheme, order):
    # Superposition of k-space spinor eigenstates; each composed step multiplies each
    # component by prod_c (1 - i a_c E)/(1 + i a_c E), a_c = tau_c dt / 2.
    n, qmin, qmax, M, f, v = 64, 0.0, 10.0, 2.0, 0.3, 0.01
    q = I.uniform_grid(n, qmin, qmax)
    L = qmax - qmin
    m = O.Model((n,), (qmin,), (qmax,), (M,), v * np.ones((2, n)), f * np.ones((1, n)))
    rng = np.random.default_rng(order)
    comps = []
    psi = np.zeros((2, n), complex)
    for mode in [-3, 0, 2, 5]:
        for sign in [+1, -1]:
            cf = rng.standard_normal() + 1j * rng.standard_normal()
            p = 2 * math.pi * mode / L
            vec = np.stack([np.exp(1j * p * q), sign * 1j * np.exp(1j * p * q)])
            E = (p + sign * f) ** 2 / (2 * M) + v
            comps.append((cf, vec, E))
            psi += cf * vec
    dt, nsteps = 1.3, 3
    taus = O.substep_fractions(scheme, order)
    out = O.propagate(m, psi, O.MIDP, scheme, order, dt, nsteps, O.SolverOpts(tol=1e-15))
    ref = np.zeros_like(psi)
    for cf, vec, E in comps:
        fac = 1.0 + 0j
        for _ in range(nsteps):
            for t in taus:
                a = 0.5 * t * dt
                fac *= (1 - 1j * a * E) / (1 + 1j * a * E)
        ref += cf * fac * vec
    # roundoff grows with the number of substeps; a sign or order slip is O(1)
    assert np.linalg.norm(out - ref) < 2e-15 * len(taus) * nsteps * np.linalg.norm(ref) + 1e-14 * np.linalg.norm(ref)
