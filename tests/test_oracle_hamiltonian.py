"""Pins for the oracle's grid, dynamic Fourier method and Hamiltonian (Sec. II.E-F, Eq. 22).

Nothing here re-types the oracle's formulas: the expected values come from a dense DFT
matrix written out from its definition, from analytic derivatives of Gaussians, and from
the closed-form spectrum of a constant-coupling model."""
import cmath
import math

import numpy as np
import pytest

import oracle as O
from paper_1902_04661_amd import inputs as I


def dft_matrix(n):
    """W[k, j] = exp(-2 pi i j k / n), element by element."""
    return np.array([[cmath.exp(-2j * math.pi * j * k / n) for j in range(n)] for k in range(n)])


def model_1d(n, qmin, qmax, mass, V, F):
    return O.Model((n,), (qmin,), (qmax,), (mass,), V, F[None, :] if F.ndim == 1 else F)


@pytest.mark.parametrize("n", [8, 16, 32])
def test_momentum_operator_matches_dense_dft(n):
    L = 7.5
    W = dft_matrix(n)
    kp = [k if k < n // 2 else k - n for k in range(n)]
    p = np.array([2 * math.pi * k / L for k in kp])
    P_dense = (W.conj().T @ np.diag(p) @ W) / n
    m = model_1d(n, 0.0, L, 1.0, np.zeros((2, n)), np.zeros(n))
    rng = np.random.default_rng(n)
    psi = rng.standard_normal((2, n)) + 1j * rng.standard_normal((2, n))
    out = O.apply_P(m, psi, 0)
    ref = np.stack([P_dense @ psi[0], P_dense @ psi[1]])
    assert np.max(np.abs(out - ref)) < 1e-13 * np.max(np.abs(ref))


def test_plane_wave_eigenvalue_sign_and_nyquist():
    # p = -i d/dq: a plane wave exp(+i k q) has momentum +k; the Nyquist mode gets -pi n / L.
    n, qmin, qmax = 64, 3.0, 16.0
    L = qmax - qmin
    q = I.uniform_grid(n, qmin, qmax)
    m = model_1d(n, qmin, qmax, 1.0, np.zeros((2, n)), np.zeros(n))
    for mode in [1, 5, -7, 31]:
        k = 2 * math.pi * mode / L
        psi = np.stack([np.exp(1j * k * q), np.zeros(n)])
        out = O.apply_P(m, psi, 0)
        np.testing.assert_allclose(out[0], k * psi[0], atol=1e-12)
    nyq = np.stack([np.exp(1j * math.pi * np.arange(n)), np.zeros(n)])
    out = O.apply_P(m, nyq, 0)
    np.testing.assert_allclose(out[0], (-math.pi * n / L) * nyq[0], atol=1e-11)


def test_momentum_of_gaussian_is_minus_i_derivative():
    n, qmin, qmax = 512, 3.0, 16.0
    q = I.uniform_grid(n, qmin, qmax)
    c, s, p0 = 9.0, 0.3, 4.0
    g = np.exp(-(q - c) ** 2 / (4 * s * s) + 1j * p0 * (q - c))
    dg = (-(q - c) / (2 * s * s) + 1j * p0) * g
    m = model_1d(n, qmin, qmax, 1.0, np.zeros((2, n)), np.zeros(n))
    out = O.apply_P(m, np.stack([g, g]), 0)
    np.testing.assert_allclose(out[0], -1j * dg, atol=1e-10 * np.max(np.abs(dg)))


@pytest.mark.parametrize("n", [8, 16])
def test_hamiltonian_is_hermitian_and_matches_dense_assembly(n):
    rng = np.random.default_rng(100 + n)
    L, mass = 5.0, 1.7
    V = rng.standard_normal((2, n))
    f = rng.standard_normal(n)
    m = model_1d(n, 0.0, L, mass, V, f)
    H = O.dense_H(m)
    assert np.max(np.abs(H - H.conj().T)) < 1e-13 * np.max(np.abs(H))
    # independent assembly: A = P (x) 1_2 - i F, with F = [[0, f], [-f, 0]] pointwise
    W = dft_matrix(n)
    kp = [k if k < n // 2 else k - n for k in range(n)]
    P = (W.conj().T @ np.diag([2 * math.pi * k / L for k in kp]) @ W) / n
    Z = np.zeros((n, n))
    Fm = np.block([[Z, np.diag(f)], [-np.diag(f), Z]])
    A = np.kron(np.eye(2), P) - 1j * Fm
    Hd = A.conj().T @ A / (2 * mass) + np.diag(V.ravel())
    assert np.max(np.abs(H - Hd)) < 1e-12 * np.max(np.abs(Hd))


def test_factored_form_equals_expanded_continuum_operator():
    # H psi = -(1/2M)[psi'' + 2 F psi' + (F' + F^2) psi] + V psi for smooth fields,
    # derived from Eq. (22) with p = -i d/dq; F^2 = -f^2 1 for the 2x2 antisymmetric F.
    n, qmin, qmax, M = 512, 3.0, 16.0, 1.0
    q = I.uniform_grid(n, qmin, qmax)
    A0, cf, wf = 0.4, 8.0, 0.5
    f = A0 * np.exp(-((q - cf) / wf) ** 2)
    df = -2 * (q - cf) / wf ** 2 * f
    V = np.stack([0.01 * (q - 9) ** 2, 0.02 * np.ones(n)])
    def gauss(c, s, p):
        g = np.exp(-(q - c) ** 2 / (4 * s * s) + 1j * p * (q - c))
        d1 = (-(q - c) / (2 * s * s) + 1j * p)
        return g, d1 * g, (d1 * d1 - 1 / (2 * s * s)) * g
    g0, g0p, g0pp = gauss(8.2, 0.35, 3.0)
    g1, g1p, g1pp = gauss(7.7, 0.30, -2.0)
    psi = np.stack([g0, g1])
    ref0 = -(g0pp + 2 * f * g1p + df * g1 - f * f * g0) / (2 * M) + V[0] * g0
    ref1 = -(g1pp - 2 * f * g0p - df * g0 - f * f * g1) / (2 * M) + V[1] * g1
    out = O.apply_H(model_1d(n, qmin, qmax, M, V, f), psi)
    scale = np.max(np.abs(ref0)) + np.max(np.abs(ref1))
    assert np.max(np.abs(out[0] - ref0)) < 1e-10 * scale
    assert np.max(np.abs(out[1] - ref1)) < 1e-10 * scale


@pytest.mark.parametrize("mode,sign", [(3, +1), (3, -1), (-11, +1), (-11, -1), (0, +1)])
def test_constant_coupling_spectrum(mode, sign):
    # With F12 = f and V = v on both surfaces, -iF = f sigma_y; the spinor (1, sign*i)/sqrt2
    # times a plane wave of momentum p is an eigenvector with E = (p + sign f)^2/(2M) + v.
    n, qmin, qmax, M, f, v = 64, 0.0, 9.0, 1.3, 0.7, 0.05
    L = qmax - qmin
    q = I.uniform_grid(n, qmin, qmax)
    p = 2 * math.pi * mode / L
    psi = np.stack([np.exp(1j * p * q), sign * 1j * np.exp(1j * p * q)]) / math.sqrt(2)
    m = model_1d(n, qmin, qmax, M, v * np.ones((2, n)), f * np.ones(n))
    E = (p + sign * f) ** 2 / (2 * M) + v
    np.testing.assert_allclose(O.apply_H(m, psi), E * psi, atol=1e-12)


def test_two_dimensional_hamiltonian_matches_kronecker_assembly():
    n1, n2, L1, L2, M1, M2 = 8, 4, 4.0, 3.0, 1.1, 2.3
    rng = np.random.default_rng(7)
    V = rng.standard_normal((2, n1, n2))
    F = rng.standard_normal((2, n1, n2))
    m = O.Model((n1, n2), (0.0, 0.0), (L1, L2), (M1, M2), V, F)
    H = O.dense_H(m)
    def Pmat(n, L):
        W = dft_matrix(n)
        kp = [k if k < n // 2 else k - n for k in range(n)]
        return (W.conj().T @ np.diag([2 * math.pi * k / L for k in kp]) @ W) / n
    P1 = np.kron(Pmat(n1, L1), np.eye(n2))
    P2 = np.kron(np.eye(n1), Pmat(n2, L2))
    pts = n1 * n2
    Hd = np.diag(V.ravel()).astype(complex)
    for P, Fd, Md in [(P1, F[0].ravel(), M1), (P2, F[1].ravel(), M2)]:
        Z = np.zeros((pts, pts))
        Fm = np.block([[Z, np.diag(Fd)], [-np.diag(Fd), Z]])
        A = np.kron(np.eye(2), P) - 1j * Fm
        Hd = Hd + A.conj().T @ A / (2 * Md)
    assert np.max(np.abs(H - Hd)) < 1e-12 * np.max(np.abs(Hd))


def test_invariant_definitions_on_known_states():
    n, qmin, qmax = 256, 3.0, 16.0
    it = I.nai_like_item(n)
    m = O.model_from_item(it)
    assert abs(O.norm(m, it.psi0) - 1.0) < 1e-14
    P = O.populations(m, it.psi0)
    assert abs(P[0] - 1.0) < 1e-14 and P[1] == 0.0
    # omega(psi, i psi) = -2 Im <psi | i psi> = -2 ||psi||^2
    assert abs(O.symplectic_form(m, it.psi0, 1j * it.psi0) + 2.0) < 1e-14
    # energy of a plane-wave eigenstate equals its eigenvalue
    q = it.q
    L = qmax - qmin
    p = 2 * math.pi * 4 / L
    mc = O.Model((n,), (qmin,), (qmax,), (3.0,), 0.02 * np.ones((2, n)), np.zeros((1, n)))
    pw = np.stack([np.exp(1j * p * q), np.zeros(n)]) / math.sqrt(L)
    assert abs(O.energy(mc, pw) - (p * p / 6.0 + 0.02)) < 1e-14
