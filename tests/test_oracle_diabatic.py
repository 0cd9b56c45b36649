"""Pins of the oracle's diabatic -> adiabatic transformation (Sec. II.F, Eqs. 24-28) and
of its split-operator method in the diabatic representation (Table I): O^T W O is
diagonal with the printed energies, F12 agrees with Eq. (28) as printed, with the
textbook Hellmann-Feynman form and with a finite difference of the mixing angle; the
split-operator step is exact when W commutes with T, has the composed orders, is
unitary and time-reversible; and the adiabatic propagation agrees with the transformed
diabatic one at the composition's order."""
import numpy as np
import scipy.linalg

import oracle as O
from paper_1902_04661_amd import inputs as I


def test_rotation_diagonalises_W_with_the_printed_energies():
    it = I.diabatic_crossing_item(512)
    V, F12, c, s = O.diabatic_to_adiabatic(it.W, it.dW)
    W11, W22, W12 = it.W
    # O^T W O with O = [[c, -s], [s, c]] (Eq. 24)
    d1 = c * c * W11 + 2 * c * s * W12 + s * s * W22
    d2 = s * s * W11 - 2 * c * s * W12 + c * c * W22
    off = c * s * (W22 - W11) + (c * c - s * s) * W12
    scale = np.abs(it.W).max()
    assert np.abs(d1 - V[0]).max() < 1e-15 * scale and np.abs(d2 - V[1]).max() < 1e-15 * scale
    assert np.abs(off).max() < 1e-15 * scale
    # Eq. (26)'s orientation: the first column is along (W12, Delta), Delta = V_1 - W11,
    # where Delta is well conditioned (within 1.5 bohr of the crossing)
    near = np.abs(it.q - 6.0) < 1.5
    delta = V[0] - W11
    nrm = np.sqrt(W12 ** 2 + delta ** 2)
    assert np.abs(c - W12 / nrm)[near].max() < 1e-12 and np.abs(s - delta / nrm)[near].max() < 1e-12


def test_coupling_matches_eq_28_hellmann_feynman_and_the_mixing_angle():
    it = I.diabatic_crossing_item(2048)
    V, F12, c, s = O.diabatic_to_adiabatic(it.W, it.dW)
    W11, W22, W12 = it.W
    dW11, dW22, dW12 = it.dW
    near = np.abs(it.q - 6.0) < 1.5
    # Eq. (28) as printed, with Delta' differentiated from Delta = dW/2 + r
    dw, ddw = W22 - W11, dW22 - dW11
    r = np.sqrt((dw / 2) ** 2 + W12 ** 2)
    delta = dw / 2 + r
    ddelta = ddw / 2 + ((dw / 2) * (ddw / 2) + W12 * dW12) / r
    eq28 = (dW12 * delta - W12 * ddelta) / (W12 ** 2 + delta ** 2)
    assert np.abs(F12 - eq28)[near].max() < 1e-10 * np.abs(F12).max()
    # <phi_1|phi_2'> = <phi_1|W'|phi_2> / (V_2 - V_1) with phi_1 = (c, s), phi_2 = (-s, c)
    hf = (c * (-s) * dW11 + (c * c - s * s) * dW12 + s * c * dW22) / (V[1] - V[0])
    assert np.abs(F12 - hf).max() < 1e-10 * np.abs(F12).max()
    # F12 = -theta': centred differences of theta = atan2(s, c) on the grid, whose own
    # error across the 0.09-bohr peak is ~ (dq / 0.09)^2 / 6 ~ 1e-3 of it
    theta = np.arctan2(s, c)
    fd = -(theta[2:] - theta[:-2]) / (2 * it.dq)
    assert np.abs(F12[1:-1] - fd).max() < 5e-3 * np.abs(F12).max()
    assert F12.max() > 5.0  # a sharp coupling at the crossing


def small_diabatic(n=32, constant=False):
    q = I.uniform_grid(n, 0.0, 6.0)
    if constant:
        W = np.stack([0.2 * np.ones(n), 0.5 * np.ones(n), 0.15 * np.ones(n)])
    else:
        W = np.stack([0.3 * np.cos(2 * np.pi * q / 6), 0.1 + 0.2 * np.sin(2 * np.pi * q / 6),
                      0.2 * np.exp(-((q - 3) ** 2))])
    psi = np.stack([np.exp(-((q - 2.5) ** 2) + 1j * 1.5 * q), 0.3 * np.exp(-((q - 3.5) ** 2))])
    return q, W, psi / np.sqrt((6.0 / n) * np.sum(np.abs(psi) ** 2))


def dense_H_diabatic(n, W, mass):
    cols = []
    for k in range(2 * n):
        e = np.zeros(2 * n, complex)
        e[k] = 1.0
        cols.append(O.apply_H_diabatic(n, 0.0, 6.0, mass, W, e.reshape(2, n)).ravel())
    return np.array(cols).T


def test_split_operator_is_exact_when_W_commutes_with_T():
    n, mass = 32, 1.5
    q, W, psi = small_diabatic(n, constant=True)
    H = dense_H_diabatic(n, W, mass)
    out = O.split_operator_propagate(n, 0.0, 6.0, mass, W, psi, "suzuki", 2, 0.7, 5)
    ex = (scipy.linalg.expm(-1j * 3.5 * H) @ psi.ravel()).reshape(2, n)
    assert np.linalg.norm(out - ex) < 1e-13 * np.linalg.norm(ex)


def test_split_operator_orders_unitarity_and_reversibility():
    n, mass = 32, 1.5
    q, W, psi = small_diabatic(n)
    H = dense_H_diabatic(n, W, mass)
    assert np.abs(H - H.conj().T).max() < 1e-14
    T = 2.0
    ex = (scipy.linalg.expm(-1j * T * H) @ psi.ravel()).reshape(2, n)
    for order, lo, hi in ((2, 3.5, 4.5), (4, 13.0, 19.0)):
        errs = []
        for k in (0, 1):
            dt = 0.2 / 2 ** k
            out = O.split_operator_propagate(n, 0.0, 6.0, mass, W, psi, "suzuki", order, dt, int(round(T / dt)))
            errs.append(np.linalg.norm(out - ex))
            assert abs(np.linalg.norm(out) - np.linalg.norm(psi)) < 1e-13 * np.linalg.norm(psi)
        assert lo < errs[0] / errs[1] < hi
    fwd = O.split_operator_propagate(n, 0.0, 6.0, mass, W, psi, "triple_jump", 4, 0.3, 7)
    back = O.split_operator_propagate(n, 0.0, 6.0, mass, W, fwd, "triple_jump", 4, -0.3, 7)
    assert np.linalg.norm(back - psi) < 1e-13 * np.linalg.norm(psi)


def test_adiabatic_and_diabatic_propagations_agree_at_the_composition_order():
    it = I.diabatic_crossing_item(1024)
    V, F12, c, s = O.diabatic_to_adiabatic(it.W, it.dW)
    m = O.Model((it.n,), (it.qmin,), (it.qmax,), (it.mass,), V, F12[None, :])
    psi_ad0 = O.to_adiabatic(it.psi0, c, s)
    diffs = []
    for dt, nsteps in ((20.0, 40), (10.0, 80)):
        ad = O.propagate(m, psi_ad0, O.MIDP, O.SUZUKI, 6, dt, nsteps, O.SolverOpts(tol=1e-14, restart=48))
        so = O.to_adiabatic(O.split_operator_propagate(it.n, it.qmin, it.qmax, it.mass, it.W, it.psi0,
                                                       "suzuki", 6, dt, nsteps), c, s)
        diffs.append(np.linalg.norm(ad - so) / np.linalg.norm(so))
    upper = it.dq * np.sum(np.abs(ad[0]) ** 2)
    assert upper > 0.03  # population crossed to the upper adiabatic surface
    assert diffs[1] < 1e-6 and 40.0 < diffs[0] / diffs[1] < 90.0  # sixth order: 64


def test_library_transform_matches_the_oracle():
    # paper_1902_04661_amd.diabatic is written apart from the oracle; pin it to it
    from paper_1902_04661_amd import diabatic as D
    it = I.diabatic_crossing_item(1024)
    V, F12, c, s = O.diabatic_to_adiabatic(it.W, it.dW)
    V2, F2, theta = D.adiabatic_surfaces(it.W, it.dW)
    scale = np.abs(V).max()
    assert np.abs(V - V2).max() < 1e-15 * scale
    assert np.abs(F12 - F2).max() < 1e-13 * np.abs(F12).max()
    assert np.abs(np.cos(theta) - c).max() < 1e-15 and np.abs(np.sin(theta) - s).max() < 1e-15
    ad, th = D.adiabatic_item(it)
    assert np.abs(ad.psi0 - O.to_adiabatic(it.psi0, c, s)).max() < 1e-15
    assert np.abs(D.rotate(ad.psi0, th, inverse=True) - it.psi0).max() < 1e-15
