"""Pins for the oracle's right-preconditioned GMRES (the option precond): the
preconditioner is the exact inverse of 1 + i a T (T the kinetic operator), and the
preconditioned solve reaches the same solution as a dense solve and as the plain GMRES
of Sec. II.C."""
import numpy as np
import pytest

import oracle as O
from paper_1902_04661_amd import inputs as I


def two_dim_model(n=16):
    it = I.two_dim_item(n, n)
    return O.model_from_item(it), it.psi0


@pytest.mark.parametrize("dims", [1, 2])
def test_kinetic_inverse_undoes_one_plus_i_a_T(dims):
    # T x = sum_d P_d P_d x / 2 m_d through the oracle's (pinned) momentum operator
    if dims == 1:
        it = I.nai_like_item(128, p0=3.0)
        m, x = O.model_from_item(it), it.psi0
    else:
        m, x = two_dim_model()
    rng = np.random.default_rng(5)
    x = x + 0.1 * (rng.standard_normal(x.shape) + 1j * rng.standard_normal(x.shape))
    for a in (0.7, -2.5):
        Tx = sum(O.apply_P(m, O.apply_P(m, x, d), d) / (2.0 * m.mass[d]) for d in range(m.D))
        y = O.kinetic_inverse(m, a)(x + 1j * a * Tx)
        assert np.linalg.norm(y - x) <= 1e-14 * np.linalg.norm(x)


@pytest.mark.parametrize("restart", [64, 3])
def test_preconditioned_gmres_matches_dense_solve(restart):
    it = I.nai_like_item(64, p0=4.0, amp=0.8)
    m = O.model_from_item(it)
    H = O.dense_H(m)
    for a in (3.0, -7.0):
        X = np.eye(H.shape[0]) + 1j * a * H
        b = it.psi0.ravel()
        ref = np.linalg.solve(X, b)
        st = O.Stats()
        x = O.implicit_euler(m, it.psi0, a, O.SolverOpts(tol=1e-15, restart=restart, precond=True), st)
        assert st.failures == 0
        assert np.linalg.norm(x.ravel() - ref) <= 1e-13 * np.linalg.norm(ref)
        # the stop test is on the residual of X x = b itself
        assert np.linalg.norm(b - X @ x.ravel()) <= 2e-15 * np.linalg.norm(b)


def test_preconditioned_propagation_matches_plain_gmres():
    it = I.nai_like_item(256, q0=4.7, p0=-3.0, amp=0.6)
    m = O.model_from_item(it)
    for method in (O.MIDP, O.TRAP):
        outs = [O.propagate(m, it.psi0, method, O.SUZUKI, 4, 10.0, 3, O.SolverOpts(tol=1e-15, precond=pc))
                for pc in (False, True)]
        assert np.linalg.norm(outs[1] - outs[0]) <= 1e-13


def test_preconditioning_removes_the_kinetic_stiffness():
    # on finer grids the kinetic spectrum widens and plain GMRES needs more iterations;
    # with the kinetic part inverted the count stays put
    counts = {}
    for n in (512, 2048):
        it = I.nai_like_item(n, q0=4.6, p0=-4.5, amp=0.6)
        m = O.model_from_item(it)
        for pc in (False, True):
            st = O.Stats()
            O.propagate(m, it.psi0, O.MIDP, O.SUZUKI, 4, 20.0, 1, O.SolverOpts(tol=1e-15, precond=pc), st)
            counts[n, pc] = st.iterations / st.solves
    assert counts[2048, False] > 1.5 * counts[512, False]
    assert counts[2048, True] < 0.6 * counts[2048, False]
    assert abs(counts[2048, True] - counts[512, True]) < 1.5
