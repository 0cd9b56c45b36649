"""The grid-convergence study of App. B on the GPU: five grids of 256-4096 points, ranges
and densities growing by sqrt(2) per doubling, propagated in one ragged launch with the
8th-order Suzuki trapezoidal rule; the error against the densest grid falls
exponentially at t = 0 and at t_f."""
import pytest

pytestmark = pytest.mark.gpu


def test_grid_convergence_is_exponential_after_propagation():
    from paper_1902_04661_amd import gqd, gridconv as G
    gqd.load_library()
    res = G.grid_study(tf=100.0, dt=2.0)
    print(res, flush=True)
    e0, ef = res["error_t0"], res["error_tf"]
    assert ef[0] > 1e-5 and ef[-1] < 1e-11
    assert all(ef[k + 1] < 1e-2 * ef[k] for k in range(len(ef) - 2))
    # the packet spreads, so the ranges cut deeper into its tails at t_f than at t = 0
    assert ef[0] >= e0[0]


def test_study_items_match_oracle():
    # every grid of the study (256-4096 points on 0.5-2.0 bohr, far from the [3, 16)
    # grids of the other parity cases) against the oracle over two steps of the study's
    # own scheme (8th-order Suzuki trapezoidal rule, dt = 2 a.u.)
    import numpy as np

    import oracle as O
    from paper_1902_04661_amd import gqd, gridconv as G
    gqd.load_library()
    items = G.study_items()
    opts = dict(tol=1e-14, restart=48)
    with gqd.from_items(items) as prop:
        psi = prop.pack([it.psi0 for it in items])
        st = prop.propagate(psi, "trap", "suzuki", 8, 2.0, 2, gqd.SolverOpts(**opts))
        outs = prop.unpack(psi)
    for it, out in zip(items, outs):
        ost = O.Stats()
        ref = O.propagate(O.model_from_item(it), it.psi0, O.TRAP, O.SUZUKI, 8, 2.0, 2, O.SolverOpts(**opts), ost)
        r = float(np.linalg.norm(out - ref) / np.linalg.norm(ref))
        print(f"study grid n={it.n} L={it.qmax - it.qmin:.3f}: rel {r:.2e}, oracle mean iterations "
              f"{ost.iterations / ost.solves:.2f}", flush=True)
        assert r <= 1e-12
    assert st.failures == 0
