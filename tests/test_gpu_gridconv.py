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
