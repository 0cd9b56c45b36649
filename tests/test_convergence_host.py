"""Host-side helpers of the convergence and efficiency studies."""
import math

import pytest

from paper_1902_04661_amd import convergence as C


def test_cost_at_interpolates_on_log_log_axes():
    # errors 1e-3, 1e-6 at costs 1, 8: the geometric midpoint error costs sqrt(8)
    c, x = C.cost_at([1e-3, 1e-6], [1.0, 8.0], math.sqrt(1e-3 * 1e-6), 2)
    assert not x and c == pytest.approx(math.sqrt(8.0), rel=1e-12)


def test_cost_at_extrapolates_along_the_order():
    # second order: 100x smaller error needs a 10x smaller step, 10x the cost
    c, x = C.cost_at([1e-4, 1e-6], [1.0, 10.0], 1e-8, 2)
    assert x and c == pytest.approx(100.0, rel=1e-12)


def test_cost_at_unresolved_above_the_coarsest_run():
    assert C.cost_at([1e-9, 1e-12], [1.0, 2.0], 1e-5, 8) == (None, False)
