"""CPU pins of the grid-convergence tools (App. B): the trigonometric interpolant takes
the grid values and reproduces band-limited functions between them, and the initial
packet converges exponentially on grids whose range and density grow by sqrt(2) per
doubling; plus the phase measure of Sec. III."""
import math

import numpy as np

from paper_1902_04661_amd import convergence as C
from paper_1902_04661_amd import gridconv as G
from paper_1902_04661_amd import inputs as I


def test_trig_interpolant_is_exact_for_band_limited_functions():
    n, a, b = 64, 1.0, 4.0
    q = I.uniform_grid(n, a, b)
    L = b - a

    def f(x):  # modes 5, -17 and the Nyquist cosine
        return (0.3 * np.exp(2j * np.pi * 5 * (x - a) / L) - 1.1 * np.exp(-2j * np.pi * 17 * (x - a) / L)
                + 0.7 * np.cos(2 * np.pi * 32 * (x - a) / L))

    psi = np.stack([f(q), 2 * f(q)])
    assert np.abs(G.trig_interpolate(psi, a, b, q) - psi).max() < 1e-13
    x = a + L * np.random.default_rng(0).random(50)
    assert np.abs(G.trig_interpolate(psi, a, b, x) - np.stack([f(x), 2 * f(x)])).max() < 1e-12


def test_initial_packet_converges_exponentially_with_the_grid():
    items = G.study_items()
    lengths = [it.qmax - it.qmin for it in items]
    for k in range(1, len(items)):  # both grids scale by sqrt(2) per doubling of n
        assert items[k].n == 2 * items[k - 1].n
        assert abs(lengths[k] / lengths[k - 1] - math.sqrt(2)) < 1e-12
        assert abs(items[k - 1].dq / items[k].dq - math.sqrt(2)) < 1e-12
    errs = G.compare_to_densest(items, [it.psi0 for it in items])
    assert errs[0] > 1e-4 and errs[-1] < 1e-12
    assert all(errs[k + 1] < 1e-2 * errs[k] for k in range(len(errs) - 2))


def test_phase_at_peak_and_its_error():
    q = I.uniform_grid(256, 3.0, 16.0)
    psi = I.gaussian_packet_1d(q, 6.0, 0.0, 0.2) * np.exp(1j * 2.5)
    psi[1] = 0.5 * psi[0] * np.exp(1j * 1.0)  # smaller amplitude on the second surface
    assert abs(C.phase_at_peak(psi) - 2.5) < 1e-14
    other = psi * np.exp(-1j * 6.2)  # phases 2.5 and -3.7 differ by 6.2, i.e. by 2 pi - 6.2
    assert abs(C.phase_error(other, psi) - (2 * math.pi - 6.2)) < 1e-12
