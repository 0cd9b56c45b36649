"""The differentiable torch input builders reproduce the numpy input module."""
import numpy as np
import torch

from paper_1902_04661_amd import autograd as ag
from paper_1902_04661_amd import inputs as I


def test_torch_builders_match_numpy_inputs():
    it = I.nai_like_item(1024, q0=5.3, p0=-2.0, amp=0.55, center=7.2)
    q = ag.grid(it.n, it.qmin, it.qmax, "cpu")
    np.testing.assert_allclose(q.numpy(), it.q, rtol=0, atol=1e-14)
    psi = ag.gaussian_packet(q, torch.tensor(5.3, dtype=torch.float64), torch.tensor(-2.0, dtype=torch.float64),
                             torch.tensor(0.12, dtype=torch.float64))
    np.testing.assert_allclose(psi.numpy(), it.psi0, rtol=0, atol=1e-13)
    F = ag.coupling(q, torch.tensor(0.55, dtype=torch.float64), torch.tensor(7.2, dtype=torch.float64))
    np.testing.assert_allclose(F.numpy(), it.F[0], rtol=0, atol=1e-15)
    assert abs(float(ag.surface_population(psi, it.dq, 0)) - 1.0) < 1e-14



def test_batched_builders_match_the_per_packet_ones():
    items = I.adjoint_batch(5, seed=1, n=512)
    q = ag.grid(512, items[0].qmin, items[0].qmax, "cpu")
    P = {k: torch.tensor([it.params[k] for it in items], dtype=torch.float64)
         for k in ["q0", "p0", "width", "amp", "center"]}
    psi = ag.gaussian_packets(q, P["q0"], P["p0"], P["width"])
    F = ag.couplings(q, P["amp"], P["center"])
    for b, it in enumerate(items):
        one = ag.gaussian_packet(q, P["q0"][b], P["p0"][b], P["width"][b])
        assert torch.equal(psi[b], one)
        assert torch.equal(F[b], ag.coupling(q, P["amp"][b], P["center"][b]))
        np.testing.assert_allclose(psi[b].numpy(), it.psi0, rtol=0, atol=1e-12)


def test_ragged_batch_draws_are_seeded_and_in_range():
    a = I.ragged_batch_draws(64, seed=0)
    b = I.ragged_batch_draws(64, seed=0)
    for k in a:
        assert np.array_equal(a[k], b[k])
    assert set(np.unique(a["n"])) <= {256, 512, 1024, 2048, 4096}
    assert a["q0"].min() >= 4.5 and a["q0"].max() <= 6.0
    assert a["p0"].min() >= -5 and a["p0"].max() <= 5
    assert a["amp"].min() >= 0.1 and a["amp"].max() <= 0.8
