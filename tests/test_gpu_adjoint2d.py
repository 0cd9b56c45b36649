"""GPU gradients on a 2D grid through torch.autograd: d P_2(T) / d (A, c1, c2, w) of the
vector coupling F12^(d) = A exp(-((q1-c1)^2 + (q2-c2)^2)/w^2) (0.8, 0.6)_d, against
central finite differences of GPU forward runs."""
import pytest
import torch

from paper_1902_04661_amd import inputs as I

pytestmark = pytest.mark.gpu

N = 128
SCHEME, ORDER, DT, NSTEPS = "suzuki", 4, 10.0, 100   # T = 1000 a.u.
NAMES = ["amp", "c1", "c2", "w"]


@pytest.fixture(scope="module")
def mods():
    from paper_1902_04661_amd import autograd, gqd
    gqd.load_library()
    return gqd, autograd


def loss(gqd, ag, prop, it, P, Q, opts, grad=True):
    F = ag.coupling_2d(Q[0], Q[1], P["amp"], P["c1"], P["c2"], P["w"]).reshape(-1)
    psi0 = prop.pack([it.psi0])
    if grad:
        psiT = ag.propagate(prop, psi0, F, SCHEME, ORDER, DT, NSTEPS, opts)
    else:
        psiT = psi0
        prop.set_surfaces(prop.V, F.detach().contiguous())
        prop.propagate(psiT, "midp", SCHEME, ORDER, DT, NSTEPS, opts)
    dv = ((it.qmax[0] - it.qmin[0]) / N) * ((it.qmax[1] - it.qmin[1]) / N)
    return ag.surface_population(psiT.reshape(2, N, N), dv)


def test_coupling_gradients_match_central_differences_2d(mods):
    gqd, ag = mods
    dev = torch.device("cuda", 0)
    # a packet displaced toward the coupling region, moving along q1
    it = I.two_dim_item(N, N, q0=(6.2, 5.0), p0=(4.0, 1.0))
    prop = gqd.from_items([it], device=dev)
    Q = ag.grid2d(N, it.qmin, it.qmax, dev)
    base = dict(zip(NAMES, it.params["cparams"]))
    P = {k: torch.tensor(v, dtype=torch.float64, device=dev, requires_grad=True) for k, v in base.items()}
    opts = gqd.SolverOpts(tol=1e-15, restart=32)
    L = loss(gqd, ag, prop, it, P, Q, opts)
    L.backward()
    Lv = float(L)
    print(f"L = P_2(T) = {Lv:.6e}", flush=True)
    assert Lv > 1e-8
    h = 1e-5
    for name in NAMES:
        Pp = {k: torch.tensor(v + (h if k == name else 0.0), dtype=torch.float64, device=dev)
              for k, v in base.items()}
        Pm = {k: torch.tensor(v - (h if k == name else 0.0), dtype=torch.float64, device=dev)
              for k, v in base.items()}
        fd = (float(loss(gqd, ag, prop, it, Pp, Q, opts, grad=False))
              - float(loss(gqd, ag, prop, it, Pm, Q, opts, grad=False))) / (2 * h)
        g = float(P[name].grad)
        print(f"d L / d {name}: adjoint {g:.10e}  central difference {fd:.10e}", flush=True)
        assert abs(g - fd) <= 1e-6 * abs(fd) + 1e-9 * Lv
