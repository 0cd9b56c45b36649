"""GPU gradients of the surface-2 population through torch.autograd (reverse sweep in the
HIP library): against central finite differences of GPU forward runs and against the
oracle's reverse sweep on the same inputs."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1902_04661_amd import inputs as I

pytestmark = pytest.mark.gpu

N, B = 1024, 4
SCHEME, ORDER, DT, NSTEPS = "suzuki", 4, 4.0, 1000   # T = 4000 a.u.
NAMES = ["q0", "p0", "w", "amp", "center"]


@pytest.fixture(scope="module")
def mods():
    from paper_1902_04661_amd import autograd, gqd
    gqd.load_library()
    return gqd, autograd


def make_params(dev):
    items = I.adjoint_batch(B, seed=1, n=N)
    P = {"q0": [it.params["q0"] for it in items], "p0": [it.params["p0"] for it in items],
         "w": [it.params["width"] for it in items], "amp": [it.params["amp"] for it in items],
         "center": [it.params["center"] for it in items]}
    return items, {k: torch.tensor(v, dtype=torch.float64, device=dev) for k, v in P.items()}


def loss_and_inputs(ag, prop, items, P):
    q = ag.grid(N, items[0].qmin, items[0].qmax, prop.device)
    psi0 = torch.cat([ag.gaussian_packet(q, P["q0"][b], P["p0"][b], P["w"][b]).reshape(-1) for b in range(B)])
    F = torch.cat([ag.coupling(q, P["amp"][b], P["center"][b]) for b in range(B)])
    return psi0, F


def total_loss(gqd, ag, prop, items, P, opts, grad=True):
    psi0, F = loss_and_inputs(ag, prop, items, P)
    psiT = ag.propagate(prop, psi0, F, SCHEME, ORDER, DT, NSTEPS, opts) if grad else None
    if not grad:
        psiT = psi0.detach().clone()
        prop.set_surfaces(prop.V, F.detach().contiguous())
        prop.propagate(psiT, "midp", SCHEME, ORDER, DT, NSTEPS, opts)
    dq = items[0].dq
    return sum(ag.surface_population(psiT[2 * N * b:2 * N * (b + 1)].reshape(2, N), dq) for b in range(B))


def test_gradients_match_central_differences(mods):
    gqd, ag = mods
    dev = torch.device("cuda", 0)
    items, P = make_params(dev)
    prop = gqd.from_items(items, device=dev)
    opts = gqd.SolverOpts(tol=1e-15, restart=32)
    Pg = {k: v.clone().requires_grad_(True) for k, v in P.items()}
    L = total_loss(gqd, ag, prop, items, Pg, opts)
    L.backward()
    Lv = float(L)
    print(f"L = {Lv:.6e}", flush=True)
    h = 1e-5
    for name in NAMES:
        for b in [0, 2]:
            Pp = {k: v.clone() for k, v in P.items()}
            Pm = {k: v.clone() for k, v in P.items()}
            Pp[name][b] += h
            Pm[name][b] -= h
            fd = (float(total_loss(gqd, ag, prop, items, Pp, opts, grad=False))
                  - float(total_loss(gqd, ag, prop, items, Pm, opts, grad=False))) / (2 * h)
            g = float(Pg[name].grad[b])
            print(f"d L / d {name}[{b}]: adjoint {g:.10e}  central difference {fd:.10e}", flush=True)
            # finite differences resolve about 1e-9 of L at h = 1e-5 and tol 1e-15
            assert abs(g - fd) <= 1e-6 * abs(fd) + 1e-9 * Lv


def test_reverse_sweep_matches_oracle(mods):
    # both reverse sweeps start from the same psi(T) and lambda(T) = dq Pi_2 psi(T),
    # those of the oracle's forward run; the GPU's own forward run is compared with the
    # oracle's separately (its surface-2 part is small, so an independent lambda(T)
    # would carry the forward runs' difference into every relative figure)
    gqd, ag = mods
    dev = torch.device("cuda", 0)
    items = I.adjoint_batch(2, seed=1, n=N)
    prop = gqd.from_items(items, device=dev)
    opts = dict(tol=1e-15, restart=32)
    fwd = []
    for it in items:
        m = O.model_from_item(it)
        oT = O.propagate(m, it.psi0, O.MIDP, SCHEME, ORDER, DT, 10, O.SolverOpts(**opts))
        fwd.append((oT, O.population_loss(m, oT)[1]))
    psi = prop.pack([it.psi0 for it in items])
    prop.propagate(psi, "midp", SCHEME, ORDER, DT, 10, gqd.SolverOpts(**opts))
    for b, (g_T, (oT, _)) in enumerate(zip(prop.unpack(psi), fwd)):
        print(f"item {b}: forward psi(T) rel {np.linalg.norm(g_T - oT) / np.linalg.norm(oT):.2e}", flush=True)
    psi = prop.pack([f[0] for f in fwd])
    lam_t = prop.pack([f[1] for f in fwd])
    gF = torch.zeros(prop.state_size // 2, dtype=torch.float64, device=dev)
    prop.adjoint(psi, lam_t, gF, SCHEME, ORDER, DT, 10, gqd.SolverOpts(**opts))
    l0 = prop.unpack(lam_t)
    p0 = prop.unpack(psi)
    g = gF.cpu().numpy()
    for b, (it, (oT, lT)) in enumerate(zip(items, fwd)):
        po, lo, go = O.adjoint(O.model_from_item(it), oT, lT, SCHEME, ORDER, DT, 10, O.SolverOpts(**opts))
        rl = np.linalg.norm(l0[b] - lo) / np.linalg.norm(lo)
        rg = np.linalg.norm(g[b * N:(b + 1) * N] - go[0]) / np.linalg.norm(go[0])
        rp = np.linalg.norm(p0[b] - it.psi0) / np.linalg.norm(it.psi0)
        print(f"item {b}: lambda(0) rel {rl:.2e}, dL/dF12 rel {rg:.2e}, psi(0) reconstruction {rp:.2e}", flush=True)
        assert rl <= 1e-10 and rg <= 1e-10 and rp <= 2e-12
