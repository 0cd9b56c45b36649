"""GPU parity on 2D grids: the cooperative n x n kernel through the C ABI against the
CPU oracle on the same seeded inputs (relative L2 per wavefunction)."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1902_04661_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gqd():
    from paper_1902_04661_amd import gqd as g
    g.load_library()
    return g


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def moving_item(n, seed=2, p0=(2.0, -1.5), q0=(5.8, 5.0), cparams=(0.4, 7.0, 5.0, 0.5)):
    return I.two_dim_item(n, n, seed=seed, q0=q0, p0=p0, cparams=cparams)


@pytest.mark.parametrize("n", [64, 128, 256, 512])
def test_apply_H_matches_oracle_2d(gqd, n):
    it = moving_item(n)
    prop = gqd.from_items([it])
    x = I.random_state((2, n, n), seed=n)
    print(f"apply_H 2D n={n}: start", flush=True)
    out = prop.unpack(prop.apply_H(prop.pack([x])))[0]
    ref = O.apply_H(O.model_from_item(it), x)
    print(f"apply_H 2D n={n}: rel {rel(out, ref):.2e}", flush=True)
    assert rel(out, ref) <= 1e-13


def test_apply_H_batch_with_distinct_grids_2d(gqd):
    # three items of one size on different boxes (different momentum grids and dq)
    items = [moving_item(64, seed=s) for s in (2, 3, 4)]
    items[1].qmin, items[1].qmax = (2.0, 1.0), (15.0, 9.0)
    items[2].qmin, items[2].qmax = (3.5, 0.5), (18.0, 7.5)
    prop = gqd.from_items(items)
    xs = [I.random_state((2, 64, 64), seed=30 + b) for b in range(3)]
    outs = prop.unpack(prop.apply_H(prop.pack(xs)))
    for b, (it, x, out) in enumerate(zip(items, xs, outs)):
        r = rel(out, O.apply_H(O.model_from_item(it), x))
        print(f"item {b}: rel {r:.2e}", flush=True)
        assert r <= 1e-13


def test_diag_and_inner_match_oracle_2d(gqd):
    it = moving_item(128)
    prop = gqd.from_items([it])
    psi = prop.pack([it.psi0])
    phi_l = I.random_state((2, 128, 128), seed=5) * 0.01
    d = prop.diag(psi).cpu().numpy()[0]
    ip = prop.inner(psi, prop.pack([phi_l])).cpu().numpy()[0]
    m = O.model_from_item(it)
    E = O.energy(m, it.psi0)
    print(f"diag {d}, oracle norm {O.norm(m, it.psi0)} energy {E}", flush=True)
    assert abs(d[0] - O.norm(m, it.psi0)) < 1e-14
    assert abs(d[1] - E) < 1e-13 * abs(E)
    assert np.allclose(d[2:], O.populations(m, it.psi0), rtol=0, atol=1e-14)
    assert abs(ip - O.inner(m, it.psi0, phi_l)) < 1e-13 * np.linalg.norm(phi_l)


@pytest.mark.parametrize("method", ["midp", "trap"])
@pytest.mark.parametrize("literal", [False, True])
def test_single_step_matches_oracle_2d(gqd, method, literal):
    it = moving_item(64)
    prop = gqd.from_items([it])
    psi = prop.pack([it.psi0])
    opts = dict(tol=1e-14, restart=32, literal=literal)
    print(f"2D {method} literal={literal}: start", flush=True)
    st = prop.implicit_step(psi, method, 10.0, gqd.SolverOpts(**opts))
    ost = O.Stats()
    ref = O.propagate(O.model_from_item(it), it.psi0, method, O.SUZUKI, 2, 10.0, 1, O.SolverOpts(**opts), ost)
    r = rel(prop.unpack(psi)[0], ref)
    print(f"2D {method} literal={literal}: rel {r:.2e}, iterations gpu {st.iterations} "
          f"oracle {ost.iterations}", flush=True)
    assert r <= 1e-13
    assert st.failures == 0


@pytest.mark.parametrize("scheme,order,n", [("suzuki", 4, 64), ("triple_jump", 6, 128), ("suzuki", 8, 64)])
def test_composed_propagation_matches_oracle_2d(gqd, scheme, order, n):
    it = moving_item(n)
    prop = gqd.from_items([it])
    psi = prop.pack([it.psi0])
    opts = dict(tol=1e-14, restart=32)
    dt, nsteps = 10.0, 2
    print(f"2D {scheme}-{order} n={n}: start", flush=True)
    st = prop.propagate(psi, "midp", scheme, order, dt, nsteps, gqd.SolverOpts(**opts))
    ost = O.Stats()
    ref = O.propagate(O.model_from_item(it), it.psi0, O.MIDP, scheme, order, dt, nsteps, O.SolverOpts(**opts), ost)
    r = rel(prop.unpack(psi)[0], ref)
    print(f"2D {scheme}-{order} n={n}: rel {r:.2e}, iterations gpu {st.iterations} oracle {ost.iterations}",
          flush=True)
    assert r <= 1e-12
    assert abs(st.iterations - ost.iterations) <= max(2, ost.iterations // 50)


def test_batch_of_2d_items_matches_oracle(gqd):
    items = [moving_item(64, seed=s, p0=(1.0 + s, -0.5 * s)) for s in (2, 3, 4)]
    prop = gqd.from_items(items)
    psi = prop.pack([it.psi0 for it in items])
    opts = dict(tol=1e-14, restart=32)
    prop.propagate(psi, "midp", "suzuki", 4, 10.0, 2, gqd.SolverOpts(**opts))
    for b, (it, out) in enumerate(zip(items, prop.unpack(psi))):
        ref = O.propagate(O.model_from_item(it), it.psi0, O.MIDP, O.SUZUKI, 4, 10.0, 2, O.SolverOpts(**opts))
        r = rel(out, ref)
        print(f"batch item {b}: rel {r:.2e}", flush=True)
        assert r <= 1e-12


def test_full_size_step_matches_oracle_2d(gqd):
    # the 256 x 256 model at its own step: one Suzuki order-4 step of 10 a.u.
    it = I.two_dim_item(256, 256)
    prop = gqd.from_items([it])
    psi = prop.pack([it.psi0])
    opts = dict(tol=1e-14, restart=32)
    st = prop.propagate(psi, "midp", "suzuki", 4, 10.0, 1, gqd.SolverOpts(**opts))
    ref = O.propagate(O.model_from_item(it), it.psi0, O.MIDP, O.SUZUKI, 4, 10.0, 1, O.SolverOpts(**opts))
    r = rel(prop.unpack(psi)[0], ref)
    print(f"2D 256x256 SZ-4: rel {r:.2e}, iterations {st.iterations} in {st.solves} solves", flush=True)
    assert r <= 1e-12


def oracle_forward(it, scheme, order, dt, nsteps, opts):
    """The oracle's forward run and its loss gradient dL/dpsi*(T) = dv Pi_2 psi(T): both
    reverse sweeps start from these."""
    m = O.model_from_item(it)
    oT = O.propagate(m, it.psi0, O.MIDP, scheme, order, dt, nsteps, O.SolverOpts(**opts))
    return m, oT, O.population_loss(m, oT)[1]


def test_adjoint_matches_oracle_2d(gqd):
    it = moving_item(64)
    prop = gqd.from_items([it])
    opts = dict(tol=1e-15, restart=32)
    m, oT, lT = oracle_forward(it, O.SUZUKI, 4, 10.0, 3, opts)
    psi = prop.pack([oT])
    lam = prop.pack([lT])
    gF = torch.zeros(prop.f_size, dtype=torch.float64, device=psi.device)
    st = prop.adjoint(psi, lam, gF, "suzuki", 4, 10.0, 3, gqd.SolverOpts(**opts))
    # phi and mu are solved by two groups of workgroups; the statistics count both
    assert st.solves == 2 * 5 * 3 and st.failures == 0 and st.nonfinite == 0
    po, lo, go = O.adjoint(m, oT, lT, O.SUZUKI, 4, 10.0, 3, O.SolverOpts(**opts))
    rl = rel(prop.unpack(lam)[0], lo)
    rg0 = rel(gF.cpu().numpy()[:64 * 64], go[0].ravel())
    rg1 = rel(gF.cpu().numpy()[64 * 64:], go[1].ravel())
    rp = rel(prop.unpack(psi)[0], it.psi0)
    print(f"2D adjoint: lambda rel {rl:.2e}, gF_1 rel {rg0:.2e}, gF_2 rel {rg1:.2e}, psi(0) rel {rp:.2e}",
          flush=True)
    assert rl <= 1e-10 and rg0 <= 1e-10 and rg1 <= 1e-10 and rp <= 2e-12


def test_adjoint_batch_of_2d_items_matches_oracle(gqd):
    # three items in one reverse sweep: every item has two groups (phi and mu), its own
    # pair of workspace regions and hand-off counters, and merged statistics
    items = [moving_item(64, seed=s, p0=(1.0 + s, -0.5 * s)) for s in (2, 3, 4)]
    prop = gqd.from_items(items)
    opts = dict(tol=1e-15, restart=32)
    fwd = [oracle_forward(it, O.SUZUKI, 2, 10.0, 3, opts) for it in items]
    psi = prop.pack([f[1] for f in fwd])
    lam = prop.pack([f[2] for f in fwd])
    gF = torch.zeros(prop.f_size, dtype=torch.float64, device=psi.device)
    st = prop.adjoint(psi, lam, gF, "suzuki", 2, 10.0, 3, gqd.SolverOpts(**opts))
    assert st.solves == 3 * 2 * 1 * 3 and st.failures == 0 and st.nonfinite == 0
    g = gF.cpu().numpy().reshape(3, 2, 64 * 64)
    for b, (it, (m, oT, lT), out_lam, out_psi) in enumerate(zip(items, fwd, prop.unpack(lam), prop.unpack(psi))):
        po, lo, go = O.adjoint(m, oT, lT, O.SUZUKI, 2, 10.0, 3, O.SolverOpts(**opts))
        rl, rp = rel(out_lam, lo), rel(out_psi, it.psi0)
        rg = max(rel(g[b, 0], go[0].ravel()), rel(g[b, 1], go[1].ravel()))
        print(f"2D adjoint batch item {b}: lambda rel {rl:.2e}, gF rel {rg:.2e}, psi(0) rel {rp:.2e}",
              flush=True)
        assert rl <= 1e-10 and rg <= 1e-10 and rp <= 2e-12


def test_adjoint_matches_oracle_full_size_2d(gqd):
    # the 256 x 256 model of the 2D gradient workload: one Suzuki order-4 step, then its
    # reverse sweep on two groups of 64 workgroups each (phi and mu) with the hand-offs
    # between them, from the oracle's psi(T) and loss gradient
    it = I.two_dim_item(256, 256)
    n = 256
    prop = gqd.from_items([it])
    opts = dict(tol=1e-14, restart=32)
    m, oT, lT = oracle_forward(it, O.SUZUKI, 4, 10.0, 1, opts)
    psi = prop.pack([it.psi0])
    prop.propagate(psi, "midp", "suzuki", 4, 10.0, 1, gqd.SolverOpts(**opts))
    print(f"2D 256x256 forward: psi(T) rel {rel(prop.unpack(psi)[0], oT):.2e}", flush=True)
    psi = prop.pack([oT])
    lam = prop.pack([lT])
    gF = torch.zeros(prop.f_size, dtype=torch.float64, device=psi.device)
    st = prop.adjoint(psi, lam, gF, "suzuki", 4, 10.0, 1, gqd.SolverOpts(**opts))
    assert st.solves == 2 * 5 and st.failures == 0 and st.nonfinite == 0
    po, lo, go = O.adjoint(m, oT, lT, O.SUZUKI, 4, 10.0, 1, O.SolverOpts(**opts))
    g = gF.cpu().numpy()
    rl = rel(prop.unpack(lam)[0], lo)
    rg0 = rel(g[:n * n], go[0].ravel())
    rg1 = rel(g[n * n:], go[1].ravel())
    rp = rel(prop.unpack(psi)[0], it.psi0)
    print(f"2D 256x256 adjoint: lambda rel {rl:.2e}, gF_1 rel {rg0:.2e}, gF_2 rel {rg1:.2e}, "
          f"psi(0) rel {rp:.2e} (oracle {rel(po, it.psi0):.2e}), {st.iterations} iterations in "
          f"{st.solves} solves", flush=True)
    assert rl <= 1e-10 and rg0 <= 1e-10 and rg1 <= 1e-10 and rp <= 2e-12


def test_wait_limit_gives_up_and_recovers_2d(gqd):
    # a one-poll limit on the bounded grid waits (forced from the host): the item stops,
    # every workgroup leaves, the call reports the timeout; the default limit then works
    it = moving_item(64)
    prop = gqd.from_items([it])
    opts = gqd.SolverOpts(tol=1e-14, restart=32)
    psi = prop.pack([it.psi0])
    prop.set_wait_limit(1)
    with pytest.raises(RuntimeError, match="timed out"):
        prop.propagate(psi, "midp", "suzuki", 4, 10.0, 4, opts)
    # the two-group reverse sweep gives up the same way
    lam = prop.pack([it.psi0])
    gF = torch.zeros(prop.f_size, dtype=torch.float64, device=psi.device)
    with pytest.raises(RuntimeError, match="timed out"):
        prop.adjoint(psi, lam, gF, "suzuki", 4, 10.0, 4, opts)
    with pytest.raises(RuntimeError, match="INVALID"):
        prop.set_wait_limit(-1)
    prop.set_wait_limit(0)
    psi = prop.pack([it.psi0])
    st = prop.propagate(psi, "midp", "suzuki", 4, 10.0, 2, opts)
    ref = prop.pack([it.psi0])
    gqd.from_items([it]).propagate(ref, "midp", "suzuki", 4, 10.0, 2, opts)
    print(f"after the limit is restored: {st.solves} solves, max |diff| "
          f"{float((psi - ref).abs().max()):.1e}", flush=True)
    assert st.nonfinite == 0 and torch.equal(psi, ref)


def test_preconditioner_is_rejected_on_2d_grids(gqd):
    it = moving_item(64, seed=2, p0=(1.0, 0.0))
    prop = gqd.from_items([it])
    psi = prop.pack([it.psi0])
    with pytest.raises(gqd.GqdError, match="1D grids"):
        prop.propagate(psi, "midp", "suzuki", 2, 10.0, 1, gqd.SolverOpts(tol=1e-14, precond=True))
    # the automatic choice is the plain solver on 2D grids
    x, y = prop.pack([it.psi0]), prop.pack([it.psi0])
    prop.propagate(x, "midp", "suzuki", 2, 10.0, 1, gqd.SolverOpts(tol=1e-14, precond="auto"))
    prop.propagate(y, "midp", "suzuki", 2, 10.0, 1, gqd.SolverOpts(tol=1e-14))
    assert torch.equal(x, y)
    prop.close()


def test_plain_launch_matches_cooperative_2d(gqd, monkeypatch):
    # GQD_2D_PLAIN_LAUNCH=1 launches the same grid as an ordinary kernel (for profilers
    # that fail on cooperative launches): the results must not change by a bit
    it = moving_item(128, seed=4, p0=(1.5, -1.0))
    prop = gqd.from_items([it])
    x, y = prop.pack([it.psi0]), prop.pack([it.psi0])
    opts = gqd.SolverOpts(tol=1e-14)
    sx = prop.propagate(x, "midp", "suzuki", 4, 10.0, 2, opts)
    monkeypatch.setenv("GQD_2D_PLAIN_LAUNCH", "1")
    sy = prop.propagate(y, "midp", "suzuki", 4, 10.0, 2, opts)
    monkeypatch.delenv("GQD_2D_PLAIN_LAUNCH")
    print(f"cooperative {sx.iterations} iterations, ordinary launch {sy.iterations}", flush=True)
    assert torch.equal(x, y) and sx.iterations == sy.iterations
    prop.close()


def test_implementation_bytes_count_second_passes_2d(gqd):
    # the 2D solver makes no three-term pre-projection: the extra vector passes are both
    # sweeps of its second Gram-Schmidt passes, an even count
    it = moving_item(64, seed=5)
    prop = gqd.from_items([it])
    psi = prop.pack([it.psi0])
    st = prop.propagate(psi, "midp", "suzuki", 4, 10.0, 2, gqd.SolverOpts(tol=1e-14))
    extra = (st.impl_bytes - st.alg_bytes) / (32.0 * 64 * 64)
    print(f"2D: {extra:.0f} extra vector passes, {st.iterations} iterations", flush=True)
    assert extra == round(extra) and extra >= 0 and round(extra) % 2 == 0
    prop.close()
