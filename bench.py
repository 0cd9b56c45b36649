"""Benchmark: grid-point.steps/s of 8th-order composed implicit midpoint at the step
that reaches convergence error 1e-10, on one MI355X.

Workload.  1024 seeded draws of the two-surface NaI-like adiabatic model on N = 2048
points of [3, 16) bohr (Morse + repulsive surfaces, Gaussian coupling): packet centre
q0 ~ U[4.5, 6], momentum p0 ~ U[-5, 5], coupling amplitude ~ U[0.1, 0.8], width 0.12 (the
ragged batch's draws on one grid size).  Suzuki-fractal composition of the implicit
midpoint method to order 8 (125 substeps per step) at dt = 20 a.u.: the largest
dt_k = 40 * 2^-k whose convergence error at T = 4000 a.u. stays <= 1e-10 for the six
highest-energy draws of this batch (6.2e-11 at 20 a.u., 1.4e-8 at 40 a.u.; see
paper_1902_04661_amd.convergence), every system solved to stagnation (GMRES tolerance
1e-17), as in that sweep.  One "step" advances every packet by dt in one kernel launch;
by default 200 timed steps (after two warmup steps) cover the sweep's 4000 a.u.
Side legs: the 8th-order triple jump (0.625 a.u.) and the non-recursive optimal
compositions of orders 8 and 10 (2.5 and 10 a.u.) on the same batch, each at its own
1e-10 step from the same sweep; one packet alone; the 4096-packet ragged batch (N in
256..4096, Suzuki order 6 at its verified step 2.5 a.u.); 1D and 2D gradients; the 2D
model; the elementary and diabatic controls.

Solver: GMRES right-preconditioned by the exact inverse of the kinetic part of
1 + i a H (option precond; about half the iterations of the plain GMRES at N = 2048,
whose rate on the same batch is reported beside it as `plain_gmres`).

Roofline: the propagation kernel against the HBM peak (8 TB/s) with algorithmic bytes
32 (I^2 + 6I + 10) per grid point per substep for a preconditioned solve of I Arnoldi
iterations (32 (I^2 + 4I + 8) for the plain one; S = 2 complex128 vectors, one
Gram-Schmidt pass, fused H application), summed over the solves of one launch and
divided by the launch's average duration (HIP events on the launch stream).  cpu_baseline: the CPU oracle on draws of the same batch, one
packet per process on the host's cores, over a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "grid-point·steps/s at 1e-10 error, 8th order; adjoint grads/s; % HBM roofline"
HBM_PEAK_GBS = 8000.0
N = 2048
BATCH = 1024
ORDER, SCHEME, METHOD = 8, "suzuki", "midp"
# the step-size sweep's results for this batch (Suzuki and triple jump, order 8) and its
# solve tolerance; the ragged batch's step is verified by tests/test_gpu_step_verification
DT_STAR = 20.0
DT_STAR_TJ = 0.625
# the non-recursive optimal compositions (17 and 35 substeps) at their own 1e-10 steps
DT_STAR_OPT8 = 2.5
DT_STAR_OPT10 = 10.0
TOL = 1e-17
RAGGED_DT = 2.5
# GMRES right-preconditioned by the exact inverse of the kinetic part of 1 + i a H (the
# solver option precond, 1D): the same solutions to the solve tolerance in about half
# the iterations at N = 2048 and 20 a.u.; the legs whose systems are not stiff (the
# gradient at N = 1024 and 4 a.u., the diabatic comparison) and the 2D legs (no 2D
# preconditioner) run the plain solver
PRECOND = True
# the 2D model and the 1D gradient workload run at their configurations' own steps
DT_2D = 10.0
TOL_2D = 1e-14
TOL_ADJ = 1e-14

# Memory traffic of the propagation kernel (the preconditioned solver) from two rocprofv3
# --pmc passes (FETCH_SIZE, then WRITE_SIZE) over one launch from t = 0 of this workload,
# scaled by what the counters read for a 1 GiB device copy (FETCH_SIZE 0.5x, WRITE_SIZE
# 1.0x of the true bytes).  The
# counters see what leaves the L2 caches, so reads served by the Infinity Cache count as
# well.  Valid only for the device sources it was taken on: reported as null once they
# change.
TRAFFIC = {
    "sources_sha256": "333defb93d6eefbbe0ce562759214722a212ad56242de9fc71bc3be368adb126",
    "fetch_kib": 154135353.4375, "fetch_scale": 2.0,
    "write_kib": 109018168.0, "write_scale": 1.0,
    "alg_bytes_same_launch": 587887935488.0,
    "precond": True,
    "summary": "profiles/k_run_2048_sz8_draws1024_precond.md",
}
DEVICE_SOURCES = ["gqd_kernels.hip", "gqd_device.hpp", "gqd_internal.h", "gqd_compositions.h"]
DEVICE_SOURCES_2D = ["gqd_kernels2d.hip", "gqd_device.hpp", "gqd_internal.h", "gqd_compositions.h"]

# Memory traffic of the 2D kernel (256 x 256, Suzuki-8, dt = 10 a.u., tol 1e-14): the same
# two counter passes over one 5-step launch, with the same scale factors; reported as a
# ratio to the algorithmic bytes, valid only for the 2D device sources it was taken on.
TRAFFIC_2D = {
    "sources_sha256": "7bc5574f64499d8d1e4991857a96c6f336b54b760f89e573f35118b5094e1dd2",
    "fetch_kib": 14750646.9375, "fetch_scale": 2.0,
    "write_kib": 20801486.0625, "write_scale": 1.0,
    "alg_bytes_same_launch": 39048970240.0,
    "summary": "profiles/k_run2d_256_sz8.md",
}


def device_sources_sha(names=DEVICE_SOURCES) -> str:
    import hashlib
    outer = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, "paper_1902_04661_amd", "csrc", name), "rb") as f:
            outer.update((hashlib.sha256(f.read()).hexdigest() + "  paper_1902_04661_amd/csrc/"
                          + name + "\n").encode())
    return outer.hexdigest()


def measured_traffic(precond: bool):
    """(bytes per launch, ratio to that launch's algorithmic bytes), or (None, None)."""
    if device_sources_sha() != TRAFFIC["sources_sha256"] or precond != TRAFFIC["precond"]:
        return None, None
    t = 1024.0 * (TRAFFIC["fetch_kib"] * TRAFFIC["fetch_scale"] + TRAFFIC["write_kib"] * TRAFFIC["write_scale"])
    return t, t / TRAFFIC["alg_bytes_same_launch"]


def measured_traffic_2d():
    """Measured over algorithmic bytes of the 2D kernel, or None."""
    if device_sources_sha(DEVICE_SOURCES_2D) != TRAFFIC_2D["sources_sha256"]:
        return None
    t = 1024.0 * (TRAFFIC_2D["fetch_kib"] * TRAFFIC_2D["fetch_scale"]
                  + TRAFFIC_2D["write_kib"] * TRAFFIC_2D["write_scale"])
    return t / TRAFFIC_2D["alg_bytes_same_launch"]


def alg_bytes(n: int, st) -> float:
    """32 (I^2 + 4I + 8) bytes per grid point per solve, summed over the solves."""
    return 32.0 * n * (st.iterations_sq + 4 * st.iterations + 8 * st.solves)


def timed_launches(prop, psi, steps, method, scheme, order, dt, opts):
    """`steps` launches of one composed step each, timed with HIP events on the launch
    stream; returns (average launch seconds, wall seconds, summed statistics)."""
    import torch
    stream = torch.cuda.current_stream()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    tot = dict(bytes=0.0, impl_bytes=0.0, iterations=0, iterations_sq=0, solves=0, h_applies=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        starts[k].record(stream)
        st = prop.propagate(psi, method, scheme, order, dt, 1, opts)   # one launch
        ends[k].record(stream)
        tot["bytes"] += st.alg_bytes
        tot["impl_bytes"] += st.impl_bytes
        for key in ("iterations", "iterations_sq", "solves", "h_applies"):
            tot[key] += getattr(st, key)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern = sum(a.elapsed_time(b) for a, b in zip(starts, ends)) / steps / 1e3
    return kern, wall, tot


def ragged_leg(gqd, inputs, dev, batch: int, steps: int) -> dict:
    """Ragged batch: seeded N in {256..4096}, centres, momenta, amplitudes; Suzuki order 6
    at its verified step; one launch per grid size on forked streams per step."""
    import torch
    items = inputs.ragged_batch(batch, seed=0)
    # each size class with the solver its kinetic stiffness calls for (at 2.5 a.u. the
    # preconditioner pays on the N = 2048 and 4096 grids)
    opts = gqd.SolverOpts(tol=TOL, restart=32, precond="auto")
    with gqd.from_items(items, device=dev) as prop:
        psi = prop.pack([it.psi0 for it in items])
        prop.propagate(psi, METHOD, SCHEME, 6, RAGGED_DT, 1, opts)
        kern, wall, tot = timed_launches(prop, psi, steps, METHOD, SCHEME, 6, RAGGED_DT, opts)
    pts = int(sum(it.n for it in items))
    return {"value": pts * steps / wall, "unit": "grid-point·steps/s", "ms_per_step": 1e3 * wall / steps,
            "alg_GBps": tot["bytes"] / wall / 1e9, "hbm_frac": tot["bytes"] / wall / 1e9 / HBM_PEAK_GBS,
            "mean_gmres_iterations": tot["iterations"] / max(tot["solves"], 1),
            "workload": f"{batch} packets, N in {{256..4096}} (sum {pts}), Suzuki order 6, dt={RAGGED_DT}, "
                        f"GMRES tol {TOL:g}, preconditioner chosen per size class"}


def scheme_leg(gqd, inputs, dev, items, steps: int, scheme: str, order: int, dt: float) -> dict:
    """The same drawn batch under another composition at its own 1e-10 step: throughput
    per step and, comparable across schemes, simulated time per second (a.u./s)."""
    opts = gqd.SolverOpts(tol=TOL, restart=32, precond=PRECOND)
    with gqd.from_items(items, device=dev) as prop:
        psi = prop.pack([it.psi0 for it in items])
        prop.propagate(psi, METHOD, scheme, order, dt, 1, opts)
        kern, wall, tot = timed_launches(prop, psi, steps, METHOD, scheme, order, dt, opts)
        count = len(gqd.composition(scheme, order))
    return {"value": len(items) * N * steps / wall, "unit": "grid-point·steps/s",
            "ms_per_step": 1e3 * wall / steps, "simulated_au_per_s": dt * steps / wall,
            "mean_gmres_iterations": tot["iterations"] / max(tot["solves"], 1),
            "h_applies_per_au": tot["h_applies"] / (dt * steps) / len(items),
            "alg_GBps": tot["bytes"] / steps / kern / 1e9,
            "workload": f"{len(items)} drawn packets, N={N}, {scheme} order {order} ({count} substeps), "
                        f"dt={dt}, GMRES tol {TOL:g}"}


SOD_DT = 0.15  # below 1 / E_max of the N = 2048 grid on [3, 16) (E_max ~ 4.3 Ha)


def elementary_leg(gqd, inputs, dev, batch: int, steps: int) -> dict:
    """Second-order differencing (Eq. 16) on the resting packet replicated `batch` times,
    at the largest round step below its stability limit.  One H application per step and
    grid point; algorithmic traffic 128 bytes per grid point per step (read psi(t) and
    psi(t - dt), write psi(t + dt) and the new previous state)."""
    import torch
    it = inputs.nai_like_item(N)
    with gqd.from_items([it] * batch, device=dev) as prop:
        psi = prop.pack([it.psi0] * batch)
        prop.propagate(psi, "sod", "suzuki", 2, SOD_DT, 2, stats=False)
        s = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(s)
        prop.propagate(psi, "sod", "suzuki", 2, SOD_DT, steps, stats=False)
        e1.record(s)
        torch.cuda.synchronize()
        el = e0.elapsed_time(e1) * 1e-3
    gps = batch * N * steps / el
    return {"value": gps, "unit": "grid-point·steps/s", "ms_per_step": 1e3 * el / steps,
            "us_per_h_apply_per_packet": 1e6 * el * 256 / (batch * (steps + 1)),
            "alg_GBps": 128.0 * gps / 1e9, "hbm_frac": 128.0 * gps / 1e9 / HBM_PEAK_GBS,
            "workload": f"second-order differencing, {batch} x N={N} packet, dt={SOD_DT}, {steps} steps"}


def split_leg(gqd, inputs, dev, batch: int, steps: int) -> dict:
    """The two-state crossing model in both representations, `batch` copies of N = 2048,
    8th-order Suzuki at dt = 10 a.u.: the diabatic split-operator method (Table I; no
    linear solves, the state stays in registers) against the adiabatic implicit
    midpoint on the surfaces and coupling that Eqs. (24-28) give for the same model."""
    import torch
    from paper_1902_04661_amd import diabatic
    d = inputs.diabatic_crossing_item(N)
    ad, _ = diabatic.adiabatic_item(d)
    dt = 10.0
    out = {"workload": f"diabatic crossing model, {batch} x N={N}, Suzuki order {ORDER}, dt={dt}, GMRES tol 1e-14"}
    s = torch.cuda.current_stream()
    for name, item, method, nsteps in (("split_operator", diabatic.diabatic_as_surfaces(d), "split_operator", steps),
                                       ("adiabatic_midpoint", ad, METHOD, 1)):
        with gqd.from_items([item] * batch, device=dev) as prop:
            psi = prop.pack([item.psi0] * batch)
            # plain GMRES: at 10 a.u. on this model the preconditioner's extra transform
            # pair per iteration costs more than the iterations it saves
            opts = gqd.SolverOpts(tol=1e-14, restart=32)
            prop.propagate(psi, method, SCHEME, ORDER, dt, 1, opts, stats=False)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(s)
            prop.propagate(psi, method, SCHEME, ORDER, dt, nsteps, opts, stats=False)
            e1.record(s)
            torch.cuda.synchronize()
            el = e0.elapsed_time(e1) * 1e-3
        out[name] = {"value": batch * N * nsteps / el, "unit": "grid-point·steps/s",
                     "ms_per_step": 1e3 * el / nsteps}
    out["split_over_adiabatic"] = out["split_operator"]["value"] / out["adiabatic_midpoint"]["value"]
    return out


def twod_leg(gqd, inputs, dev, steps: int) -> dict:
    """256 x 256 two-surface model (vector coupling, seeded ridge), Suzuki order 8,
    implicit midpoint, dt = 10 a.u.: one item shared by a group of workgroups."""
    import torch
    it = inputs.two_dim_item(256, 256)
    opts = gqd.SolverOpts(tol=TOL_2D, restart=32)
    with gqd.from_items([it], device=dev) as prop:
        psi = prop.pack([it.psi0])
        prop.propagate(psi, METHOD, SCHEME, ORDER, DT_2D, 1, opts)
        s = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(s)
        st = prop.propagate(psi, METHOD, SCHEME, ORDER, DT_2D, steps, opts)
        e1.record(s)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        kern = e0.elapsed_time(e1) * 1e-3
    gbs = st.alg_bytes / kern / 1e9
    ratio = measured_traffic_2d()
    return {"value": 256 * 256 * steps / el, "unit": "grid-point·steps/s", "ms_per_step": 1e3 * el / steps,
            "mean_gmres_iterations": st.iterations / max(st.solves, 1),
            "us_per_h_apply": 1e6 * el / max(st.h_applies, 1),
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBS, "kernel": "k_run2d<256>", "launch_ms": kern * 1e3,
                         "alg_bytes": st.alg_bytes, "impl_over_alg_bytes": st.impl_bytes / st.alg_bytes,
                         "traffic": None if ratio is None else ratio * st.alg_bytes,
                         "traffic_over_alg_bytes": ratio,
                         "traffic_source": TRAFFIC_2D["summary"]},
            "workload": f"2D 256x256, Suzuki order 8 midpoint, dt={DT_2D}, {steps} steps, GMRES tol {TOL_2D:g}"}


def adjoint2d_leg(gqd, inputs, dev, nsteps: int) -> dict:
    """Gradient of the final surface-2 population with respect to the four coupling
    parameters (A, c1, c2, w) on the 256 x 256 model: forward plus reverse sweep."""
    import torch
    from paper_1902_04661_amd import autograd as ag
    it = inputs.two_dim_item(256, 256)
    Q = ag.grid2d(256, it.qmin, it.qmax, dev)
    P = [torch.tensor(v, dtype=torch.float64, device=dev, requires_grad=True) for v in it.params["cparams"]]
    opts = gqd.SolverOpts(tol=TOL_2D, restart=32)
    dv = ((it.qmax[0] - it.qmin[0]) / 256) * ((it.qmax[1] - it.qmin[1]) / 256)
    with gqd.from_items([it], device=dev) as prop:
        def gradient(steps):
            F = ag.coupling_2d(Q[0], Q[1], *P).reshape(-1)
            psiT = ag.propagate(prop, prop.pack([it.psi0]), F, "suzuki", 8, DT_2D, steps, opts)
            L = ag.surface_population(psiT.reshape(2, 256, 256), dv)
            L.backward()
            return L

        gradient(1)  # warm-up: workspace, kernel loading, autograd set-up
        for p in P:
            p.grad = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L = gradient(nsteps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    return {"value": 1.0 / el, "unit": "gradients/s", "params_per_gradient": 4, "seconds": el,
            "loss": float(L.detach()), "grad": [float(p.grad) for p in P],
            "workload": f"2D 256x256, Suzuki order 8, dt={DT_2D}, {nsteps} steps, forward + reverse"}


def adjoint_leg(gqd, inputs, dev, batch: int, nsteps: int) -> dict:
    """Gradients of the final surface-2 population with respect to (q0, p0, width, coupling
    amplitude, coupling centre) per packet: forward propagation plus the reverse sweep."""
    import torch
    from paper_1902_04661_amd import autograd as ag
    items = inputs.adjoint_batch(batch, seed=1, n=1024)
    q = ag.grid(1024, items[0].qmin, items[0].qmax, dev)
    P = {k: torch.tensor([it.params[k] for it in items], dtype=torch.float64, device=dev, requires_grad=True)
         for k in ["q0", "p0", "width", "amp", "center"]}
    # plain GMRES: at N = 1024 and 4 a.u. the kinetic part is not stiff (a T_max = 1.15),
    # and over the 1000 steps the preconditioner's extra transform pair per iteration
    # costs more than the 3 % of iterations it saves (78.9 against 86.7 gradients/s; over
    # the first 200 steps, where it saves 13 %, it is the faster, 364 against 311)
    opts = gqd.SolverOpts(tol=TOL_ADJ, restart=32)
    with gqd.from_items(items, device=dev) as prop:
        def gradient(steps):
            psi0 = ag.gaussian_packets(q, P["q0"], P["p0"], P["width"]).reshape(-1)
            F = ag.couplings(q, P["amp"], P["center"]).reshape(-1)
            psiT = ag.propagate(prop, psi0, F, "suzuki", 4, 4.0, steps, opts)
            L = (items[0].dq * torch.abs(psiT.reshape(batch, 2, 1024)[:, 1]) ** 2).sum()
            L.backward()
            return psi0

        gradient(1)  # warm-up: workspace, kernel loading, autograd set-up
        for v in P.values():
            v.grad = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        psi0 = gradient(nsteps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        # the plain forward solve of the same packets at the same tolerance, for comparison
        psi = psi0.detach().clone()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        prop.propagate(psi, "midp", "suzuki", 4, 4.0, nsteps, opts, stats=False)
        torch.cuda.synchronize()
        fwd = time.perf_counter() - t1
        # the reverse sweep alone from that psi(T), timed on its stream: its algorithmic
        # bytes are those of its solves (two per substep) plus, per grid point and
        # substep, reading phi, mu, psi and lambda, writing psi and lambda (6 state
        # vectors of 32 B) and updating dL/dF12 (16 B)
        lam = torch.zeros_like(psi)
        lv = lam.view(batch, 2, 1024)
        lv[:, 1] = items[0].dq * psi.view(batch, 2, 1024)[:, 1]
        gF = torch.zeros(batch * 1024, dtype=torch.float64, device=dev)
        s = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(s)
        st = prop.adjoint(psi, lam, gF, "suzuki", 4, 4.0, nsteps, opts)
        e1.record(s)
        torch.cuda.synchronize()
        rev = e0.elapsed_time(e1) * 1e-3
    rev_bytes = st.alg_bytes + 208.0 * 1024 * batch * 5 * nsteps
    return {"value": batch / el, "unit": "gradients/s", "params_per_gradient": 5, "seconds": el,
            "forward_only_seconds": fwd, "gradient_over_forward": el / fwd,
            "reverse_sweep": {"seconds": rev, "mean_gmres_iterations": st.iterations / max(st.solves, 1),
                              "roofline": {"bound": "hbm", "achieved": rev_bytes / rev / 1e9, "peak": HBM_PEAK_GBS,
                                           "unit": "GB/s", "frac": rev_bytes / rev / 1e9 / HBM_PEAK_GBS,
                                           "kernel": "k_run<4> (reverse sweep, N = 1024)", "alg_bytes": rev_bytes}},
            "workload": f"{batch} packets, N=1024, Suzuki order 4, dt=4, {nsteps} steps, forward + reverse, "
                        f"GMRES tol {TOL_ADJ:g}"}


CPU_PACKET = """
import sys, time, json
sys.path.insert(0, {root!r})
import oracle as O
from paper_1902_04661_amd import inputs as I
b = int(sys.argv[1])
it = I.ragged_batch({batch}, seed=0, fixed_n={n})[b]
m = O.model_from_item(it)
opts = O.SolverOpts(tol={tol}, restart=32, precond={precond})
psi = it.psi0
t0 = time.time(); steps = 0
while True:
    psi = O.propagate(m, psi, O.MIDP, O.SUZUKI, {order}, {dt}, 1, opts)
    steps += 1
    if time.time() - t0 > {seconds}:
        break
print(json.dumps(dict(steps=steps, seconds=time.time() - t0)))
"""


def cpu_leg(seconds: float = 20.0, workers: int = 0) -> dict:
    """The oracle on the host's cores: one process per core, each propagating one packet
    of the benchmark's drawn batch (draw b on process b) by whole Suzuki-8 steps of dt*
    at the same solve tolerance for about `seconds`.  value = sum over processes of
    N x steps, over the wall time of the pool."""
    cores = workers or min(16, os.cpu_count() or 1)
    code = CPU_PACKET.format(root=ROOT, batch=BATCH, n=N, tol=TOL, order=ORDER, dt=DT_STAR, seconds=seconds,
                             precond=PRECOND)
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    t0 = time.perf_counter()
    procs = [subprocess.Popen([sys.executable, "-c", code, str(b)], env=env, stdout=subprocess.PIPE, text=True)
             for b in range(cores)]
    outs = [json.loads(p.communicate()[0].strip().splitlines()[-1]) for p in procs]
    wall = time.perf_counter() - t0
    if any(p.returncode for p in procs):
        raise RuntimeError("a CPU oracle process failed")
    steps = sum(o["steps"] for o in outs)
    return {"value": N * steps / wall, "unit": "grid-point·steps/s", "cores": cores, "kind": "oracle",
            "sample": f"draws 0..{cores - 1} of the benchmark batch, N={N}, one process (numpy FP64, one "
                      f"thread) per packet, {steps} SZ-8 steps of dt={DT_STAR} in total (each process "
                      f"{min(o['steps'] for o in outs)}-{max(o['steps'] for o in outs)} steps), "
                      f"GMRES tol {TOL:g}{', kinetic preconditioner' if PRECOND else ''}, {wall:.1f} s wall"}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    # 200 steps of 20 a.u.: the whole 4000 a.u. of the step-size sweep
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=BATCH)
    ap.add_argument("--single-steps", type=int, default=4)
    ap.add_argument("--tj-steps", type=int, default=20, help="triple-jump leg (0: skip)")
    ap.add_argument("--opt-steps", type=int, default=8, help="optimal 8th- and 10th-order legs (0: skip)")
    ap.add_argument("--no-precond", action="store_true", help="headline with the plain GMRES of Sec. II.C")
    ap.add_argument("--plain-steps", type=int, default=10,
                    help="the headline batch under the plain GMRES, for comparison (0: skip)")
    ap.add_argument("--ragged-batch", type=int, default=4096)
    ap.add_argument("--ragged-steps", type=int, default=2)
    ap.add_argument("--adjoint-batch", type=int, default=256)
    ap.add_argument("--adjoint-steps", type=int, default=1000)
    ap.add_argument("--twod-steps", type=int, default=100)
    ap.add_argument("--sod-steps", type=int, default=400, help="elementary-method leg (0: skip)")
    ap.add_argument("--split-steps", type=int, default=8, help="diabatic split-operator leg (0: skip)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default transform plans")
    ap.add_argument("--adjoint2d-steps", type=int, default=400)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device once (HBM counter calibration)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs each batch on a single MI355X; "
              "items are independent, and sharding a batch across GPUs is not implemented.",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch
    from paper_1902_04661_amd import gqd, inputs

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        src = torch.ones(args.copy_calibration << 17, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 8}), flush=True)
        return 0
    precond = PRECOND and not args.no_precond
    opts = gqd.SolverOpts(tol=TOL, restart=32, precond=precond)

    # ---------------------------------------------------------------- batched run
    items = inputs.ragged_batch(args.batch, seed=0, fixed_n=N)
    prop = gqd.from_items(items, device=dev)
    psi0 = prop.pack([it.psi0 for it in items])
    psi = psi0.clone()
    plans = prop.autotune(psi, METHOD, SCHEME, 2, DT_STAR, 1, opts) if not args.no_autotune else {}
    print(f"[bench] transform plans: {plans}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        prop.propagate(psi, METHOD, SCHEME, ORDER, DT_STAR, 1, opts)
    print(f"[bench] warmup {args.warmup} steps done, batch {args.batch}", file=sys.stderr, flush=True)
    avg_kernel_s, wall, tot = timed_launches(prop, psi, args.steps, METHOD, SCHEME, ORDER, DT_STAR, opts)
    value = args.batch * N * args.steps / wall
    achieved = tot["bytes"] / args.steps / avg_kernel_s / 1e9
    iters, solves = tot["iterations"], tot["solves"]
    print(f"[bench] timed {args.steps} steps: {wall:.2f} s wall, kernel {avg_kernel_s * 1e3:.1f} ms/step, "
          f"mean GMRES iterations {iters / solves:.2f}", file=sys.stderr, flush=True)

    # conservation check on the batch (outside the timed region)
    check = {}
    if not args.no_check:
        d0 = prop.diag(psi0).cpu().numpy()
        d1 = prop.diag(psi).cpu().numpy()
        check = {"max_norm_drift": float(np.max(np.abs(d1[:, 0] - d0[:, 0]))),
                 "max_energy_drift": float(np.max(np.abs(d1[:, 1] - d0[:, 1])))}
    prop.close()

    # ------------------------------------------------------------- single packet
    single = {}
    if args.single_steps > 0:
        it = items[0]
        with gqd.from_items([it], device=dev) as p1:
            s1 = p1.pack([it.psi0])
            p1.propagate(s1, METHOD, SCHEME, ORDER, DT_STAR, 1, opts)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st1 = p1.propagate(s1, METHOD, SCHEME, ORDER, DT_STAR, args.single_steps, opts)
            torch.cuda.synchronize()
            el1 = time.perf_counter() - t1
        single = {"value": N * args.single_steps / el1, "unit": "grid-point·steps/s",
                  "ms_per_step": 1e3 * el1 / args.single_steps,
                  "mean_gmres_iterations": st1.iterations / max(st1.solves, 1),
                  "us_per_h_apply": 1e6 * el1 / max(st1.h_applies, 1),
                  "workload": f"draw 0 of the batch alone, N={N}, SZ-8 midpoint, dt={DT_STAR}, GMRES tol {TOL:g}"}
        print(f"[bench] single packet: {single['value']:.3e} gp.steps/s", file=sys.stderr, flush=True)

    # the same batch under the plain GMRES (Sec. II.C, no preconditioner) from t = 0
    plain = {}
    if precond and args.plain_steps > 0:
        popts = gqd.SolverOpts(tol=TOL, restart=32)
        with gqd.from_items(items, device=dev) as pp:
            ps = pp.pack([it.psi0 for it in items])
            pp.propagate(ps, METHOD, SCHEME, ORDER, DT_STAR, 1, popts)
            pk, pw, pt = timed_launches(pp, ps, args.plain_steps, METHOD, SCHEME, ORDER, DT_STAR, popts)
        pa = pt["bytes"] / args.plain_steps / pk / 1e9
        plain = {"value": args.batch * N * args.plain_steps / pw, "unit": "grid-point·steps/s",
                 "ms_per_step": 1e3 * pw / args.plain_steps,
                 "mean_gmres_iterations": pt["iterations"] / max(pt["solves"], 1),
                 "roofline": {"bound": "hbm", "achieved": pa, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": pa / HBM_PEAK_GBS, "kernel": "k_run<7> (plain GMRES)",
                              "impl_over_alg_bytes": pt["impl_bytes"] / pt["bytes"]},
                 "workload": f"the headline batch from t = 20 a.u., {args.plain_steps} steps, plain GMRES"}
        print(f"[bench] plain GMRES: {plain['ms_per_step']:.1f} ms/step, "
              f"{plain['mean_gmres_iterations']:.2f} iterations per solve", file=sys.stderr, flush=True)

    # the scheme comparisons take Suzuki-8 over a window like the other legs' (from one
    # warmup step on, a few steps), not the headline's 4000 a.u., whose later steps need
    # more iterations as the packets move
    tj, opt8, opt10, sz_early = {}, {}, {}, {}
    if args.tj_steps > 0 or args.opt_steps > 0:
        sz_early = scheme_leg(gqd, inputs, dev, items, 4, SCHEME, ORDER, DT_STAR)
    if args.tj_steps > 0:
        tj = scheme_leg(gqd, inputs, dev, items, args.tj_steps, "triple_jump", ORDER, DT_STAR_TJ)
        print(f"[bench] triple jump 8: {tj['value']:.3e} gp.steps/s, {tj['simulated_au_per_s']:.1f} a.u./s",
              file=sys.stderr, flush=True)
    if args.opt_steps > 0:
        opt8 = scheme_leg(gqd, inputs, dev, items, args.opt_steps, "optimal", 8, DT_STAR_OPT8)
        opt10 = scheme_leg(gqd, inputs, dev, items, args.opt_steps, "optimal", 10, DT_STAR_OPT10)
        print(f"[bench] optimal 8: {opt8['simulated_au_per_s']:.1f} a.u./s; optimal 10: "
              f"{opt10['simulated_au_per_s']:.1f} a.u./s", file=sys.stderr, flush=True)
    ragged = {}
    if args.ragged_batch > 0 and args.ragged_steps > 0:
        ragged = ragged_leg(gqd, inputs, dev, args.ragged_batch, args.ragged_steps)
        print(f"[bench] ragged batch: {ragged['value']:.3e} gp.steps/s", file=sys.stderr, flush=True)
    adjoint = {}
    if args.adjoint_batch > 0 and args.adjoint_steps > 0:
        adjoint = adjoint_leg(gqd, inputs, dev, args.adjoint_batch, args.adjoint_steps)
        print(f"[bench] adjoint: {adjoint['value']:.1f} gradients/s", file=sys.stderr, flush=True)

    elementary = {}
    if args.sod_steps > 0:
        elementary = elementary_leg(gqd, inputs, dev, args.batch, args.sod_steps)
        print(f"[bench] second-order differencing: {elementary['value']:.3e} gp.steps/s "
              f"({100 * elementary['hbm_frac']:.0f} % of HBM peak)", file=sys.stderr, flush=True)
    split = {}
    if args.split_steps > 0:
        split = split_leg(gqd, inputs, dev, args.batch, args.split_steps)
        print(f"[bench] split operator: {split['split_operator']['value']:.3e} gp.steps/s, "
              f"{split['split_over_adiabatic']:.1f}x the adiabatic midpoint on the same model",
              file=sys.stderr, flush=True)
    twod = {}
    if args.twod_steps > 0:
        twod = twod_leg(gqd, inputs, dev, args.twod_steps)
        print(f"[bench] 2D: {twod['value']:.3e} gp.steps/s", file=sys.stderr, flush=True)
    adjoint2d = {}
    if args.adjoint2d_steps > 0:
        adjoint2d = adjoint2d_leg(gqd, inputs, dev, args.adjoint2d_steps)
        print(f"[bench] 2D adjoint: {adjoint2d['value']:.4f} gradients/s", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_leg(args.cpu_seconds)
        print(f"[bench] cpu oracle: {cpu['value']:.3e} gp.steps/s on {cpu['cores']} cores",
              file=sys.stderr, flush=True)

    traffic, traffic_ratio = (measured_traffic(precond) if args.batch == BATCH and not args.no_autotune
                              else (None, None))
    sim = DT_STAR * args.steps / wall
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "grid-point·steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"nai2048_draws{args.batch}_sz8_midpoint_dt{DT_STAR:g}",
                   "model": "two-surface NaI-like adiabatic model, N=2048 on [3,16) bohr; seeded draws "
                            "q0~U[4.5,6], p0~U[-5,5], coupling amplitude~U[0.1,0.8], width 0.12 (seed 0)",
                   "batch": args.batch, "n": N, "method": "implicit midpoint", "scheme": "suzuki",
                   "order": ORDER, "dt": DT_STAR, "gmres_tol": TOL, "restart": 32,
                   "gmres_preconditioner": "right, (1 + i a p^2/2m)^-1" if precond else None,
                   "substeps_per_step": 125, "parallelism": "one workgroup per wavepacket",
                   "dt_star_error": "<= 1e-10 at T=4000 a.u. for the batch's six highest-energy draws "
                                    "(6.2e-11 worst; 1.4e-8 at dt=40)",
                   "transform_plan": list(plans.get(N, ())) or None},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_unit": "bytes per launch (launch from t = 0, rocprofv3 --pmc)",
                     "traffic_over_alg_bytes": traffic_ratio,
                     "kernel": "k_run<7%s> (propagate, N = 2048 plan 4-8-8-8)" % (", precond" if precond else ""),
                     "alg_bytes_per_launch": tot["bytes"] / args.steps,
                     # the implementation's own sweeps beyond the algorithmic count (second
                     # Gram-Schmidt passes), from the library's statistics
                     "impl_bytes_per_launch": tot["impl_bytes"] / args.steps,
                     "impl_over_alg_bytes": tot["impl_bytes"] / tot["bytes"],
                     "avg_launch_ms": avg_kernel_s * 1e3},
        "cpu_baseline": cpu,
        "single_packet": single,
        "plain_gmres": plain,
        "triple_jump_8": tj,
        "optimal_8": opt8,
        "optimal_10": opt10,
        "ragged_batch": ragged,
        "adjoint": adjoint,
        "two_dim": twod,
        "adjoint_2d": adjoint2d,
        "elementary": elementary,
        "split_operator": split,
        # the batched and the differentiated forms against the plain one-packet solve, all
        # at the same tolerance and step; the other compositions at their own 1e-10 steps
        "comparisons": {
            "batch_over_single_packet": value / single["value"] if single else None,
            "gradient_over_forward": adjoint.get("gradient_over_forward") if adjoint else None,
            "simulated_au_per_s_suzuki8": sim,
            "suzuki8_early_window": sz_early,
            "suzuki8_over_triple_jump8_at_1e-10":
                sz_early["simulated_au_per_s"] / tj["simulated_au_per_s"] if tj else None,
            "optimal8_over_suzuki8_at_1e-10":
                opt8["simulated_au_per_s"] / sz_early["simulated_au_per_s"] if opt8 else None,
            "optimal10_over_suzuki8_at_1e-10":
                opt10["simulated_au_per_s"] / sz_early["simulated_au_per_s"] if opt10 else None,
            "h_applies_per_au_suzuki8": tot["h_applies"] / (DT_STAR * args.steps) / args.batch,
        },
        "gmres": {"mean_iterations": iters / solves, "h_applies_per_step": tot["h_applies"] / args.steps,
                  "solves_per_step": solves / args.steps,
                  "substeps_per_s": solves / (avg_kernel_s * args.steps),
                  "h_applies_per_s": tot["h_applies"] / (avg_kernel_s * args.steps)},
        "check": check,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
