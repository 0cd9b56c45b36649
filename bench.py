"""Benchmark: grid-point.steps/s of 8th-order composed implicit midpoint at the step
that reaches convergence error 1e-10, on one MI355X.

Workload.  The two-surface NaI-like adiabatic model on N = 2048 points of [3, 16) bohr
(Morse + repulsive surfaces, Gaussian coupling), Suzuki-fractal composition of the
implicit midpoint method to order 8 (125 substeps per step), step dt = 10 a.u. (the
largest dt_k = 40 * 2^-k whose error at T = 4000 a.u. against the dt/8 order-8
reference is <= 1e-10; see paper_1902_04661_amd.convergence), GMRES tolerance 1e-14.
That packet (q0 = 5, p0 = 0, width 0.12, coupling amplitude 0.4 at q = 7), the one the
step-size sweep was run on, is replicated B times to fill the GPU (weak scaling by
batch); one "step" advances every copy by dt in one kernel launch.  One packet alone is
timed too (single_packet), and a seeded ragged batch of different packets and sizes
(ragged_batch).

Roofline: the propagation kernel against the HBM peak (8 TB/s) with algorithmic bytes
32 (I^2 + 4I + 8) per grid point per substep for a solve of I Arnoldi iterations
(S = 2 complex128 vectors, one Gram-Schmidt pass, fused H application), summed over
the solves of one launch and divided by the launch's average duration (HIP events
on the launch stream).  cpu_baseline: the CPU oracle timed on one host core over a
bounded sample of the same workload.
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
DT_STAR = 10.0
N = 2048
ORDER, SCHEME, METHOD = 8, "suzuki", "midp"
TOL = 1e-14

# Memory traffic of the propagation kernel from two rocprofv3 --pmc passes (FETCH_SIZE, then
# WRITE_SIZE) over one launch from t = 0 of this workload, scaled by what the counters read
# for a 1 GiB device copy (FETCH_SIZE 0.5x, WRITE_SIZE 1.0x of the true bytes).  The
# counters see what leaves the L2 caches, so reads served by the Infinity Cache count as
# well.  Valid only for the device sources it was taken on: reported as null once they
# change.
TRAFFIC = {
    "sources_sha256": "4b6731f3a4c6e76581b18648d82b3e2c2f496015a576d22917c0f8ac8f4a595f",
    "fetch_kib": 81256669.5, "fetch_scale": 2.0,
    "write_kib": 56882301.625, "write_scale": 1.0,
    "alg_bytes_same_launch": 330511155200.0,
    "summary": "profiles/k_run_2048_sz8_x1024.md",
}
DEVICE_SOURCES = ["gqd_kernels.hip", "gqd_device.hpp", "gqd_internal.h"]


def device_sources_sha() -> str:
    import hashlib
    outer = hashlib.sha256()
    for name in DEVICE_SOURCES:
        with open(os.path.join(ROOT, "paper_1902_04661_amd", "csrc", name), "rb") as f:
            outer.update((hashlib.sha256(f.read()).hexdigest() + "  paper_1902_04661_amd/csrc/"
                          + name + "\n").encode())
    return outer.hexdigest()


def measured_traffic():
    """(bytes per launch, ratio to that launch's algorithmic bytes), or (None, None)."""
    if device_sources_sha() != TRAFFIC["sources_sha256"]:
        return None, None
    t = 1024.0 * (TRAFFIC["fetch_kib"] * TRAFFIC["fetch_scale"] + TRAFFIC["write_kib"] * TRAFFIC["write_scale"])
    return t, t / TRAFFIC["alg_bytes_same_launch"]


def alg_bytes(n: int, st) -> float:
    """32 (I^2 + 4I + 8) bytes per grid point per solve, summed over the solves."""
    return 32.0 * n * (st.iterations_sq + 4 * st.iterations + 8 * st.solves)


def ragged_leg(gqd, inputs, dev, batch: int, steps: int) -> dict:
    """Ragged batch: seeded N in {256..4096}, centres, momenta, amplitudes; Suzuki order 6,
    dt = 10 a.u.; one launch per grid size on forked streams per step."""
    import torch
    items = inputs.ragged_batch(batch, seed=0)
    prop = gqd.from_items(items, device=dev)
    psi = prop.pack([it.psi0 for it in items])
    opts = gqd.SolverOpts(tol=TOL, restart=32)
    prop.propagate(psi, METHOD, SCHEME, 6, DT_STAR, 1, opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    byts = 0.0
    for _ in range(steps):
        st = prop.propagate(psi, METHOD, SCHEME, 6, DT_STAR, 1, opts)
        byts += st.alg_bytes
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    pts = int(sum(it.n for it in items))
    return {"value": pts * steps / el, "unit": "grid-point·steps/s", "ms_per_step": 1e3 * el / steps,
            "alg_GBps": byts / el / 1e9, "hbm_frac": byts / el / 1e9 / HBM_PEAK_GBS,
            "workload": f"{batch} packets, N in {{256..4096}} (sum {pts}), Suzuki order 6, dt={DT_STAR}"}


SOD_DT = 0.15  # below 1 / E_max of the N = 2048 grid on [3, 16) (E_max ~ 4.3 Ha)


def elementary_leg(gqd, inputs, dev, batch: int, steps: int) -> dict:
    """Second-order differencing (Eq. 16) on the benchmark's packet replicated `batch`
    times, at the largest round step below its stability limit.  One H application per
    step and grid point; algorithmic traffic 128 bytes per grid point per step (read
    psi(t) and psi(t - dt), write psi(t + dt) and the new previous state)."""
    import torch
    it = inputs.nai_like_item(N)
    prop = gqd.from_items([it] * batch, device=dev)
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
    out = {"workload": f"diabatic crossing model, {batch} x N={N}, Suzuki order {ORDER}, dt={DT_STAR}"}
    s = torch.cuda.current_stream()
    for name, item, method, nsteps in (("split_operator", diabatic.diabatic_as_surfaces(d), "split_operator", steps),
                                       ("adiabatic_midpoint", ad, METHOD, 1)):
        prop = gqd.from_items([item] * batch, device=dev)
        psi = prop.pack([item.psi0] * batch)
        opts = gqd.SolverOpts(tol=TOL, restart=32)
        prop.propagate(psi, method, SCHEME, ORDER, DT_STAR, 1, opts, stats=False)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(s)
        prop.propagate(psi, method, SCHEME, ORDER, DT_STAR, nsteps, opts, stats=False)
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
    prop = gqd.from_items([it], device=dev)
    psi = prop.pack([it.psi0])
    opts = gqd.SolverOpts(tol=TOL, restart=32)
    prop.propagate(psi, METHOD, SCHEME, ORDER, DT_STAR, 1, opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = prop.propagate(psi, METHOD, SCHEME, ORDER, DT_STAR, steps, opts)
    el = time.perf_counter() - t0
    return {"value": 256 * 256 * steps / el, "unit": "grid-point·steps/s", "ms_per_step": 1e3 * el / steps,
            "mean_gmres_iterations": st.iterations / max(st.solves, 1),
            "us_per_h_apply": 1e6 * el / max(st.h_applies, 1), "alg_GBps": st.alg_bytes / el / 1e9,
            "workload": f"2D 256x256, Suzuki order 8 midpoint, dt={DT_STAR}, {steps} steps"}


def adjoint2d_leg(gqd, inputs, dev, nsteps: int) -> dict:
    """Gradient of the final surface-2 population with respect to the four coupling
    parameters (A, c1, c2, w) on the 256 x 256 model: forward plus reverse sweep."""
    import torch
    from paper_1902_04661_amd import autograd as ag
    it = inputs.two_dim_item(256, 256)
    prop = gqd.from_items([it], device=dev)
    Q = ag.grid2d(256, it.qmin, it.qmax, dev)
    P = [torch.tensor(v, dtype=torch.float64, device=dev, requires_grad=True) for v in it.params["cparams"]]
    opts = gqd.SolverOpts(tol=TOL, restart=32)
    dv = ((it.qmax[0] - it.qmin[0]) / 256) * ((it.qmax[1] - it.qmin[1]) / 256)

    def gradient(steps):
        F = ag.coupling_2d(Q[0], Q[1], *P).reshape(-1)
        psiT = ag.propagate(prop, prop.pack([it.psi0]), F, "suzuki", 8, DT_STAR, steps, opts)
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
            "workload": f"2D 256x256, Suzuki order 8, dt={DT_STAR}, {nsteps} steps, forward + reverse"}


def adjoint_leg(gqd, inputs, dev, batch: int, nsteps: int) -> dict:
    """Gradients of the final surface-2 population with respect to (q0, p0, width, coupling
    amplitude, coupling centre) per packet: forward propagation plus the reverse sweep."""
    import torch
    from paper_1902_04661_amd import autograd as ag
    items = inputs.adjoint_batch(batch, seed=1, n=1024)
    prop = gqd.from_items(items, device=dev)
    q = ag.grid(1024, items[0].qmin, items[0].qmax, dev)
    P = {k: torch.tensor([it.params[k] for it in items], dtype=torch.float64, device=dev, requires_grad=True)
         for k in ["q0", "p0", "width", "amp", "center"]}
    opts = gqd.SolverOpts(tol=TOL, restart=32)

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
    return {"value": batch / el, "unit": "gradients/s", "params_per_gradient": 5, "seconds": el,
            "forward_only_seconds": fwd, "gradient_over_forward": el / fwd,
            "workload": f"{batch} packets, N=1024, Suzuki order 4, dt=4, {nsteps} steps, forward + reverse"}


def cpu_leg(seconds: float = 15.0) -> dict:
    """Oracle on one core: the first packet of the batch, SZ-8 steps of dt* until ~seconds."""
    code = f"""
import sys, time, json
sys.path.insert(0, {ROOT!r})
import oracle as O
from paper_1902_04661_amd import inputs as I
it = I.ragged_batch(1, seed=0, fixed_n={N})[0]
m = O.model_from_item(it)
opts = O.SolverOpts(tol={TOL}, restart=32)
psi = it.psi0
t0 = time.time(); steps = 0
while True:
    psi = O.propagate(m, psi, O.MIDP, O.SUZUKI, {ORDER}, {DT_STAR}, 1, opts)
    steps += 1
    if time.time() - t0 > {seconds} or steps >= 400:
        break
el = time.time() - t0
print(json.dumps(dict(steps=steps, seconds=el)))
"""
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, check=True)
    r = json.loads(out.stdout.strip().splitlines()[-1])
    return {"value": N * r["steps"] / r["seconds"], "unit": "grid-point·steps/s", "cores": 1,
            "kind": "oracle",
            "sample": f"1 packet, N={N}, {r['steps']} SZ-8 steps of dt={DT_STAR} in {r['seconds']:.1f} s "
                      f"(numpy FP64, one thread)"}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--single-steps", type=int, default=4)
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
    opts = gqd.SolverOpts(tol=TOL, restart=32)

    # ---------------------------------------------------------------- batched run
    items = [inputs.nai_like_item(N)] * args.batch
    prop = gqd.from_items(items, device=dev)
    psi0 = prop.pack([it.psi0 for it in items])
    psi = psi0.clone()
    stream = torch.cuda.current_stream()
    plans = prop.autotune(psi, METHOD, SCHEME, 2, DT_STAR, 1, opts) if not args.no_autotune else {}
    print(f"[bench] transform plans: {plans}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        prop.propagate(psi, METHOD, SCHEME, ORDER, DT_STAR, 1, opts)
    print(f"[bench] warmup {args.warmup} steps done, batch {args.batch}", file=sys.stderr, flush=True)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    bytes_total = 0.0
    iters = iters_sq = solves = applies = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        starts[k].record(stream)
        st = prop.propagate(psi, METHOD, SCHEME, ORDER, DT_STAR, 1, opts)   # one launch
        ends[k].record(stream)
        bytes_total += alg_bytes(N, st)
        iters += st.iterations
        iters_sq += st.iterations_sq
        solves += st.solves
        applies += st.h_applies
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    avg_kernel_s = sum(kern_ms) / len(kern_ms) / 1e3
    value = args.batch * N * args.steps / wall
    achieved = bytes_total / args.steps / avg_kernel_s / 1e9
    print(f"[bench] timed {args.steps} steps: {wall:.2f} s wall, kernel {avg_kernel_s * 1e3:.1f} ms/step, "
          f"mean GMRES iterations {iters / solves:.2f}", file=sys.stderr, flush=True)

    # conservation check on the batch (outside the timed region)
    check = {}
    if not args.no_check:
        d0 = prop.diag(psi0).cpu().numpy()
        d1 = prop.diag(psi).cpu().numpy()
        check = {"max_norm_drift": float(np.max(np.abs(d1[:, 0] - d0[:, 0]))),
                 "max_energy_drift": float(np.max(np.abs(d1[:, 1] - d0[:, 1])))}

    # ------------------------------------------------------------- single packet
    single = {}
    if args.single_steps > 0:
        it = inputs.nai_like_item(N)
        p1 = gqd.from_items([it], device=dev)
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
                  "workload": f"one packet q0=5 p0=0 w=0.12, N={N}, SZ-8 midpoint, dt={DT_STAR}"}
        print(f"[bench] single packet: {single['value']:.3e} gp.steps/s", file=sys.stderr, flush=True)

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
        cpu = cpu_leg()
        print(f"[bench] cpu oracle: {cpu['value']:.3e} gp.steps/s", file=sys.stderr, flush=True)

    traffic, traffic_ratio = measured_traffic() if args.batch == 1024 and not args.no_autotune else (None, None)
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
        "config": {"workload": f"nai2048_sz8_midpoint_dt10_x{args.batch}",
                   "model": "two-surface NaI-like adiabatic model, N=2048 on [3,16) bohr; "
                            "packet q0=5 p0=0 w=0.12 on surface 1, replicated",
                   "batch": args.batch, "n": N, "method": "implicit midpoint", "scheme": "suzuki",
                   "order": ORDER, "dt": DT_STAR, "gmres_tol": TOL, "restart": 32,
                   "substeps_per_step": 125, "parallelism": "one workgroup per wavepacket",
                   "transform_plan": list(plans.get(N, ())) or None},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_unit": "bytes per launch (launch from t = 0, rocprofv3 --pmc)",
                     "traffic_over_alg_bytes": traffic_ratio,
                     "kernel": "k_run<7> (propagate, N = 2048 plan 4-8-8-8)",
                     "alg_bytes_per_launch": bytes_total / args.steps,
                     "avg_launch_ms": avg_kernel_s * 1e3},
        "cpu_baseline": cpu,
        "single_packet": single,
        "ragged_batch": ragged,
        "adjoint": adjoint,
        "two_dim": twod,
        "adjoint_2d": adjoint2d,
        "elementary": elementary,
        "split_operator": split,
        # the batched and the differentiated forms against the plain one-packet solve, all
        # at the same tolerance and step
        "comparisons": {
            "batch_over_single_packet": value / single["value"] if single else None,
            "gradient_over_forward": adjoint.get("gradient_over_forward") if adjoint else None,
        },
        "gmres": {"mean_iterations": iters / solves, "h_applies_per_step": applies / args.steps,
                  "solves_per_step": solves / args.steps,
                  "substeps_per_s": solves / (avg_kernel_s * args.steps),
                  "h_applies_per_s": applies / (avg_kernel_s * args.steps)},
        "check": check,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
