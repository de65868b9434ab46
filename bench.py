"""Throughput of the multiphase curved-boundary LBM step on one MI355X.

A step is one pass of the whole hot path over the lattice: the fused kernel that pulls the
populations, applies the curved-boundary links (eqs. 16-18), computes the pseudopotential force and
collides. Inputs are resident in HBM before the timed region starts. Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload c2] [--precision f32s] [--bc-mode present]
                    [--collision bgk] [--model pseudo] [--gravity 0,0] [--no-cpu] [--no-adjoint]

Default: the 4096^2 D2Q9 workload (4800 circles, 640 drops) with shifted-FP32 storage, its 5000
steps, as the throughput and HBM-roofline figures are quoted on it; the oracle is timed on a
bounded sample of the same workload.  The forward + reverse-mode figure is measured on the 512^2
rough-wall workload (2000 steps, checkpoints every 100 steps), as the gradient is defined there.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2203_04508_amd.roofline import HBM_PEAK_GBS, STORAGE_BYTES, algorithmic_bytes, layout_bytes  # noqa: E402

METRIC = "MLUPS & % HBM roofline per step; fwd+adjoint MLUPS; relative mass drift"
DTYPES = {"f64": "f64", "f32s": "f32", "f16s": "f32"}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def setup_gpu(wl, precision, rho_ref, bc_mode="present", collision="bgk", model="pseudo", gravity=(0.0, 0.0, 0.0)):
    from paper_2203_04508_amd import mcb
    from paper_2203_04508_amd import workloads as W

    if model == "chempot":
        # the paper's chemical-potential model on the same geometry: Peng-Robinson at 0.8 T_c
        lat = mcb.Lattice(wl.dim, wl.dims, wl.tau, 0.8 * W.PR_TC, precision=precision, rho_ref=rho_ref,
                          bc_mode=bc_mode, collision=collision, gravity=gravity[:wl.dim], model="chempot",
                          cp_k=W.CP_K, cp_kappa=W.CP_KAPPA)
        nl, nb, nw = lat.set_geometry(wl.shapes)
        rho0, mu_s, _ = W.chempot_inputs(wl, lat.wall_nodes())
        lat.set_wettability(mu_s)
        lat.init_equilibrium(rho0)
        return lat, (nl, nb, nw)
    lat = mcb.Lattice(wl.dim, wl.dims, wl.tau, wl.T, precision=precision, rho_ref=rho_ref, bc_mode=bc_mode,
                      collision=collision, gravity=gravity[:wl.dim])
    nl, nb, nw = lat.set_geometry(wl.shapes)
    lat.set_wettability(W.phi_for_walls(wl, lat.wall_nodes()))
    lat.init_equilibrium(wl.rho0())
    return lat, (nl, nb, nw)


def fwd_adjoint(precision):
    """Forward with checkpoints + reverse mode on the 512^2 rough-wall workload.  value: lattice
    updates of the forward steps, the recomputed steps and the reverse steps per second of the whole
    (forward + backward) time; trajectory_mlups: forward lattice updates per second of that time."""
    import torch
    from paper_2203_04508_amd import mcb, workloads as W

    wl = W.make("c3")
    rr = wl.rho_v if precision != "f64" else 0.0
    lat = mcb.Lattice(wl.dim, wl.dims, wl.tau, wl.T, precision=precision, rho_ref=rr)
    lat.set_geometry(wl.shapes)
    lat.set_wettability(W.phi_for_walls(wl, lat.wall_nodes()))
    rho0 = wl.rho0()
    k = 100
    lat.adj_forward(rho0, 200, k, mcb.LOSS_COM_X, (wl.rho_v, 1.0))  # warm-up (arena, code paths)
    lat.adj_backward(1.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss = lat.adj_forward(rho0, wl.steps, k, mcb.LOSS_COM_X, (wl.rho_v, 1.0))
    t1 = time.perf_counter()
    g = lat.adj_backward(1.0)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    lat.close()
    nck = (wl.steps + k - 1) // k
    updates = wl.steps + (wl.steps - nck) + wl.steps  # forward, recomputed in the segments, reverse
    return {
        "workload": f"c3: D2Q9 {wl.dims[0]}x{wl.dims[1]} rough wall, {wl.steps} steps, checkpoint every {k}",
        "precision": precision,
        "loss": "centre-of-mass x of the drop",
        "value": wl.N * updates / (t2 - t0) / 1e6,
        "trajectory_mlups": wl.N * wl.steps / (t2 - t0) / 1e6,
        "unit": "MLUPS",
        "forward_s": t1 - t0,
        "backward_s": t2 - t1,
        "loss_value": float(loss),
        "grad_entries": int(len(g)),
    }


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, budget_s=12.0, single_s=4.0, bc_mode="present", collision="bgk", model="pseudo",
                 gravity=(0.0, 0.0)):
    """The FP64 oracle, as it stands, on a bounded sample of the same workload (same boundary
    scheme and collision): all threads OpenMP gives it, then one thread."""
    from oracle import oracle
    from paper_2203_04508_amd import workloads as W

    P = oracle.make_params(wl.dim, *wl.dims, tau=wl.tau, T=wl.T)
    sim, (solid, *_rest) = oracle.sim_from_shapes(P, wl.shapes)
    sim.set_bc_mode({"present": 0, "ibc": 1, "mibc": 2, "hbbc": 3}[bc_mode])
    if collision == "mrt":
        sim.set_mrt()
    if any(g != 0.0 for g in gravity):
        sim.set_gravity(tuple(gravity))
    if model == "chempot":
        sim.set_chempot(0.8 * W.PR_TC, k=W.CP_K, kappa=W.CP_KAPPA)
        rho0, mu_s, _ = W.chempot_inputs(wl, oracle.wall_nodes(P, solid))
        sim.set_mu_wall(mu_s)
    else:
        sim.set_phi(W.phi_for_walls(wl, oracle.wall_nodes(P, solid)))
        rho0 = wl.rho0()
    sim.init_eq(rho0)
    sim.step(1)

    def timed(budget):
        steps, t0 = 0, time.perf_counter()
        while True:
            sim.step(1)
            steps += 1
            el = time.perf_counter() - t0
            if el > budget or steps >= 1000:
                return steps, el

    threads = oracle.num_threads()
    steps, el = timed(budget_s)
    oracle.set_threads(1)
    s1, e1 = timed(single_s)
    oracle.set_threads(threads)
    return {
        "value": wl.N * steps / el / 1e6,
        "unit": "MLUPS",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{steps} steps of workload {wl.name} ({'x'.join(map(str, wl.dims[:wl.dim]))}) after set-up, FP64"
                  + (f", {model} model, {collision}" if model != "pseudo" or collision != "bgk" else "")
                  + (f", gravity {tuple(gravity)}" if any(g != 0.0 for g in gravity) else ""),
        "cpu_model": _cpu_model(),
        "single_thread_value": wl.N * s1 / e1 / 1e6,
        "single_thread_sample": f"{s1} steps, 1 thread",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--precision", default="f32s", choices=list(DTYPES))
    ap.add_argument("--bc-mode", default="present", choices=["present", "ibc", "mibc", "hbbc"])
    ap.add_argument("--collision", default="bgk", choices=["bgk", "mrt"])
    ap.add_argument("--model", default="pseudo", choices=["pseudo", "chempot"])
    ap.add_argument("--gravity", default="0,0,0", help="body-force acceleration gx,gy[,gz] (lattice units)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the step would shard by "
              "domain decomposition with a two-node halo, which is not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2203_04508_amd import workloads as W
    from paper_2203_04508_amd import build as hipbuild, mcb as _mcb

    if not os.path.exists(_mcb.LIB_PATH):
        hipbuild.build()  # nothing built yet: compile the library (the loader itself never falls back)

    # the chemical-potential model runs on the same recipe with the balls kept apart (its stencils
    # reach two nodes into the solid; nearly touching balls end it in a domain error)
    gap = W.CP_MIN_GAP if args.model == "chempot" and args.workload in ("c1", "c2") else 0.0
    wl = W.make(args.workload, min_gap=gap)
    steps = args.steps if args.steps is not None else wl.steps
    rho_ref = (W.PR_MAXWELL[0.80][0] if args.model == "chempot" else wl.rho_v) if args.precision != "f64" else 0.0
    log(f"[bench] workload {wl.name} dims {wl.dims[:wl.dim]} precision {args.precision}: set-up")
    grav = tuple(float(v) for v in args.gravity.split(",")) + (0.0, 0.0, 0.0)
    grav = grav[:3]
    lat, (nl, nb, nw) = setup_gpu(wl, args.precision, rho_ref, args.bc_mode, args.collision, args.model, grav)
    M0 = lat.mass().M
    log(f"[bench] links {nl} boundary nodes {nb} wall nodes {nw}; warmup {args.warmup}")
    lat.step(args.warmup)
    torch.cuda.synchronize()
    log(f"[bench] timed: {steps} steps")
    lat.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.step(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms, launches = lat.timing_report()
    lat.timing(False)
    rep = lat.mass()
    drift = (rep.M - M0) / M0
    # the monitors of the step (mass / momentum / eq. 18 total; the largest speed), host-synchronous
    # calls timed by the wall clock, result copy included
    monitor = {}
    for name, call in (("mass", lat.mass), ("max_speed", lat.max_speed)):
        call()
        t1 = time.perf_counter()
        for _ in range(20):
            call()
        monitor[name + "_ms_per_call"] = (time.perf_counter() - t1) / 20 * 1e3

    from paper_2203_04508_amd.traffic import kernel_digest

    alg = algorithmic_bytes(wl, args.precision, nl)
    impl = layout_bytes(wl, args.precision, nb)
    # one kernel launch per step; HIP events on the library's stream bracket each launch
    fused_ms = ms / max(1, launches)
    achieved = alg / (fused_ms * 1e-3) / 1e9
    # measured HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated on a plain copy), used only
    # when they were taken on the kernel as it is now
    traffic = None
    from paper_2203_04508_amd.traffic import out_name
    tfile = os.path.join(ROOT, "profiles", out_name(wl.name, args.precision, args.model, args.collision) + ".json")
    measured_cfg = args.bc_mode == "present" and not any(grav)
    if os.path.exists(tfile) and measured_cfg:  # the counters were taken on this configuration only
        tj = json.load(open(tfile))
        if tj.get("kernel_digest") == kernel_digest(wl.dim):
            # the bytes of one whole step, like `achieved` (the 3-D step is two launches)
            traffic = tj.get("bytes_per_step", tj.get("bytes_per_launch"))

    out = {
        "metric": METRIC,
        "value": wl.N * steps / el / 1e6,
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": el * 1e3 / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES[args.precision],
        "data": "synthetic",
        "config": {
            "workload": (f"{wl.name}: D2Q9 {wl.dims[0]}x{wl.dims[1]}" if wl.dim == 2 else f"{wl.name}: D3Q19 {wl.dims[0]}^3")
                        + (f", balls at least {gap:g} apart" if gap > 0 else ""),
            "storage": args.precision,
            "bc_mode": args.bc_mode,
            "collision": args.collision,
            "model": args.model,
            "rho_ref": rho_ref,
            "links": nl, "boundary_nodes": nb, "wall_nodes": nw,
            "T_over_Tc": 0.8 if args.model == "chempot" else wl.T_over_Tc, "tau": wl.tau,
            "gravity": list(grav[:wl.dim]),
        },
        "roofline": {
            "bound": "hbm",
            "kernel": ("k_cp_march (one step)" if args.model == "chempot"
                       else "k_step2d" if wl.dim == 2 else "k_rho3d + k_step3d (one step)"),
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "algorithmic_bytes_per_step": alg,
            "algorithmic_bytes_basis": f"N (2 Q s + 1) + 20 |L|: N {wl.N}, Q {wl.Q}, s {STORAGE_BYTES[args.precision]}, |L| {nl}",
            "layout_bytes_per_step": impl,
            "layout_frac": impl / (fused_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "kernel_ms": fused_ms,
            "kernel_launches": launches,
        },
        "mass_drift": drift,
        "mass_drift_steps": args.warmup + steps,
        "monitor": monitor,
    }
    if not args.no_adjoint:
        log("[bench] forward + reverse mode (c3)")
        out["fwd_adjoint"] = fwd_adjoint(args.precision)
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_budget, bc_mode=args.bc_mode, collision=args.collision, model=args.model,
                                           gravity=grav[:wl.dim])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
