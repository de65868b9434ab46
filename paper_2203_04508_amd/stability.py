"""Long-run stability of the workloads at their specified temperatures and relaxation times.

    python -m paper_2203_04508_amd.stability [--workloads c1,c2,c4] [--collisions bgk,mrt]
                                             [--precisions f64,f32s] [--out profiles/stability_stated]

Each run starts from the workload's equilibrium state at the stated parameters (0.6 T_c and tau 0.8
on 1024^2 and 4096^2, 0.65 T_c and tau 0.8 on 256^3, width-2 drops; --tau and --widths vary the
relaxation time and the drop profile) and steps for the workload's full count, synchronising every
100 steps.  A run that ends in a psi domain error (a density past
the real branch of the pseudopotential: the large-density-ratio instability) or a non-finite
population is recorded with the window in which it failed.  The multiple-relaxation-time collision
(eqs. 1-3 with the paper's rates) is tried as the stable route on the two-dimensional lattices; it
has no three-dimensional basis in the paper.  Results go to <out>.json and <out>.txt with the
command that made them.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_one(mcb, W, name, collision, precision, steps=None, check=100, stated=True, width=None, tau=None):
    import torch

    wl = W.make(name, stated=stated)
    if width is not None:
        wl.interface_width = width
    if tau is not None:
        wl.tau = tau
    n = steps if steps is not None else wl.steps
    lat = mcb.Lattice(wl.dim, wl.dims, wl.tau, wl.T, precision=precision,
                      rho_ref=wl.rho_v if precision != "f64" else 0.0, collision=collision)
    nl, nb, nw = lat.set_geometry(wl.shapes)
    lat.set_wettability(W.phi_for_walls(wl, lat.wall_nodes()))
    lat.init_equilibrium(wl.rho0())
    M0 = lat.mass().M
    out = {"workload": name, "dims": list(wl.dims[:wl.dim]), "T_over_Tc": wl.T_over_Tc, "tau": wl.tau,
           "width": wl.interface_width, "collision": collision, "precision": precision, "steps": n,
           "links": nl, "boundary_nodes": nb}
    t0 = time.perf_counter()
    done = 0
    status = "stable"
    while done < n:
        k = min(check if done >= 100 else 10, n - done)  # finer windows over the start-up transient
        lat.step(k)
        try:
            lat.sync()
        except mcb.MCBError as e:
            status = {mcb.MCB_EDOMAIN: "psi domain error", mcb.MCB_ENAN: "non-finite population"}.get(e.code, str(e))
            out["failed_between"] = [done, done + k]
            break
        done += k
    torch.cuda.synchronize()
    out["status"] = status
    out["steps_done"] = done
    out["seconds"] = time.perf_counter() - t0
    if status == "stable":
        rep = lat.mass()
        out["mass_drift"] = (rep.M - M0) / M0
        vmax, _ = lat.max_speed()
        out["max_speed"] = vmax
        rho, _ = lat.moments()
        r = rho[rho > 0]
        out["rho_min"], out["rho_max"] = float(r.min()), float(r.max())
        out["density_ratio"] = float(r.max() / r.min())
    lat.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workloads", default="c1,c2,c4")
    ap.add_argument("--collisions", default="bgk,mrt")
    ap.add_argument("--precisions", default="f64,f32s")
    ap.add_argument("--steps", type=int, default=None, help="override the workloads' step counts")
    ap.add_argument("--widths", default="2", help="drop profile widths to run (the stated one is 2)")
    ap.add_argument("--tau", type=float, default=None, help="relaxation time instead of the stated 0.8")
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles", "stability_stated"))
    args = ap.parse_args()
    sys.path.insert(0, ROOT)
    import torch
    from paper_2203_04508_amd import mcb, workloads as W

    assert torch.cuda.is_available(), "the stability study runs on the GPU"
    mcb.load()
    rows = []
    for name in args.workloads.split(","):
        for coll in args.collisions.split(","):
            if coll == "mrt" and W.make(name).dim == 3:
                continue
            for prec, width in [(p, float(w)) for w in args.widths.split(",") for p in args.precisions.split(",")]:
                print(f"[stability] {name} {coll} {prec} width {width:g}", flush=True)
                r = run_one(mcb, W, name, coll, prec, steps=args.steps, width=width, tau=args.tau)
                print(f"[stability]   {r['status']} after {r['steps_done']} steps "
                      f"({r['seconds']:.1f} s)", flush=True)
                rows.append(r)
    cmd = "python -m paper_2203_04508_amd.stability " + " ".join(sys.argv[1:])
    json.dump({"command": cmd, "runs": rows}, open(args.out + ".json", "w"), indent=1)
    with open(args.out + ".txt", "w") as fh:
        fh.write("Stability at the specified temperatures and relaxation times, checked every 10 steps up to step 100 "
                 "and every 100 steps after\n")
        fh.write(f"command: {cmd}\n\n")
        fh.write(f"{'workload':9} {'T/Tc':>5} {'tau':>4} {'width':>5} {'coll':>4} {'storage':>7} {'steps':>6}  result\n")
        for r in rows:
            res = (f"stable, mass drift {r['mass_drift']:+.2e}, max |v| {r['max_speed']:.2e}, "
                   f"density {r['rho_min']:.4g}..{r['rho_max']:.4g} (ratio {r['density_ratio']:.0f})"
                   if r["status"] == "stable" else f"{r['status']} between steps {r['failed_between'][0]} and "
                   f"{r['failed_between'][1]}")
            fh.write(f"{r['workload']:9} {r['T_over_Tc']:5.2f} {r['tau']:4.1f} {r['width']:5.1f} {r['collision']:>4} "
                     f"{r['precision']:>7} {r['steps']:6d}  {res}\n")
    print(open(args.out + ".txt").read(), flush=True)


if __name__ == "__main__":
    main()
