"""Precision study of the step on one workload: the same initial state run with FP64 storage (the
GPU baseline) and with shifted FP32 and FP16 storage, reporting per storage format the step time,
throughput and HBM rate (of the method's bytes, and of the layout's), the relative mass drift, and the density error against the
FP64 run, L2(rho - rho_FP64) / L2(rho_FP64) over the lattice (solid nodes hold 0 in both).

    python -m paper_2203_04508_amd.study --workload c2 --steps 5000 [--out profiles/precision_c2.json]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from paper_2203_04508_amd.roofline import HBM_PEAK_GBS, algorithmic_bytes, layout_bytes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
def run_one(wl, precision, steps, rho0):
    import torch
    from paper_2203_04508_amd import mcb, workloads as W

    rr = wl.rho_v if precision != "f64" else 0.0
    lat = mcb.Lattice(wl.dim, wl.dims, wl.tau, wl.T, precision=precision, rho_ref=rr)
    nl, nb, _ = lat.set_geometry(wl.shapes)
    lat.set_wettability(W.phi_for_walls(wl, lat.wall_nodes()))
    lat.init_equilibrium(rho0)
    M0 = lat.mass().M
    torch.cuda.synchronize()
    lat.timing(True)
    t0 = time.perf_counter()
    lat.step(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms, launches = lat.timing_report()
    lat.timing(False)
    rep = lat.mass()
    rho, _ = lat.moments()
    lat.close()
    step_ms = ms / max(1, launches)
    alg = algorithmic_bytes(wl, precision, nl)
    lay = layout_bytes(wl, precision, nb)
    return {
        "precision": precision,
        "steps": steps,
        "step_ms": step_ms,
        "mlups": wl.N / (step_ms * 1e-3) / 1e6,
        "wall_mlups": wl.N * steps / el / 1e6,
        "algorithmic_gbs": alg / (step_ms * 1e-3) / 1e9,
        "hbm_frac": alg / (step_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "layout_frac": lay / (step_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "mass_drift": (rep.M - M0) / M0,
    }, rho


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    sys.path.insert(0, ROOT)
    from paper_2203_04508_amd import workloads as W

    wl = W.make(args.workload)
    steps = args.steps if args.steps is not None else wl.steps
    rho0 = wl.rho0()
    rows, ref = [], None
    for prec in ("f64", "f32s", "f16s"):
        print(f"[study] {wl.name} {prec}: {steps} steps", file=sys.stderr, flush=True)
        r, rho = run_one(wl, prec, steps, rho0)
        if ref is None:
            ref = rho
        r["rho_l2_rel_vs_f64"] = float(np.linalg.norm(rho - ref) / np.linalg.norm(ref))
        rows.append(r)
    out = {"command": "python3 -m paper_2203_04508_amd.study " + " ".join(sys.argv[1:]),
           "workload": wl.name, "dims": list(wl.dims[:wl.dim]), "steps": steps, "runs": rows}
    text = json.dumps(out, indent=1)
    print(text)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(text + "\n")


if __name__ == "__main__":
    main()
