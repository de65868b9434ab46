"""Measured HBM traffic of the fused step kernel, calibrated against a plain copy.

Two phases:

``python -m paper_2203_04508_amd.traffic run --workload c2 --precision f32s --steps 5``
    sets up the workload, runs a few steps, then copies a 1 GiB torch tensor (a plain device copy
    of known size: 1 GiB read, 1 GiB written).  Run it under rocprofv3 once with
    ``--pmc FETCH_SIZE`` and once with ``--pmc WRITE_SIZE``.  ``--model chempot --collision mrt``
    takes the chemical-potential step of the same geometry instead (Peng-Robinson at 0.8 T_c, the
    balls four nodes apart, as the benchmark runs it).

``python -m paper_2203_04508_amd.traffic summarize --fetch-db A.db --write-db B.db --workload c2 --precision f32s``
    reads both databases, scales each counter of the step kernel by (known copy bytes / what the
    same counter reads for the copy kernel), and writes ``profiles/traffic_<workload>_<precision>.json``
    and a short text summary next to it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sqlite3
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_BYTES = 1 << 30
CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")


def kernel_digest(dim: int) -> str:
    """Hash of the sources the step kernel of a dimension is built from: counters taken on another
    version of the kernel do not describe this one."""
    h = hashlib.sha256()
    for f in ("step2d.hip" if dim == 2 else "step3d.hip", "kernels_common.h", "mcb_internal.h"):
        h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()[:16]


def out_name(workload, precision, model="pseudo", collision="bgk"):
    """profiles/ base name of a measured configuration (the pseudopotential one with BGK keeps the
    short name)."""
    tail = "" if model == "pseudo" and collision == "bgk" else f"_{model}_{collision}"
    return f"traffic_{workload}_{precision}{tail}"


def run(args):
    import torch

    sys.path.insert(0, ROOT)
    from paper_2203_04508_amd import mcb, workloads as W

    if args.model == "chempot":
        wl = W.make(args.workload, min_gap=W.CP_MIN_GAP)
        rr = W.PR_MAXWELL[0.80][0] if args.precision != "f64" else 0.0
        lat = mcb.Lattice(wl.dim, wl.dims, wl.tau, 0.8 * W.PR_TC, precision=args.precision, rho_ref=rr,
                          collision=args.collision, model="chempot", cp_k=W.CP_K, cp_kappa=W.CP_KAPPA)
        lat.set_geometry(wl.shapes)
        rho0, mu_s, _ = W.chempot_inputs(wl, lat.wall_nodes())
        lat.set_wettability(mu_s)
        lat.init_equilibrium(rho0)
    else:
        wl = W.make(args.workload)
        rr = wl.rho_v if args.precision != "f64" else 0.0
        lat = mcb.Lattice(wl.dim, wl.dims, wl.tau, wl.T, precision=args.precision, rho_ref=rr,
                          collision=args.collision)
        lat.set_geometry(wl.shapes)
        lat.set_wettability(W.phi_for_walls(wl, lat.wall_nodes()))
        lat.init_equilibrium(wl.rho0())
    lat.step(args.steps)
    torch.cuda.synchronize()
    x = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    print(f"[traffic] {args.workload} {args.precision}: {args.steps} steps and one {COPY_BYTES} B copy done", flush=True)


def _counter(db, counter):
    con = sqlite3.connect(db)
    rows = con.execute(
        "select kernel_name, dispatch_id, sum(value) from counters_collection where counter_name = ? "
        "group by kernel_name, dispatch_id", (counter,)).fetchall()
    con.close()
    return rows


def _per_dispatch(rows, match):
    vals = [v for k, d, v in rows if match(k)]
    return sum(vals) / len(vals) if vals else None, len(vals)


def _largest(rows, match):
    vals = [v for k, d, v in rows if match(k)]
    return max(vals) if vals else None, len(vals)


def _pull_kernel(name):
    """The per-step kernels of the pulling step (not the collision that starts a run), by name:
    k_step2d<S, C, W, OUT, PULL>, k_step3d<S, C, PULL, PF>, k_rho3d<S, C, PULL>,
    k_cp_march<S, C, W, OUT, PULL>."""
    for k, idx in (("k_step2d<", 4), ("k_step3d<", 2), ("k_rho3d<", 2), ("k_cp_march<", 4)):
        if k in name:
            args = name.split(k, 1)[1].split(">", 1)[0].split(",")
            return len(args) > idx and args[idx].strip() == "true"
    return False


def _short(name):
    for k in ("k_step2d", "k_step3d", "k_rho3d", "k_cp_march"):
        if k in name:
            return k
    return name


def summarize(args):
    sys.path.insert(0, ROOT)
    from paper_2203_04508_amd import workloads as W

    out = {"workload": args.workload, "precision": args.precision, "model": args.model,
           "collision": args.collision, "copy_bytes": COPY_BYTES,
           "kernel_digest": kernel_digest(W.make(args.workload).dim), "kernels": {}}
    lines = []
    # the device copy of COPY_BYTES is the largest copy dispatch of the run
    is_copy = lambda k: "copybuffer" in k.lower()
    for counter, db, key in (("FETCH_SIZE", args.fetch_db, "read"), ("WRITE_SIZE", args.write_db, "write")):
        rows = _counter(db, counter)
        copy_kib, _ = _largest(rows, is_copy)
        factor = COPY_BYTES / (copy_kib * 1024.0)
        out[f"{key}_copy_counter_kib"] = copy_kib
        out[f"{key}_scale"] = factor
        names = sorted({k for k, d, v in rows if _pull_kernel(k)})
        for name in names:
            kib, n = _per_dispatch(rows, lambda k, name=name: k == name)
            kk = out["kernels"].setdefault(_short(name), {"name": name})
            kk[f"{key}_counter_kib_per_dispatch"] = kib
            kk[f"{key}_bytes_per_launch"] = kib * 1024.0 * factor
            lines.append(f"{counter}: {_short(name)} {kib:.0f} KiB/dispatch over {n} dispatches; "
                         f"calibrated {kk[f'{key}_bytes_per_launch'] / 1e6:.1f} MB per launch")
        lines.append(f"{counter}: the {COPY_BYTES} B copy reads {copy_kib:.0f} KiB on this counter -> scale {factor:.4f}")
    step = 0.0
    for kk in out["kernels"].values():
        kk["bytes_per_launch"] = kk.get("read_bytes_per_launch", 0.0) + kk.get("write_bytes_per_launch", 0.0)
        step += kk["bytes_per_launch"]
    # the step kernel proper (the collision pass in three dimensions) is the one bench.py reports
    main = out["kernels"].get("k_step2d") or out["kernels"].get("k_step3d") or out["kernels"].get("k_cp_march")
    out["bytes_per_launch"] = main["bytes_per_launch"] if main else None
    out["bytes_per_step"] = step
    out_dir = args.out_dir or os.path.join(ROOT, "profiles")
    os.makedirs(out_dir, exist_ok=True)
    base = os.path.join(out_dir, out_name(args.workload, args.precision, args.model, args.collision))
    json.dump(out, open(base + ".json", "w"), indent=1)
    with open(base + ".txt", "w") as fh:
        fh.write(f"HBM traffic of the step kernels, workload {args.workload}, storage {args.precision}, "
                 f"{args.model} model, {args.collision} (kernel sources {out['kernel_digest']})\n")
        fh.write(f"commands: {args.commands}\n" if args.commands else "")
        fh.write("\n".join(lines) + "\n")
        for k, kk in out["kernels"].items():
            fh.write(f"{k}: {kk['bytes_per_launch'] / 1e6:.1f} MB per launch (read + write)\n")
        fh.write(f"total calibrated bytes per step: {step / 1e6:.1f} MB\n")
    print(open(base + ".txt").read())


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("run")
    r.add_argument("--workload", default="c2")
    r.add_argument("--precision", default="f32s")
    r.add_argument("--steps", type=int, default=5)
    s = sub.add_parser("summarize")
    s.add_argument("--fetch-db", required=True)
    s.add_argument("--write-db", required=True)
    s.add_argument("--workload", default="c2")
    s.add_argument("--precision", default="f32s")
    s.add_argument("--commands", default="")
    s.add_argument("--out-dir", default="", help="where the summary goes (default: profiles/)")
    for q in (r, s):
        q.add_argument("--model", default="pseudo", choices=("pseudo", "chempot"))
        q.add_argument("--collision", default="bgk", choices=("bgk", "mrt"))
    a = ap.parse_args()
    run(a) if a.cmd == "run" else summarize(a)


if __name__ == "__main__":
    main()
