"""Sessile drop on a flat wetting substrate, swept over the wall distance q, for the present boundary
scheme and the three the paper compares it with (IBC, MIBC, halfway bounce-back); the setting of
Secs. 4.1, 4.3 and 4.4 (Figs. 3, 7 and 9) with this library's pseudopotential model.

Geometry: a periodic 500 x 300 box (FP64 storage); the substrate is the band of solid rows below
y_w = y1 - q, with y1 = 11 the first fluid row, so every link from row y1 into the wall has the same
q (axis and diagonal links alike).  The band's underside, at the top of the periodic box, sits at
q = 1/2, where all four schemes coincide.  A drop of radius 50 is centred on the wall line.

Two multiphase models: "pseudo" (this library's pseudopotential, BGK, tau = 1, Carnahan-Starling at
0.7 T_c, wettability the factor phi of the eq. 15 wall density) and "chempot" (the paper's own:
chemical-potential model with the Peng-Robinson EOS at 0.8 T_c, MRT collision with the rates of
eq. 3 and tau = 0.8, wettability the assigned wall chemical potential mu_s of Sec. 2.3).

Wettability (phi or mu_s) is calibrated at q = 1/2 (where the schemes agree) to the two contact
angles of the paper, 60 and 120 degrees, by bisection on the equilibrium angle.  The angle comes from a circle fitted to the drop's interface (rho = (rho_l + rho_v) / 2,
interpolated along rows, rows at least 4 above the wall), cos(theta) = (y_w - y_c) / R.

Reported per angle, scheme and q: M/M0 - 1 and the eq. 18 total Delta M of the step at sample times;
the final contact angle; the largest speed over the fluid at the end (the spurious currents of
Sec. 4.4); the step at which a run stopped on a psi domain error, if it did.

    python -m paper_2203_04508_amd.qsweep [--model pseudo|chempot] [--steps 20000] [--out profiles/qsweep_flat.json]
    python -m paper_2203_04508_amd.qsweep --summarize profiles/qsweep_flat.json   (text table)

With --geometry curved, the setting of Sec. 4.2 (Figs. 5-6): a 500 x 600 box, a cylinder of radius
100 (off-lattice centre, so q varies along the wall) and a drop of radius 70 centred on its top;
the wettability is the flat substrate's calibration, each scheme runs --steps steps.  With
--geometry curved-angles, the spurious currents of Sec. 4.4 (Fig. 10) on that geometry: contact
angles 50 to 170 degrees (--angles), the present scheme against MIBC, the largest speed at the end.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NX, NY, Y1, R0 = 500, 300, 11, 50.0
# per model: reduced temperature, tau, collision, interface width of the initial profile, and the
# wettability search interval (the angle falls with phi, rises with mu_s)
MODELS = {
    "pseudo": dict(T_over_Tc=0.70, tau=1.0, collision="bgk", width=2.0, lo=0.50, hi=1.45, rising=False),
    "chempot": dict(T_over_Tc=0.80, tau=0.8, collision="mrt", width=6.0, lo=-0.06, hi=0.06, rising=True),
}
MODEL = "pseudo"


def _densities():
    from paper_2203_04508_amd import workloads as W

    m = MODELS[MODEL]
    return W.PR_MAXWELL[m["T_over_Tc"]] if MODEL == "chempot" else W.MAXWELL[m["T_over_Tc"]]


def setup(q):
    from paper_2203_04508_amd import workloads as W

    yw = Y1 - q
    shapes = np.array([W.band_y(-0.5, yw, 0)], np.int64)
    rv, rl = _densities()
    rho0 = W.drop_field((NX, NY, 1), 2, [((NX / 2.0, yw), R0)], rv, rl, MODELS[MODEL]["width"])
    # the half of the drop below the wall line would wrap to the top of the periodic box, against
    # the band's underside: vapour there
    rho0.reshape(NY, NX)[NY // 2:] = rv
    return shapes, rho0, yw, rv, rl


def interface_points(rho, yw, rv, rl):
    """(x, y) where rho crosses (rho_l + rho_v) / 2 along rows at least 4 above the wall."""
    rm = 0.5 * (rv + rl)
    g = rho.reshape(NY, NX)
    pts = []
    for y in range(int(math.ceil(yw + 4.0)), NY):
        row = g[y]
        liq = row > rm
        if not liq.any():
            continue
        d = np.nonzero(np.diff(liq.astype(np.int8)))[0]  # crossings between x and x + 1
        for x in d:
            a, b = row[x], row[x + 1]
            pts.append((x + (rm - a) / (b - a), float(y)))
    return np.array(pts)


def contact_angle(rho, yw, rv, rl):
    """Degrees, from an algebraic (Kasa) circle fit to the interface; nan without a drop."""
    p = interface_points(rho, yw, rv, rl)
    if len(p) < 8:
        return float("nan")
    x, y = p[:, 0], p[:, 1]
    A = np.stack([x, y, np.ones_like(x)], 1)
    c, *_ = np.linalg.lstsq(A, x * x + y * y, rcond=None)
    xc, yc = c[0] / 2.0, c[1] / 2.0
    R = math.sqrt(c[2] + xc * xc + yc * yc)
    cth = (yw - yc) / R
    return math.degrees(math.acos(max(-1.0, min(1.0, cth))))


def make_lattice(mode, q, phi):
    from paper_2203_04508_amd import mcb, workloads as W

    shapes, rho0, yw, rv, rl = setup(q)
    m = MODELS[MODEL]
    if MODEL == "chempot":
        # the wettability argument is mu_s relative to the bulk potential at coexistence
        phi = W.CP_K * W.CP_K * W.MU_PR_COEX[m["T_over_Tc"]] + phi
        lat = mcb.Lattice(2, (NX, NY, 1), m["tau"], m["T_over_Tc"] * W.PR_TC, precision="f64", bc_mode=mode,
                          collision=m["collision"], model="chempot", cp_k=W.CP_K, cp_kappa=W.CP_KAPPA)
    else:
        lat = mcb.Lattice(2, (NX, NY, 1), m["tau"], m["T_over_Tc"] * W.CS_TC, precision="f64", bc_mode=mode,
                          collision=m["collision"])
    try:
        lat.set_geometry(shapes)
        lat.set_wettability(phi)
        lat.init_equilibrium(rho0)
    except mcb.MCBError:
        lat.close()
        raise
    return lat, yw, rv, rl


def equilibrium_angle(phi, steps):
    """Contact angle after steps steps of the present scheme at q = 1/2; nan if the run stops on a
    psi domain error (phi too large for the equation of state)."""
    from paper_2203_04508_amd import mcb

    lat = None
    try:
        lat, yw, rv, rl = make_lattice("present", 0.5, phi)
        lat.step(steps)
        rho, _ = lat.moments()
        return contact_angle(rho, yw, rv, rl)
    except mcb.MCBError:
        return float("nan")
    finally:
        if lat is not None:
            lat.close()


def calibrate(target, steps, iters=10):
    """The wettability value in the model's interval with the equilibrium angle at target degrees
    (pseudo: phi, the angle falls as it rises, a domain error counts as too wetting; chempot: mu_s
    minus the bulk coexistence potential, the angle rises with it)."""
    m = MODELS[MODEL]
    lo, hi = m["lo"], m["hi"]
    log = []
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        th = equilibrium_angle(mid, steps)
        log.append((mid, th))
        print(f"[qsweep] calibrate {target}: wettability {mid:.5f} -> {th:.2f} deg", file=sys.stderr, flush=True)
        too_wetting = not np.isfinite(th) or th < target
        if too_wetting != m["rising"]:
            hi = mid
        else:
            lo = mid
    return 0.5 * (lo + hi), log


def run(mode, q, phi, steps, every):
    from paper_2203_04508_amd import mcb

    lat, yw, rv, rl = make_lattice(mode, q, phi)
    M0 = lat.mass().M
    ts, m, dm = [0], [0.0], [0.0]
    failed = None
    t = n = 0
    try:
        while t < steps:
            n = min(every, steps - t)
            lat.step(n)
            t += n
            rep = lat.mass()
            ts.append(t)
            m.append((rep.M - M0) / M0)
            dm.append(rep.dM_last)
    except mcb.MCBError as e:
        failed = {"step_before": t + n, "error": str(e)}
    out = {"mode": mode, "q": q, "t": ts, "drift": m, "dM_last": dm, "failed": failed}
    if failed is None:
        rho, _ = lat.moments()
        out["theta_end"] = contact_angle(rho, yw, rv, rl)
        out["max_speed_end"] = lat.max_speed()[0]
    lat.close()
    return out


CNX, CNY, RCYL, RDROP = 500, 600, 100.0, 70.0
CYL = (250.3, 200.7)


def curved_lattice(mode, w):
    """The Sec. 4.2 geometry with wettability w (as in make_lattice), initial state set."""
    from paper_2203_04508_amd import mcb, workloads as W

    m = MODELS[MODEL]
    rv, rl = _densities()
    shapes = np.array([W.ball(CYL, RCYL, 0)], np.int64)
    rho0 = W.drop_field((CNX, CNY, 1), 2, [((CYL[0], CYL[1] + RCYL), RDROP)], rv, rl, m["width"])
    if MODEL == "chempot":
        w = W.CP_K * W.CP_K * W.MU_PR_COEX[m["T_over_Tc"]] + w
        lat = mcb.Lattice(2, (CNX, CNY, 1), m["tau"], m["T_over_Tc"] * W.PR_TC, precision="f64", bc_mode=mode,
                          collision=m["collision"], model="chempot", cp_k=W.CP_K, cp_kappa=W.CP_KAPPA)
    else:
        lat = mcb.Lattice(2, (CNX, CNY, 1), m["tau"], m["T_over_Tc"] * W.CS_TC, precision="f64", bc_mode=mode,
                          collision=m["collision"])
    try:
        lat.set_geometry(shapes)
        lat.set_wettability(w)
        lat.init_equilibrium(rho0)
    except mcb.MCBError:
        lat.close()
        raise
    return lat, rv, rl


def run_curved(mode, w, steps, every):
    from paper_2203_04508_amd import mcb

    lat, rv, rl = curved_lattice(mode, w)
    M0 = lat.mass().M
    ts, m, dm = [0], [0.0], [0.0]
    failed = None
    t = n = 0
    try:
        while t < steps:
            n = min(every, steps - t)
            lat.step(n)
            t += n
            rep = lat.mass()
            ts.append(t)
            m.append((rep.M - M0) / M0)
            dm.append(rep.dM_last)
    except mcb.MCBError as e:
        failed = {"step_before": t + n, "error": str(e)}
    out = {"mode": mode, "t": ts, "drift": m, "dM_last": dm, "failed": failed}
    if failed is None:
        rho, _ = lat.moments()
        out["liquid_nodes_end"] = int((rho > 0.5 * (rv + rl)).sum())
        out["max_speed_end"] = lat.max_speed()[0]
    lat.close()
    return out


def summarize_curved(res) -> str:
    lines = [f"curved-substrate runs, model {res['model']}, {res['box'][0]}x{res['box'][1]} D2Q9 FP64, cylinder r "
             f"{res['cylinder_radius']}, drop r {res['drop_radius']}, {res['steps']} steps, T/Tc {res['T_over_Tc']}, "
             f"tau {res['tau']}", f"command: {res['command']}"]
    for a in res["angles"]:
        lines.append("")
        lines.append(f"target {a['target_deg']:.0f} deg (flat calibration, wettability {a['phi']:.5f})")
        lines.append("  scheme   M/M0-1 at steps " + " ".join(f"{t:>9d}" for t in a["runs"][0]["t"][1::max(1, len(a['runs'][0]['t']) // 5)]) +
                     "   liquid nodes   max|v|    max|dM| last quarter")
        for r in a["runs"]:
            idx = list(range(1, len(r["t"]), max(1, len(a['runs'][0]['t']) // 5)))
            vals = " ".join(f"{r['drift'][k]:+9.2e}" if k < len(r["drift"]) else f"{'-':>9s}" for k in idx)
            k0 = 3 * len(r["dM_last"]) // 4
            tail = (f"   {r['liquid_nodes_end']:10d}   {r['max_speed_end']:.2e}" if r["failed"] is None
                    else f"   stopped before step {r['failed']['step_before']}")
            lines.append(f"  {r['mode']:7s}  {vals}{tail}   {max(abs(v) for v in r['dM_last'][k0:]):.2e}")
    return "\n".join(lines) + "\n"


def summarize_angles(res) -> str:
    lines = [f"spurious currents on the curved substrate, model {res['model']}, {res['box'][0]}x{res['box'][1]}, "
             f"cylinder r {res['cylinder_radius']}, drop r {res['drop_radius']}, {res['steps']} steps",
             f"command: {res['command']}", "",
             "  target  flat-calibrated  | max|v| present   max|v| MIBC   ratio | M/M0-1 present   MIBC"]
    for r in res["rows"]:
        p, m = r["present"], r["mibc"]
        vp, vm = p["max_speed_end"], m["max_speed_end"]
        ratio = f"{vm / vp:6.1f}" if vp and vm else "     -"
        fmt = lambda v: f"{v:.2e}" if v is not None else "stopped "
        lines.append(f"  {r['target_deg']:6.0f}  {r['theta_flat']:15.1f}  |   {fmt(vp)}        {fmt(vm)}   {ratio} |"
                     f" {p['drift']:+.1e}       {m['drift']:+.1e}")
    return "\n".join(lines) + "\n"


def _round(x, sig=6):
    if isinstance(x, float):
        return float(f"{x:.{sig}g}")
    if isinstance(x, list):
        return [_round(v, sig) for v in x]
    if isinstance(x, dict):
        return {k: _round(v, sig) for k, v in x.items()}
    return x


def summarize(res) -> str:
    """Per angle: for each q, M/M0 at the end (or the step a run stopped before), the final contact
    angle and the final largest speed, per scheme; and the largest |Delta M| sampled after the
    first quarter of the run for MIBC and the present scheme."""
    lines = [f"flat-substrate q-sweep, model {res.get('model', 'pseudo')}, {res['box'][0]}x{res['box'][1]} D2Q9 FP64, "
             f"drop r {res['drop_radius']}, {res['steps']} steps, T/Tc {res['T_over_Tc']}, tau {res['tau']}",
             f"command: {res['command']}"]
    for a in res["angles"]:
        th05 = a["theta_present_q05"]
        lines.append("")
        lines.append(f"target {a['target_deg']:.0f} deg: wettability {a['phi']:.5f}, equilibrium angle at q = 1/2 {th05:.1f} deg")
        runs = {(r["mode"], r["q"]): r for r in a["runs"]}
        hb = next(r for r in a["runs"] if r["mode"] == "hbbc")
        lines.append(f"halfway bounce-back (q-independent): M/M0-1 {hb['drift'][-1]:+.1e}, theta {hb['theta_end']:.1f}, "
                     f"max|v| {hb['max_speed_end']:.2e}")
        lines.append("  q   | present: M/M0-1   theta  max|v|  | IBC: M/M0 (theta)        | MIBC: M/M0-1  theta  max|v|  "
                     "| max|dM| late: MIBC   present")
        for q in sorted({r["q"] for r in a["runs"] if r["mode"] == "present"}):
            p, i, m = runs[("present", q)], runs[("ibc", q)], runs[("mibc", q)]
            k0 = len(p["t"]) // 4

            def late(r):
                return max(abs(v) for v in r["dM_last"][k0:]) if len(r["dM_last"]) > k0 else float("nan")

            ibc = (f"{1 + i['drift'][-1]:.3f} ({i['theta_end']:.0f})" if i["failed"] is None
                   else f"stop < {i['failed']['step_before']} ({1 + i['drift'][-1]:.3f})")
            lines.append(f"  {q:.1f} | {p['drift'][-1]:+.1e}  {p['theta_end']:6.1f}  {p['max_speed_end']:.2e} | "
                         f"{ibc:24s} | {m['drift'][-1]:+.1e}  {m['theta_end']:6.1f}  {m['max_speed_end']:.2e} | "
                         f"{late(m):.2e}  {late(p):.2e}")
    return "\n".join(lines) + "\n"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--summarize", default=None, help="print the text table of a stored result")
    ap.add_argument("--model", default="pseudo", choices=list(MODELS))
    ap.add_argument("--geometry", default="flat", choices=["flat", "curved", "curved-angles"])
    ap.add_argument("--angles", default="50,70,90,110,130,150,170")
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--every", type=int, default=1000)
    ap.add_argument("--calib-steps", type=int, default=10000)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    if args.summarize:
        res = json.load(open(args.summarize))
        g = res.get("geometry")
        print((summarize_curved(res) if g == "curved" else summarize_angles(res) if g == "curved-angles"
               else summarize(res)), end="")
        return
    sys.path.insert(0, ROOT)
    global MODEL
    MODEL = args.model
    t0 = time.time()
    if args.geometry == "curved-angles":
        res = {"command": "python3 -m paper_2203_04508_amd.qsweep " + " ".join(sys.argv[1:]), "geometry": "curved-angles",
               "model": MODEL, "box": [CNX, CNY], "cylinder_radius": RCYL, "drop_radius": RDROP,
               "T_over_Tc": MODELS[MODEL]["T_over_Tc"], "tau": MODELS[MODEL]["tau"], "steps": args.steps, "rows": []}
        for target in [float(a) for a in args.angles.split(",")]:
            w, log = calibrate(target, args.calib_steps)
            th = equilibrium_angle(w, args.calib_steps)
            row = {"target_deg": target, "phi": w, "theta_flat": th}
            for mode in ("present", "mibc"):
                r = run_curved(mode, w, args.steps, args.steps)
                row[mode] = {"drift": r["drift"][-1], "max_speed_end": r.get("max_speed_end"),
                             "failed": r["failed"]}
            print(f"[qsweep] curved angle {target:.0f} (flat {th:.1f}): present {row['present']['max_speed_end']}, "
                  f"mibc {row['mibc']['max_speed_end']}", file=sys.stderr, flush=True)
            res["rows"].append(row)
        res["wall_seconds"] = time.time() - t0
        res = _round(res)
        if args.out:
            with open(args.out, "w") as fh:
                fh.write(json.dumps(res, separators=(",", ":")) + "\n")
        print(summarize_angles(res), end="")
        return
    if args.geometry == "curved":
        res = {"command": "python3 -m paper_2203_04508_amd.qsweep " + " ".join(sys.argv[1:]), "geometry": "curved",
               "model": MODEL, "box": [CNX, CNY], "cylinder_radius": RCYL, "cylinder_centre": list(CYL),
               "drop_radius": RDROP, "T_over_Tc": MODELS[MODEL]["T_over_Tc"], "tau": MODELS[MODEL]["tau"],
               "collision": MODELS[MODEL]["collision"], "precision": "f64", "steps": args.steps, "angles": []}
        for target in (60.0, 120.0):
            w, log = calibrate(target, args.calib_steps)
            ang = {"target_deg": target, "phi": w, "runs": []}
            for mode in ("present", "ibc", "mibc", "hbbc"):
                r = run_curved(mode, w, args.steps, args.every)
                ang["runs"].append(r)
                f = r["failed"]
                print(f"[qsweep] curved {target:.0f} deg {mode:7s}: M/M0-1 {r['drift'][-1]:+.3e}"
                      + (f" stopped: {f['error']}" if f else f", liquid nodes {r['liquid_nodes_end']}, max|v| {r['max_speed_end']:.2e}"),
                      file=sys.stderr, flush=True)
            res["angles"].append(ang)
        res["wall_seconds"] = time.time() - t0
        res = _round(res)
        if args.out:
            with open(args.out, "w") as fh:
                fh.write(json.dumps(res, separators=(",", ":")) + "\n")
        print(summarize_curved(res), end="")
        return
    qs = [round(0.1 * k, 1) for k in range(10)]
    res = {"command": "python3 -m paper_2203_04508_amd.qsweep " + " ".join(sys.argv[1:]),
           "model": MODEL, "box": [NX, NY], "first_fluid_row": Y1, "drop_radius": R0,
           "T_over_Tc": MODELS[MODEL]["T_over_Tc"], "tau": MODELS[MODEL]["tau"], "collision": MODELS[MODEL]["collision"],
           "precision": "f64", "steps": args.steps, "angles": []}
    for target in (60.0, 120.0):
        phi, log = calibrate(target, args.calib_steps)
        ang = {"target_deg": target, "phi": phi, "calibration": [[p, th] for p, th in log],
               "theta_present_q05": equilibrium_angle(phi, args.calib_steps), "runs": []}
        for mode in ("present", "ibc", "mibc", "hbbc"):
            for q in (qs if mode != "hbbc" else [0.3]):  # halfway bounce-back does not see q
                r = run(mode, q, phi, args.steps, args.every)
                ang["runs"].append(r)
                f = r["failed"]
                print(f"[qsweep] {target:.0f} deg {mode:7s} q={q:.1f}: M/M0-1 {r['drift'][-1]:+.3e}"
                      + (f" stopped: {f['error']}" if f else f", theta {r['theta_end']:.1f}, max|v| {r['max_speed_end']:.2e}"),
                      file=sys.stderr, flush=True)
        res["angles"].append(ang)
    res["wall_seconds"] = time.time() - t0
    res = _round(res)
    text = json.dumps(res, separators=(",", ":"))
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(text + "\n")
    print(json.dumps({"angles": [{"target": a["target_deg"], "phi": a["phi"],
                                  "final_drift": {f"{r['mode']}@{r['q']}": r["drift"][-1] for r in a["runs"]}}
                                 for a in res["angles"]]}, indent=1))


if __name__ == "__main__":
    main()
