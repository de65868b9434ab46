"""Write c3_oracle_duals.json: the oracle's forward-mode (dual-number) derivatives of the c3 loss.

    python tests/golden/make_c3_duals.py [--jobs 5]

c3 is the 512^2 rough wall (a slab with 60 half-circles, one drop, per-wall-node wettability drawn
from its seed), 2000 steps at its temperature and relaxation time.  The loss is the vapour-side
mass below rho = rho_v (loss kind 0, parameters (rho_v, 1)), the one whose gradient the reverse mode
takes on this workload.  Twenty tangent directions in the space of the wall nodes' wettability
factors are drawn with numpy's PCG64 from the seed stored in the file (standard normal, in the
order of the oracle's wall-node list); the oracle carries four at a time, so the twenty come from
five dual runs.  Only the oracle computes anything here; the file holds its loss value, the
twenty directional derivatives, and a hash of the wall-node list that the GPU test checks first.
"""
import argparse
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_oracle_duals.json")
SEED = 2203
NDIR = 20


def setup():
    from oracle import oracle
    from paper_2203_04508_amd import workloads as W

    wl = W.make("c3")
    P = oracle.make_params(2, *wl.dims, tau=wl.tau, T=wl.T)
    solid = oracle.classify(P, wl.shapes)
    node, d, cls, q = oracle.links(P, wl.shapes, solid)
    walls = oracle.wall_nodes(P, solid)
    return oracle, W, wl, P, solid, node, d, q, walls


def directions(n_wall):
    return np.random.Generator(np.random.PCG64(SEED)).standard_normal((NDIR, n_wall))


def run(block):
    oracle, W, wl, P, solid, node, d, q, walls = setup()
    kd = oracle.dual_kd()
    dirs = directions(len(walls))[block * kd:(block + 1) * kd]
    ds = oracle.DualSim(P, solid, node, d, q)
    ds.set_phi(W.phi_for_walls(wl, walls), dirs)
    ds.init_eq(wl.rho0())
    ds.step(wl.steps)
    L, dL = ds.loss(0, (wl.rho_v, 1.0))
    ds.close()
    return L, dL[:len(dirs)].tolist()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=5)
    args = ap.parse_args()
    oracle, W, wl, P, solid, node, d, q, walls = setup()
    kd = oracle.dual_kd()
    assert NDIR % kd == 0
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=args.jobs) as ex:
        res = list(ex.map(run, range(NDIR // kd)))
    losses = {r[0] for r in res}
    assert len(losses) == 1, losses  # the primal part does not depend on the tangents
    out = {
        "workload": "c3", "dims": list(wl.dims[:2]), "steps": wl.steps, "tau": wl.tau, "T": wl.T,
        "loss_kind": 0, "loss_prm": [wl.rho_v, 1.0], "direction_seed": SEED, "n_directions": NDIR,
        "n_wall": int(len(walls)), "wall_sha256": hashlib.sha256(np.ascontiguousarray(walls, np.int64).tobytes()).hexdigest(),
        "loss": res[0][0], "derivatives": [v for r in res for v in r[1]],
        "command": "python tests/golden/make_c3_duals.py", "seconds": round(time.perf_counter() - t0, 1),
    }
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps({k: out[k] for k in ("loss", "n_wall", "seconds")}))


if __name__ == "__main__":
    main()
