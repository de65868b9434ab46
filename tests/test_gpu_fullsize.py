"""GPU parity at the benchmark sizes, in the launch configuration bench.py times: the 4096^2 D2Q9
workload (c2: 4800 off-lattice circles, 640 drops, per-circle wettability) and the 256^3 D3Q19
geometry (c4: 400 spheres; a uniform wettability and eight of its drops stand in for the per-sphere
factors and the 200 drops, whose Python set-up would dominate the test), against the FP64 oracle on
every node.

Bars: FP64 1e-12 relative after one step; shifted FP32 (the benchmarked storage) 3e-6 (2-D) and
2e-6 (3-D) per step, relative error per direction plane as in the other parity tests. The
chemical-potential model with MRT runs on c2's recipe with the circles kept 4 apart (as the
benchmark runs it), FP32 within 2e-5 per step.
"""
import sys

import numpy as np
import pytest

from oracle import oracle
from paper_2203_04508_amd import workloads as W

pytestmark = pytest.mark.gpu


def banner(msg):
    print(f"\n[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mcb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_04508_amd import mcb as m
    m.load()
    return m


def rel_err(a, b, fluid):
    worst = 0.0
    for i in range(a.shape[0]):
        d = np.abs(a[i, fluid] - b[i, fluid]).max()
        s = np.abs(b[i, fluid]).max()
        worst = max(worst, d / s)
    return worst


def _case(name):
    wl = W.make(name)
    P = oracle.make_params(wl.dim, *wl.dims, tau=wl.tau, T=wl.T)
    solid = oracle.classify(P, wl.shapes)
    node, d, cls, q = oracle.links(P, wl.shapes, solid)
    walls = oracle.wall_nodes(P, solid)
    if name == "c2":
        phi = W.phi_for_walls(wl, walls)
        rho0 = wl.rho0()
    else:
        phi = np.full(len(walls), 1.02)
        rho0 = W.drop_field(wl.dims, 3, wl.drops[:8], wl.rho_v, wl.rho_l, wl.interface_width)
    return wl, P, solid, (node, d, q), phi, rho0


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name,tol32", [("c2", 3e-6), ("c4", 2e-6)])
def test_benchmark_size_parity(mcb, name, tol32):
    banner(f"full-size parity {name}: oracle set-up")
    wl, P, solid, (node, d, q), phi, rho0 = _case(name)
    fluid = solid == 0
    sim = oracle.Sim(P, solid, node, d, q)
    sim.set_phi(phi)
    sim.init_eq(rho0)
    f_init = sim.get_f()
    sim.step(1)
    f_one = sim.get_f()
    banner(f"full-size parity {name}: FP64, 1 step")
    lat = mcb.Lattice(wl.dim, wl.dims, wl.tau, wl.T, precision="f64")
    assert lat.set_geometry(wl.shapes)[0] == len(node)
    lat.set_wettability(phi)
    lat.init_equilibrium(rho0)
    assert rel_err(lat.get_f(), f_init, fluid) < 1e-13
    lat.step(1)
    e = rel_err(lat.get_f(), f_one, fluid)
    assert e < 1e-12, e
    lat.close()
    banner(f"full-size parity {name}: shifted FP32, 2 steps")
    lat = mcb.Lattice(wl.dim, wl.dims, wl.tau, wl.T, precision="f32s", rho_ref=wl.rho_v)
    lat.set_geometry(wl.shapes)
    lat.set_wettability(phi)
    lat.init_equilibrium(rho0)
    lat.step(1)
    e1 = rel_err(lat.get_f(), f_one, fluid)
    assert e1 < 2 * tol32, e1
    sim.step(1)
    lat.step(1)
    e2 = rel_err(lat.get_f(), sim.get_f(), fluid)
    assert e2 < 3 * tol32, e2
    lat.close()
    sim.close()


@pytest.mark.timeout(900)
def test_benchmark_size_parity_chempot(mcb):
    """The chemical-potential model with MRT at the benchmark size (c2's recipe with the circles at
    least 4 apart, as bench.py runs it): FP64 1e-12 after one step, shifted FP32 2e-5 per step."""
    banner("full-size parity c2 chemical potential + MRT: oracle set-up")
    wl = W.make("c2", min_gap=W.CP_MIN_GAP)
    T = 0.8 * W.PR_TC
    P = oracle.make_params(2, *wl.dims, tau=wl.tau, T=0.05)
    solid = oracle.classify(P, wl.shapes)
    node, d, cls, q = oracle.links(P, wl.shapes, solid)
    rho0, mu_s, rv = W.chempot_inputs(wl, oracle.wall_nodes(P, solid))
    fluid = solid == 0
    sim = oracle.Sim(P, solid, node, d, q)
    sim.set_chempot(T, k=W.CP_K, kappa=W.CP_KAPPA)
    sim.set_mrt()
    sim.set_mu_wall(mu_s)
    sim.init_eq(rho0)
    f_init = sim.get_f()
    sim.step(1)
    f_one = sim.get_f()
    opts = dict(model="chempot", cp_k=W.CP_K, cp_kappa=W.CP_KAPPA, collision="mrt")
    banner("full-size parity c2 chemical potential + MRT: FP64, 1 step")
    lat = mcb.Lattice(2, wl.dims, wl.tau, T, precision="f64", **opts)
    assert lat.set_geometry(wl.shapes)[0] == len(node)
    lat.set_wettability(mu_s)
    lat.init_equilibrium(rho0)
    assert rel_err(lat.get_f(), f_init, fluid) < 1e-13
    lat.step(1)
    e = rel_err(lat.get_f(), f_one, fluid)
    assert e < 1e-12, e
    lat.close()
    banner("full-size parity c2 chemical potential + MRT: shifted FP32, 2 steps")
    lat = mcb.Lattice(2, wl.dims, wl.tau, T, precision="f32s", rho_ref=rv, **opts)
    lat.set_geometry(wl.shapes)
    lat.set_wettability(mu_s)
    lat.init_equilibrium(rho0)
    lat.step(1)
    e1 = rel_err(lat.get_f(), f_one, fluid)
    assert e1 < 2 * 2e-5, e1
    sim.step(1)
    lat.step(1)
    e2 = rel_err(lat.get_f(), sim.get_f(), fluid)
    assert e2 < 3 * 2e-5, e2
    lat.close()
    sim.close()
