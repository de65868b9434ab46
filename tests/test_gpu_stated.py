"""GPU parity at the specified temperatures and relaxation times of the 1024^2, 4096^2 and 256^3
workloads: 0.6 T_c (1024^2 and 4096^2) and 0.65 T_c (256^3), tau 0.8, width-2 drop profiles, the
full geometry, drops and wettability of each workload.  The FP64 oracle runs the same 20 steps.

Bars: link lists bit-exact (every entry, the 4096^2 list included); FP64 populations within
1e-12 relative per step (1e-12 k after k steps), shifted FP32 within 3e-6 per step (3e-6 (k + 1)
after k steps), the relative error of a direction plane being max|f_gpu - f_oracle| /
max|f_oracle| over fluid nodes; FP64 mass to 1e-13.  On the 4096^2 and 256^3 lattices these
settings leave the domain of the pseudopotential within the twenty steps, in the oracle itself: the
GPU's FP64 path must then report MCB_EDOMAIN in the same step as the oracle, and agree with it
before.  How long each setting runs is measured by the stability study.
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


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("name", ["c1", "c2", "c4"])
def test_stated_parameters_parity(mcb, name):
    wl = W.make(name, stated=True)
    banner(f"{name} at T = {wl.T_over_Tc} T_c, tau {wl.tau}, width {wl.interface_width}: oracle set-up")
    P = oracle.make_params(wl.dim, *wl.dims, tau=wl.tau, T=wl.T)
    solid = oracle.classify(P, wl.shapes)
    node, d, cls, q = oracle.links(P, wl.shapes, solid)
    walls = oracle.wall_nodes(P, solid)
    phi = W.phi_for_walls(wl, walls)
    rho0 = wl.rho0()
    fluid = solid == 0
    sim = oracle.Sim(P, solid, node, d, q)
    sim.set_phi(phi)
    sim.init_eq(rho0)
    M0 = sim.mass()
    banner(f"{name}: GPU lattices (FP64, shifted FP32), geometry")
    lat64 = mcb.Lattice(wl.dim, wl.dims, wl.tau, wl.T, precision="f64")
    lat32 = mcb.Lattice(wl.dim, wl.dims, wl.tau, wl.T, precision="f32s", rho_ref=wl.rho_v)
    for lat in (lat64, lat32):
        nl, nb, nw = lat.set_geometry(wl.shapes)
        assert (nl, nw) == (len(node), len(walls))
        lat.set_wettability(phi)
        lat.init_equilibrium(rho0)
    got = lat64.links()
    assert np.array_equal(got["node"], node) and np.array_equal(got["dir"], d)
    assert np.array_equal(got["q_fixed"], q) and np.array_equal(got["cls"], cls)
    assert np.array_equal(lat64.wall_nodes(), walls)
    del got
    assert rel_err(lat64.get_f(), sim.get_f(), fluid) < 1e-13
    # one step at a time: the oracle and the FP64 GPU path must leave the domain of psi (the
    # large-density-ratio instability of these settings) in the same step, and agree before it
    fail_o = fail_g = None
    for k in range(1, 21):
        try:
            sim.step(1)
        except oracle.OracleError:
            fail_o = k
        lat64.step(1)
        lat32.step(1)
        try:
            lat64.sync()
        except mcb.MCBError as e:
            assert e.code == mcb.MCB_EDOMAIN, e
            fail_g = k
        if fail_o is not None or fail_g is not None:
            break
        if k in (1, 20):
            fo = sim.get_f()
            e64 = rel_err(lat64.get_f(), fo, fluid)
            e32 = rel_err(lat32.get_f(), fo, fluid)
            print(f"  after {k} steps: FP64 {e64:.2e}, FP32 {e32:.2e}", flush=True)
            assert e64 < 1e-12 * k, (k, e64)
            assert e32 < 3e-6 * (k + 1), (k, e32)
            del fo
    print(f"  psi domain error: oracle at step {fail_o}, GPU FP64 at step {fail_g}", flush=True)
    assert fail_o == fail_g, (fail_o, fail_g)
    if fail_o is None:
        assert abs(lat64.mass().M - M0) <= 1e-13 * M0
        assert abs(sim.mass() - M0) <= 1e-13 * M0
    lat64.close()
    lat32.close()
    sim.close()
