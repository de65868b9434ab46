"""Reverse mode (the differentiation growth) on the GPU, through the C ABI, against references
that share nothing with it:
  * the oracle's forward-mode dual numbers (exact directional derivatives of the same discrete
    map, obtained without any transposition): FP64 adjoint within 1e-8 relative;
  * central finite differences of the GPU forward map on the 512^2 rough-wall workload (2000
    steps, a checkpoint every 100): 1e-4 relative on 20 seeded wall nodes;
  * dM/dphi = 0: eq. 18 conserves the mass for any wettability.
"""
import sys

import numpy as np
import pytest

from oracle import oracle
from paper_2203_04508_amd import workloads as W

pytestmark = pytest.mark.gpu

TC = W.CS_TC
RV, RL = W.MAXWELL[0.7]


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


def small_case():
    dims = (32, 24, 1)
    shapes = np.array([W.band_y(-0.5, 3.4, 0), W.ball((10.3, 3.4), 3.1, 0), W.ball((21.7, 3.4), 2.6, 0)], np.int64)
    rho0 = W.drop_field(dims, 2, [((16.0, 11.0), 6.0)], RV, RL, 2.0)
    return dims, shapes, rho0


LOSSES = [(0, (RV, 1.0)), (1, ((RV + RL) / 2, 0.1 * (RL - RV))), (2, (0.0, 1.0))]


@pytest.mark.parametrize("nsteps,k", [(0, 1), (1, 1), (20, 7), (60, 16)])
@pytest.mark.parametrize("kind", [0, 1, 2])
def test_adjoint_matches_dual_numbers(mcb, nsteps, k, kind):
    banner(f"adjoint vs oracle duals, 32x24, {nsteps} steps, k={k}, loss {kind}")
    dims, shapes, rho0 = small_case()
    prm = LOSSES[kind][1]
    P = oracle.make_params(2, *dims, tau=0.8, T=0.7 * TC)
    solid = oracle.classify(P, shapes)
    node, d, cls, q = oracle.links(P, shapes, solid)
    walls = oracle.wall_nodes(P, solid)
    rng = np.random.default_rng(100 + nsteps + kind)
    phi = rng.uniform(0.9, 1.1, len(walls))
    dirs = rng.standard_normal((4, len(walls)))
    dirs[0] = 0.0
    dirs[0][len(walls) // 2] = 1.0
    ds = oracle.DualSim(P, solid, node, d, q)
    ds.set_phi(phi, dirs)
    ds.init_eq(rho0)
    ds.step(nsteps)
    L_o, dL_o = ds.loss(kind, prm)

    lat = mcb.Lattice(2, dims, 0.8, 0.7 * TC)
    lat.set_geometry(shapes)
    lat.set_wettability(phi)
    L_g = lat.adj_forward(rho0, nsteps, k, kind, prm)
    assert abs(L_g - L_o) <= 1e-12 * max(1.0, abs(L_o)), (L_g, L_o)
    grad = lat.adj_backward(1.0)
    dL_g = dirs @ grad
    scale = max(np.abs(dL_o).max(), 1e-300)
    if kind == 2:
        # total mass: the derivative vanishes; both sides stay at rounding level
        assert np.abs(dL_g).max() < 1e-11 and np.abs(dL_o).max() < 1e-11, (dL_g, dL_o)
    else:
        # (after 0 steps the density, hence every loss, does not depend on phi: both sides vanish)
        assert np.abs(dL_g - dL_o).max() <= 1e-8 * scale + 1e-14, (dL_g, dL_o)
    lat.close()


def test_state_is_restored_after_backward(mcb):
    banner("forward + backward leave the state as a plain run's")
    dims, shapes, rho0 = small_case()
    out = []
    for use_adj in (True, False):
        lat = mcb.Lattice(2, dims, 0.8, 0.7 * TC)
        lat.set_geometry(shapes)
        lat.set_wettability(1.03)
        if use_adj:
            lat.adj_forward(rho0, 25, 6, 0, (RV, 1.0))
            lat.adj_backward(1.0)
        else:
            lat.init_equilibrium(rho0)
            lat.step(25)
        lat.step(7)
        out.append(lat.get_f())
        lat.close()
    assert np.array_equal(out[0], out[1])
