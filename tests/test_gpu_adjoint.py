"""Reverse mode (the differentiation growth) on the GPU, through the C ABI, against references
that share nothing with it:
  * the oracle's forward-mode dual numbers (exact directional derivatives of the same discrete
    map, obtained without any transposition): FP64 adjoint within 1e-8 relative;
  * central finite differences of the GPU forward map on the 512^2 rough-wall workload (2000
    steps, a checkpoint every 100): 1e-4 relative on 20 seeded wall nodes;
  * on that workload itself, the oracle's dual numbers along twenty seeded directions over the
    full run (stored by tests/golden/make_c3_duals.py): 1e-8 relative;
  * dM/dphi = 0: eq. 18 conserves the mass for any wettability.
"""
import hashlib
import json
import os
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


@pytest.mark.parametrize("nsteps,k,grav", [(1, 1, (0.0, 0.0, 0.0)), (12, 5, (0.0, 0.0, 0.0)), (12, 5, (1e-5, -3e-5, 2e-5))],
                         ids=["1-step", "12-steps", "12-steps-gravity"])
@pytest.mark.parametrize("kind", [0, 1])
def test_adjoint_3d_matches_dual_numbers(mcb, nsteps, k, grav, kind):
    """D3Q19: slab + sphere, one drop; the gradient against the oracle's dual numbers (1e-8)."""
    banner(f"adjoint vs oracle duals, D3Q19 16x14x12, {nsteps} steps, k={k}, gravity {grav}, loss {kind}")
    dims = (16, 14, 12)
    shapes = np.array([W.band_y(-0.5, 2.6, 0), W.ball((8.3, 2.6, 5.7), 2.9, 0)], np.int64)
    rho0 = W.drop_field(dims, 3, [((8.0, 7.5, 6.0), 4.0)], RV, RL, 2.0)
    prm = LOSSES[kind][1]
    P = oracle.make_params(3, *dims, tau=0.8, T=0.7 * TC)
    solid = oracle.classify(P, shapes)
    node, d, cls, q = oracle.links(P, shapes, solid)
    walls = oracle.wall_nodes(P, solid)
    rng = np.random.default_rng(300 + nsteps + kind)
    phi = rng.uniform(0.9, 1.1, len(walls))
    dirs = rng.standard_normal((4, len(walls)))
    ds = oracle.DualSim(P, solid, node, d, q)
    ds.set_phi(phi, dirs)
    ds.set_gravity(grav)
    ds.init_eq(rho0)
    ds.step(nsteps)
    L_o, dL_o = ds.loss(kind, prm)
    lat = mcb.Lattice(3, dims, 0.8, 0.7 * TC, gravity=grav)
    lat.set_geometry(shapes)
    lat.set_wettability(phi)
    L_g = lat.adj_forward(rho0, nsteps, k, kind, prm)
    assert abs(L_g - L_o) <= 1e-12 * max(1.0, abs(L_o)), (L_g, L_o)
    dL_g = dirs @ lat.adj_backward(1.0)
    scale = max(np.abs(dL_o).max(), 1e-300)
    assert np.abs(dL_o).max() > 0.0
    assert np.abs(dL_g - dL_o).max() <= 1e-8 * scale + 1e-14, (dL_g, dL_o)
    lat.close()


@pytest.mark.parametrize("mode", ["ibc", "mibc", "hbbc"])
def test_adjoint_3d_schemes_match_dual_numbers(mcb, mode):
    """D3Q19 with the comparison schemes (IBC: no eq. 18): the gradient against the oracle's dual
    numbers run with the same scheme (1e-8)."""
    banner(f"adjoint vs oracle duals, D3Q19 16x14x12, {mode}, 12 steps")
    dims = (16, 14, 12)
    shapes = np.array([W.band_y(-0.5, 2.6, 0), W.ball((8.3, 2.6, 5.7), 2.9, 0)], np.int64)
    rho0 = W.drop_field(dims, 3, [((8.0, 7.5, 6.0), 4.0)], RV, RL, 2.0)
    prm = LOSSES[0][1]
    P = oracle.make_params(3, *dims, tau=0.8, T=0.7 * TC)
    solid = oracle.classify(P, shapes)
    node, d, cls, q = oracle.links(P, shapes, solid)
    walls = oracle.wall_nodes(P, solid)
    rng = np.random.default_rng(400 + len(mode))
    phi = rng.uniform(0.9, 1.1, len(walls))
    dirs = rng.standard_normal((4, len(walls)))
    ds = oracle.DualSim(P, solid, node, d, q)
    ds.set_bc_mode({"ibc": 1, "mibc": 2, "hbbc": 3}[mode])
    ds.set_phi(phi, dirs)
    ds.init_eq(rho0)
    ds.step(12)
    L_o, dL_o = ds.loss(0, prm)
    lat = mcb.Lattice(3, dims, 0.8, 0.7 * TC, bc_mode=mode)
    lat.set_geometry(shapes)
    lat.set_wettability(phi)
    L_g = lat.adj_forward(rho0, 12, 5, 0, prm)
    assert abs(L_g - L_o) <= 1e-12 * max(1.0, abs(L_o)), (L_g, L_o)
    dL_g = dirs @ lat.adj_backward(1.0)
    scale = max(np.abs(dL_o).max(), 1e-300)
    assert np.abs(dL_o).max() > 0.0
    assert np.abs(dL_g - dL_o).max() <= 1e-8 * scale + 1e-14, (dL_g, dL_o)
    lat.close()


CONFIGS = [("mrt", dict(collision="mrt"), {}), ("gravity", dict(gravity=(2e-5, -4e-5)), {}),
           ("mibc", dict(bc_mode="mibc"), {}), ("ibc", dict(bc_mode="ibc"), {}), ("hbbc", dict(bc_mode="hbbc"), {}),
           ("mrt-gravity-mibc", dict(collision="mrt", gravity=(0.0, -3e-5), bc_mode="mibc"), {})]


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("name,opts,_", CONFIGS, ids=[c[0] for c in CONFIGS])
def test_adjoint_other_collisions_forces_and_schemes(mcb, name, opts, _, kind):
    """Reverse mode with the MRT collision, a body force and the comparison boundary schemes against
    the oracle's dual numbers run with the same settings (20 steps, checkpoint every 7)."""
    banner(f"adjoint vs oracle duals, {name}, loss {kind}")
    dims, shapes, rho0 = small_case()
    prm = LOSSES[kind][1]
    P = oracle.make_params(2, *dims, tau=0.8, T=0.7 * TC)
    solid = oracle.classify(P, shapes)
    node, d, cls, q = oracle.links(P, shapes, solid)
    walls = oracle.wall_nodes(P, solid)
    rng = np.random.default_rng(300 + kind + len(name))
    phi = rng.uniform(0.9, 1.1, len(walls))
    dirs = rng.standard_normal((4, len(walls)))
    ds = oracle.DualSim(P, solid, node, d, q)
    ds.set_phi(phi, dirs)
    if opts.get("collision") == "mrt":
        ds.set_mrt()
    if "gravity" in opts:
        ds.set_gravity(opts["gravity"])
    ds.set_bc_mode({"present": 0, "ibc": 1, "mibc": 2, "hbbc": 3}[opts.get("bc_mode", "present")])
    ds.init_eq(rho0)
    ds.step(20)
    L_o, dL_o = ds.loss(kind, prm)
    lat = mcb.Lattice(2, dims, 0.8, 0.7 * TC, **opts)
    lat.set_geometry(shapes)
    lat.set_wettability(phi)
    L_g = lat.adj_forward(rho0, 20, 7, kind, prm)
    assert abs(L_g - L_o) <= 1e-12 * max(1.0, abs(L_o)), (L_g, L_o)
    dL_g = dirs @ lat.adj_backward(1.0)
    scale = max(np.abs(dL_o).max(), 1e-300)
    assert np.abs(dL_g - dL_o).max() <= 1e-8 * scale + 1e-14, (dL_g, dL_o)
    lat.close()


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("name,opts", [("chempot", {}), ("chempot-mrt-gravity", dict(collision="mrt", gravity=(0.0, -2e-5)))],
                         ids=["chempot", "chempot-mrt-gravity"])
def test_adjoint_chempot_wall_potential(mcb, name, opts, kind):
    """The chemical-potential model: the gradient with respect to every wall node's assigned chemical
    potential against the oracle's dual numbers (20 steps, checkpoint every 7)."""
    from oracle import thermo

    banner(f"adjoint vs oracle duals, {name}, loss {kind}")
    _, Tc = thermo.critical_point_pr()
    T = 0.8 * Tc
    rv, rl = W.PR_MAXWELL[0.80]
    dims, shapes, _ = small_case()
    rho0 = W.drop_field(dims, 2, [((16.0, 11.0), 6.0)], rv, rl, 6.0)
    prm = (rv, 1.0) if kind == 0 else ((rv + rl) / 2, 0.1 * (rl - rv))
    P = oracle.make_params(2, *dims, tau=0.8, T=0.05)
    solid = oracle.classify(P, shapes)
    node, d, cls, q = oracle.links(P, shapes, solid)
    walls = oracle.wall_nodes(P, solid)
    rng = np.random.default_rng(400 + kind)
    mu_s = W.CP_K ** 2 * W.MU_PR_COEX[0.80] + rng.uniform(-0.01, 0.01, len(walls))
    dirs = rng.standard_normal((4, len(walls)))
    ds = oracle.DualSim(P, solid, node, d, q)
    ds.set_chempot(T, k=W.CP_K, kappa=W.CP_KAPPA)
    ds.set_phi(np.ones(len(walls)))
    ds.set_mu_wall(mu_s, dirs)
    if opts.get("collision") == "mrt":
        ds.set_mrt()
    if "gravity" in opts:
        ds.set_gravity(opts["gravity"])
    ds.init_eq(rho0)
    ds.step(20)
    L_o, dL_o = ds.loss(kind, prm)
    lat = mcb.Lattice(2, dims, 0.8, T, model="chempot", cp_k=W.CP_K, cp_kappa=W.CP_KAPPA, **opts)
    lat.set_geometry(shapes)
    lat.set_wettability(mu_s)
    L_g = lat.adj_forward(rho0, 20, 7, kind, prm)
    assert abs(L_g - L_o) <= 1e-12 * max(1.0, abs(L_o)), (L_g, L_o)
    dL_g = dirs @ lat.adj_backward(1.0)
    scale = max(np.abs(dL_o).max(), 1e-300)
    assert np.abs(dL_o).max() > 0.0
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


def test_c3_gradient_against_central_differences(mcb):
    banner("c3 (512^2 rough wall, 2000 steps, k = 100): adjoint vs central differences on 20 entries")
    wl = W.make("c3")
    lat = mcb.Lattice(2, wl.dims, wl.tau, wl.T)
    lat.set_geometry(wl.shapes)
    walls = lat.wall_nodes()
    phi = W.phi_for_walls(wl, walls)
    rho0 = wl.rho0()
    prm = (wl.rho_v, 1.0)
    lat.set_wettability(phi)
    L0 = lat.adj_forward(rho0, wl.steps, 100, 0, prm)
    g = lat.adj_backward(1.0)
    assert np.isfinite(g).all() and np.abs(g).max() > 0
    # 20 seeded entries drawn uniformly from all wall nodes (an adjoint that wrongly returned ~0 for
    # some wall nodes could be sampled); the bound is relative to the entry, floored at 1e-2 of the
    # largest entry for the many nodes whose derivative is nearly zero
    rng = np.random.default_rng(33)
    idx = rng.choice(len(walls), 20, replace=False)
    gmax = np.abs(g).max()
    worst = 0.0
    for w in idx:
        h = 1e-6 * max(1.0, abs(phi[w]))
        vals = []
        for sgn in (1.0, -1.0):
            ph = phi.copy()
            ph[w] += sgn * h
            lat.set_wettability(ph)
            vals.append(lat.adj_forward(rho0, wl.steps, 100, 0, prm))
        fd = (vals[0] - vals[1]) / (2 * h)
        r = abs(fd - g[w]) / max(abs(fd), 1e-2 * gmax)
        print(f"  wall {w}: adjoint {g[w]: .6e}  central difference {fd: .6e}  ratio {r:.2e}", flush=True)
        worst = max(worst, r)
    print(f"loss {L0:.6f}, largest |g| {gmax:.3e}, worst mixed relative difference {worst:.2e}", flush=True)
    assert worst < 1e-4, worst
    # the total mass has no derivative with respect to phi
    lat.set_wettability(phi)
    M = lat.adj_forward(rho0, wl.steps, 100, 2, (0.0, 1.0))
    gm = lat.adj_backward(1.0)
    assert np.abs(gm).max() < 1e-12 * M, np.abs(gm).max()
    lat.close()


def test_c3_gradient_against_oracle_duals(mcb):
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c3_oracle_duals.json")))
    banner(f"c3 (512^2 rough wall, {ref['steps']} steps, k = 100): adjoint vs the oracle's dual numbers along "
           f"{ref['n_directions']} directions")
    wl = W.make("c3")
    assert ref["steps"] == wl.steps and ref["loss_kind"] == 0
    lat = mcb.Lattice(2, wl.dims, wl.tau, wl.T)
    lat.set_geometry(wl.shapes)
    walls = lat.wall_nodes()
    # the directions are indexed by the wall-node list the oracle used
    assert len(walls) == ref["n_wall"]
    assert hashlib.sha256(np.ascontiguousarray(walls, np.int64).tobytes()).hexdigest() == ref["wall_sha256"]
    lat.set_wettability(W.phi_for_walls(wl, walls))
    L = lat.adj_forward(wl.rho0(), wl.steps, 100, 0, tuple(ref["loss_prm"]))
    g = lat.adj_backward(1.0)
    lat.close()
    dirs = np.random.Generator(np.random.PCG64(ref["direction_seed"])).standard_normal((ref["n_directions"], len(walls)))
    dL = dirs @ g
    want = np.asarray(ref["derivatives"])
    scale = np.abs(want).max()
    err = np.abs(dL - want).max() / scale
    print(f"  loss GPU {L:.15e} oracle {ref['loss']:.15e}; directional derivatives: worst {err:.2e} of the largest "
          f"({scale:.3e})", flush=True)
    assert abs(L - ref["loss"]) <= 1e-10 * abs(ref["loss"]), (L, ref["loss"])
    assert scale > 0 and err <= 1e-8, (dL, want)


def test_shifted_fp32_gradient_close_to_fp64(mcb):
    banner("c3 reverse mode over shifted-FP32 states vs FP64 states, 500 steps")
    wl = W.make("c3")
    grads = []
    for prec in ("f64", "f32s"):
        lat = mcb.Lattice(2, wl.dims, wl.tau, wl.T, precision=prec, rho_ref=wl.rho_v if prec != "f64" else 0.0)
        lat.set_geometry(wl.shapes)
        lat.set_wettability(W.phi_for_walls(wl, lat.wall_nodes()))
        lat.adj_forward(wl.rho0(), 500, 100, 0, (wl.rho_v, 1.0))
        grads.append(lat.adj_backward(1.0))
        lat.close()
    # FP32 storage perturbs the linearisation point by ~1e-7 relative per step
    assert np.abs(grads[1] - grads[0]).max() <= 1e-4 * np.abs(grads[0]).max()


def test_superseded_forward_pass_is_refused(mcb):
    banner("backward of a superseded forward pass or a changed state raises MCB_ESTATE")
    import torch
    dims, shapes, rho0 = small_case()
    lat = mcb.Lattice(2, dims, 0.8, 0.7 * TC)
    lat.set_geometry(shapes)
    lat.set_wettability(1.02)
    lat.adj_forward(rho0, 20, 7, 0, (RV, 1.0))
    gen1 = lat.adj_gen
    lat.set_wettability(0.97)  # the gradient of the old wettability can no longer be taken
    with pytest.raises(mcb.MCBError) as ei:
        lat.adj_backward(1.0)
    assert ei.value.code == mcb.MCB_ESTATE
    lat.adj_forward(rho0, 20, 7, 0, (RV, 1.0))
    with pytest.raises(mcb.MCBError) as ei:
        lat.adj_backward(1.0, generation=gen1)
    assert ei.value.code == mcb.MCB_ESTATE
    g2 = lat.adj_backward(1.0)
    assert np.isfinite(g2).all() and np.abs(g2).max() > 0
    lat.step(1)  # the state moved on
    with pytest.raises(mcb.MCBError) as ei:
        lat.adj_backward(1.0)
    assert ei.value.code == mcb.MCB_ESTATE
    # two losses on one lattice: only the last one can be differentiated
    p1 = torch.full((lat.n_wall,), 1.02, dtype=torch.float64, requires_grad=True)
    p2 = torch.full((lat.n_wall,), 0.99, dtype=torch.float64, requires_grad=True)
    l1 = mcb.WettabilityLoss.apply(p1, lat, rho0, 20, 7, 0, (RV, 1.0))
    l2 = mcb.WettabilityLoss.apply(p2, lat, rho0, 20, 7, 0, (RV, 1.0))
    with pytest.raises(mcb.MCBError):
        l1.backward()
    l2.backward()
    assert torch.isfinite(p2.grad).all()
    lat.close()


def test_wettability_loss_autograd(mcb):
    banner("WettabilityLoss through torch.autograd")
    import torch
    dims, shapes, rho0 = small_case()
    lat = mcb.Lattice(2, dims, 0.8, 0.7 * TC)
    lat.set_geometry(shapes)
    phi = torch.full((lat.n_wall,), 1.02, dtype=torch.float64, requires_grad=True)
    loss = mcb.WettabilityLoss.apply(phi, lat, rho0, 40, 9, 0, (RV, 1.0))
    loss.backward()
    lat.set_wettability(phi.detach().numpy())
    ref = lat.adj_forward(rho0, 40, 9, 0, (RV, 1.0))
    gref = lat.adj_backward(1.0)
    assert float(loss.detach()) == ref
    assert np.array_equal(phi.grad.numpy(), gref)
    lat.close()
