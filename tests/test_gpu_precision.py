"""Shifted reduced-precision storage (g_i = f_i - w_i rho_ref in FP32 or FP16, FP32 arithmetic)
against the FP64 oracle, and the mass-drift targets.

Bounds derived from the arithmetic:
  * FP32 storage rounds each population to 2^-24 relative, and the FP32 collision adds about ten
    rounded operations: one step stays within 2e-6 of the FP64 result in the plane-wise max norm,
    and the error at most adds up linearly over a few tens of steps.
  * FP16 storage rounds to 2^-11 relative: 2e-3 per step.
  * Mass: the collision hands the pulled density back exactly (f_0 takes the rounding), so the
    FP64 lattice drifts at rounding level (<= 1e-12 relative per 10^4 steps) and the FP32 one at
    <= 1e-6 per 10^4 steps (the targets).
"""
import sys

import numpy as np
import pytest

from oracle import oracle
from paper_2203_04508_amd import workloads as W

pytestmark = pytest.mark.gpu

TC = W.CS_TC


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
    return max(np.abs(a[i, fluid] - b[i, fluid]).max() / np.abs(b[i, fluid]).max() for i in range(a.shape[0]))


@pytest.mark.parametrize("prec,tol", [("f32s", 2e-6), ("f16s", 2e-3)])
def test_shifted_storage_against_fp64_oracle(mcb, prec, tol):
    banner(f"{prec} vs FP64 oracle, 37x29 random geometry")
    dims = (37, 29, 1)
    rng = np.random.default_rng(21)
    shapes = W.random_links_case(rng, dims, 2, 3, 2.0, 6.0)
    rv, rl = W.MAXWELL[0.7]
    rho0 = W.drop_field(dims, 2, [((18.0, 14.0), 7.0)], rv, rl, 2.0)
    T = 0.7 * TC
    P = oracle.make_params(2, *dims, tau=0.8, T=T)
    sim, (solid, *_r) = oracle.sim_from_shapes(P, shapes)
    sim.set_phi(1.05)
    lat = mcb.Lattice(2, dims, 0.8, T, precision=prec, rho_ref=rv)
    lat.set_geometry(shapes)
    lat.set_wettability(1.05)
    sim.init_eq(rho0)
    lat.init_equilibrium(rho0)
    fluid = solid == 0
    assert rel_err(lat.get_f(), sim.get_f(), fluid) < tol
    for k in range(1, 11):
        sim.step(1)
        lat.step(1)
        e = rel_err(lat.get_f(), sim.get_f(), fluid)
        assert e < tol * (k + 1), (k, e)


def _drift(mcb, name, prec, steps):
    wl = W.make(name)
    rr = wl.rho_v if prec != "f64" else 0.0
    lat = mcb.Lattice(2, wl.dims, wl.tau, wl.T, precision=prec, rho_ref=rr)
    lat.set_geometry(wl.shapes)
    lat.set_wettability(W.phi_for_walls(wl, lat.wall_nodes()))
    lat.init_equilibrium(wl.rho0())
    M0 = lat.mass().M
    lat.step(steps)
    rep = lat.mass()
    lat.close()
    return (rep.M - M0) / M0


def test_fp64_mass_drift_c1_10k_steps(mcb):
    banner("FP64 mass drift, 1024^2, 10^4 steps")
    d = _drift(mcb, "c1", "f64", 10000)
    assert abs(d) <= 1e-12, d


def test_fp32_mass_drift_c1_10k_steps(mcb):
    banner("shifted FP32 mass drift, 1024^2, 10^4 steps")
    d = _drift(mcb, "c1", "f32s", 10000)
    assert abs(d) <= 1e-6, d


def test_fp16_mass_drift_c1_10k_steps(mcb):
    # FP16 storage keeps the rest population in FP32, which takes the rounding of the collision's
    # mass balance, so the FP32 bound holds as well
    banner("shifted FP16 mass drift, 1024^2, 10^4 steps")
    d = _drift(mcb, "c1", "f16s", 10000)
    assert abs(d) <= 1e-6, d
