"""Pins of the oracle's body force (gravity, used by the drop-impact runs of Sec. 4.5 of arXiv
2203.04508): the total momentum grows by exactly M g per step in a periodic box (the nonideal force
sums to zero), and gravity-driven flow between two curved walls converges to the parabola with the
walls at their true positions, which the interpolated schemes recover and halfway bounce-back does
not."""
import numpy as np
import pytest

from oracle import oracle
from paper_2203_04508_amd import workloads as W

TC = W.CS_TC


def test_momentum_grows_by_mass_times_g():
    dims = (40, 36, 1)
    P = oracle.make_params(2, *dims, tau=0.9, T=0.7 * TC)
    N = 40 * 36
    e0 = np.zeros(0, np.int64)
    sim = oracle.Sim(P, np.zeros(N, np.uint8), e0, e0.astype(np.int32), e0.astype(np.uint32))
    g = (2e-5, -3e-5)
    sim.set_gravity(g)
    rv, rl = W.MAXWELL[0.70]
    sim.init_eq(W.drop_field(dims, 2, [((17.3, 19.6), 9.0)], rv, rl, 2.0))
    e, *_ = oracle.lattice(2)
    ed = e[:, :2].astype(float)
    ft = sim.get_f()
    M, J0 = ft.sum(), (ft.T @ ed).sum(0)
    n = 300
    sim.step(n)
    J1 = (sim.get_f().T @ ed).sum(0)
    assert np.abs((J1 - J0) - n * M * np.array(g)).max() < 1e-12 * n * M * 3e-5


@pytest.mark.parametrize("tau", [0.8, 1.0])
def test_gravity_driven_channel_between_curved_walls(tau):
    """Walls at y = 1.3 (links q = 0.7) and y = 22.2 (q = 0.2), uniform liquid density (so the
    nonideal force vanishes), g along x: the steady profile is u = g/(2 nu) (y - 1.3)(22.2 - y),
    nu = (tau - 1/2)/3. The present scheme and MIBC hit it within 1% of the peak; halfway
    bounce-back, which puts the walls at 1.5 and 22.5, misses by more than 3%."""
    nx, ny, ylo, yhi, g = 4, 32, 1.3, 22.2, 1e-6
    shapes = np.array([W.band_y(yhi, ny + ylo, 0)], np.int64)
    P = oracle.make_params(2, nx, ny, 1, tau=tau, T=0.7 * TC)
    solid = oracle.classify(P, shapes)
    node, d, cls, q = oracle.links(P, shapes, solid)
    rows = np.nonzero(solid.reshape(ny, nx)[:, 0] == 0)[0]
    assert rows.min() == 2 and rows.max() == 22
    y = np.arange(ny)
    want = g / (2 * (tau - 0.5) / 3) * (y - ylo) * (yhi - y)
    err = {}
    for mode in (oracle.BC_PRESENT, oracle.BC_MIBC, oracle.BC_HBBC):
        sim = oracle.Sim(P, solid, node, d, q)
        sim.set_bc_mode(mode)
        sim.set_phi(1.0)
        sim.set_gravity((g, 0.0))
        sim.init_eq(np.full(nx * ny, W.MAXWELL[0.70][1]))
        sim.step(12000)
        _, v, _ = sim.moments()
        ux = v[0].reshape(ny, nx)
        assert np.abs(ux - ux[:, :1]).max() < 1e-15  # uniform along the channel
        err[mode] = np.abs(ux[rows, 0] - want[rows]).max() / want[rows].max()
        sim.close()
    assert err[oracle.BC_PRESENT] < 1e-2 and err[oracle.BC_MIBC] < 1e-2
    assert err[oracle.BC_HBBC] > 3e-2
