"""Pins of the oracle's forward-mode derivatives (the reference the GPU reverse mode is checked
against), by things the dual numbers do not share:
  * central finite differences of the oracle's own FP64 forward map (h = 1e-6): the directional
    derivative of the centre-of-mass and wetted-length losses along seeded directions agrees to
    1e-5 relative (the finite-difference truncation and rounding error at this step);
  * the total mass does not depend on phi: eq. 18 makes every boundary node's exchange with the
    wall vanish, so its dual derivative is zero to rounding.
"""
import numpy as np
import pytest

from oracle import oracle
from paper_2203_04508_amd import workloads as W

TC = W.CS_TC
RV, RL = W.MAXWELL[0.7]


def case():
    dims = (32, 24, 1)
    shapes = np.array([W.band_y(-0.5, 3.4, 0), W.ball((10.3, 3.4), 3.1, 0), W.ball((21.7, 3.4), 2.6, 0)], np.int64)
    P = oracle.make_params(2, *dims, tau=0.8, T=0.7 * TC)
    solid = oracle.classify(P, shapes)
    node, d, cls, q = oracle.links(P, shapes, solid)
    walls = oracle.wall_nodes(P, solid)
    rho0 = W.drop_field(dims, 2, [((16.0, 11.0), 6.0)], RV, RL, 2.0)
    return P, solid, node, d, q, walls, rho0


@pytest.mark.parametrize("kind,prm", [(0, (RV, 1.0)), (1, ((RV + RL) / 2, 0.1 * (RL - RV)))])
def test_dual_derivative_matches_central_differences(kind, prm):
    P, solid, node, d, q, walls, rho0 = case()
    rng = np.random.default_rng(5)
    phi = rng.uniform(0.9, 1.1, len(walls))
    dirs = rng.standard_normal((4, len(walls)))
    nsteps = 20
    ds = oracle.DualSim(P, solid, node, d, q)
    ds.set_phi(phi, dirs)
    ds.init_eq(rho0)
    ds.step(nsteps)
    L, dL = ds.loss(kind, prm)

    def f(ph):
        s = oracle.Sim(P, solid, node, d, q)
        s.set_phi(ph)
        s.init_eq(rho0)
        s.step(nsteps)
        return oracle.sim_loss(s, kind, prm)

    assert abs(L - f(phi)) <= 1e-13 * abs(L)
    h = 1e-6
    fd = np.array([(f(phi + h * v) - f(phi - h * v)) / (2 * h) for v in dirs])
    assert np.all(np.abs(dL - fd) <= 1e-5 * np.abs(fd) + 1e-9), (dL, fd)


def test_total_mass_does_not_depend_on_phi():
    P, solid, node, d, q, walls, rho0 = case()
    rng = np.random.default_rng(6)
    ds = oracle.DualSim(P, solid, node, d, q)
    ds.set_phi(rng.uniform(0.85, 1.15, len(walls)), rng.standard_normal((4, len(walls))))
    ds.init_eq(rho0)
    ds.step(30)
    M, dM = ds.loss(2)
    assert np.abs(dM).max() < 1e-13 * M


def test_dual_chempot_wall_potential_against_central_difference():
    """Chemical-potential model: the tangent carried by a wall node's assigned potential through
    ten steps equals the central difference of the double simulation."""
    from oracle import thermo

    _, Tc = thermo.critical_point_pr()
    T = 0.8 * Tc
    rv, rl = W.PR_MAXWELL[0.80]
    dims = (24, 20, 1)
    shapes = np.array([W.band_y(-0.5, 3.4, 0), W.ball((10.3, 3.4), 3.1, 0)], np.int64)
    rho0 = W.drop_field(dims, 2, [((12.0, 9.0), 5.0)], rv, rl, 6.0)
    P = oracle.make_params(2, *dims, tau=0.8, T=0.05)
    solid = oracle.classify(P, shapes)
    node, d, cls, q = oracle.links(P, shapes, solid)
    nw = len(oracle.wall_nodes(P, solid))
    mu = 0.0106 + 0.001 * np.random.default_rng(0).standard_normal(nw)
    dirs = np.zeros((2, nw))
    dirs[0, 5] = 1.0
    dirs[1] = np.random.default_rng(1).standard_normal(nw)
    ds = oracle.DualSim(P, solid, node, d, q)
    ds.set_chempot(T, k=0.2, kappa=0.01)
    ds.set_phi(np.ones(nw))
    ds.set_mu_wall(mu, dirs)
    ds.init_eq(rho0)
    ds.step(10)
    L, dL = ds.loss(0, (rv, 1.0))

    def loss(m):
        s = oracle.Sim(P, solid, node, d, q)
        s.set_chempot(T, k=0.2, kappa=0.01)
        s.set_mu_wall(m)
        s.init_eq(rho0)
        s.step(10)
        v = oracle.sim_loss(s, 0, (rv, 1.0))
        s.close()
        return v

    assert L == loss(mu)
    h = 1e-6
    for k in range(2):
        fd = (loss(mu + h * dirs[k]) - loss(mu - h * dirs[k])) / (2 * h)
        assert abs(dL[k] - fd) < 1e-3 * abs(fd) + 1e-9, (k, dL[k], fd)
