"""GPU parity at the edges of the input space (pseudopotential model, FP64, against the oracle
through the C ABI): periodic boxes without any solid (no links, no wall nodes), and the smallest
lattices the library accepts, where the step's halo rows, columns and planes wrap through the box
more than once, with and without a solid.

Bars as in the other parity tests: populations within 1e-12 relative per step (k steps: k 1e-12),
the mass to 1e-12.
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


def rel_err(a, b, fluid):
    worst = 0.0
    for i in range(a.shape[0]):
        s = np.abs(b[i, fluid]).max()
        worst = max(worst, np.abs(a[i, fluid] - b[i, fluid]).max() / s)
    return worst


def run_pair(mcb, dim, dims, shapes, seed, steps=10):
    rng = np.random.default_rng(seed)
    P = oracle.make_params(dim, *dims, tau=0.8, T=0.7 * TC)
    solid = oracle.classify(P, shapes)
    node, d, cls, q = oracle.links(P, shapes, solid)
    lat = mcb.Lattice(dim, dims, 0.8, 0.7 * TC)
    nl, nb, nw = lat.set_geometry(shapes)
    assert nl == len(node) and nw == len(oracle.wall_nodes(P, solid))
    sim = oracle.Sim(P, solid, node, d, q)
    if nw:
        phi = rng.uniform(0.9, 1.1, nw)
        sim.set_phi(phi)
        lat.set_wettability(phi)
    N = int(np.prod(dims[:dim]))
    Q = 9 if dim == 2 else 19
    # a smooth periodic density between the vapour and a fifth of the liquid density
    xs = np.meshgrid(*[np.arange(n) for n in reversed(dims[:dim])], indexing="ij")[::-1]
    wave = np.ones(N)
    for k in range(dim):
        wave = wave * (0.5 + 0.5 * np.sin(2 * np.pi * xs[k].reshape(-1) / dims[k] + rng.uniform(0, 2 * np.pi)))
    rho = RV + 0.2 * (RL - RV) * wave
    if N > 100000:
        sim.init_eq(rho)
        lat.init_equilibrium(rho)
    else:
        f = np.stack([oracle.equilibrium(dim, rho[x], rng.uniform(-0.01, 0.01, dim)) for x in range(N)], axis=1)
        assert f.shape == (Q, N)
        sim.set_f(f)
        lat.set_f(f)
    fluid = solid == 0
    M0 = lat.mass().M
    for k in range(1, steps + 1):
        sim.step(1)
        lat.step(1)
        e = rel_err(lat.get_f(), sim.get_f(), fluid)
        assert e < 1e-12 * k, (k, e)
    M = lat.mass().M
    assert abs(M - sim.mass()) <= 1e-12 * abs(M0)
    assert abs(M - M0) <= 1e-12 * abs(M0)  # eq. 18 (or no wall at all) keeps the mass
    # the largest speed (the one-pass kernel's strip wraps through a small box several times)
    _, v, _ = sim.moments()
    sp = np.sqrt((v ** 2).sum(0))
    sp[~fluid] = -1.0
    vg, ng = lat.max_speed()
    assert abs(vg - sp.max()) <= 1e-12 * sp.max() and ng == int(np.argmax(sp)), (vg, sp.max(), ng, int(np.argmax(sp)))
    lat.close()
    return nl, nw


NO_SOLID = [("2d-64x48", 2, (64, 48, 1)), ("2d-1500x1400-wide-strips", 2, (1500, 1400, 1)), ("3d-20x18x16", 3, (20, 18, 16))]


@pytest.mark.parametrize("name,dim,dims", NO_SOLID, ids=[c[0] for c in NO_SOLID])
def test_periodic_box_without_solids(mcb, name, dim, dims):
    banner(f"no solids: {name}")
    nl, nw = run_pair(mcb, dim, dims, np.zeros((0, 8), np.int64), 11, steps=3 if dims[0] > 1000 else 10)
    assert nl == 0 and nw == 0


TINY = [("2d-3x3", 2, (3, 3, 1), False), ("2d-3x7", 2, (3, 7, 1), False), ("2d-7x3", 2, (7, 3, 1), False),
        ("2d-5x4-ball", 2, (5, 4, 1), True), ("2d-6x5-ball", 2, (6, 5, 1), True),
        ("3d-3x3x3", 3, (3, 3, 3), False), ("3d-7x6x5-ball", 3, (7, 6, 5), True)]


@pytest.mark.parametrize("name,dim,dims,ball", TINY, ids=[c[0] for c in TINY])
def test_smallest_lattices(mcb, name, dim, dims, ball):
    banner(f"smallest lattices: {name}")
    shapes = np.zeros((0, 8), np.int64)
    if ball:
        c = tuple(0.5 * n + 0.2 for n in dims[:dim])
        shapes = np.array([W.ball(c, 1.1, 0)], np.int64)
    nl, nw = run_pair(mcb, dim, dims, shapes, 12)
    assert (nl > 0) == ball
