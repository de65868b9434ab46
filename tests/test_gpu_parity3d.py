"""GPU parity of the D3Q19 path against the FP64 oracle, through the C ABI.

Bars as in two dimensions (FP64): link and wall-node lists bit-exact; post-collision populations
within 1e-12 relative per step (max over direction planes of max|f_gpu - f_oracle| / max|f_oracle|
on fluid nodes); eq. 18 total correction equal to rounding.  The small cases span several tiles
in x and y (28 x 12 output columns each), ragged tiles, several z segments, and lattices smaller
than one tile (the tile wraps around the periodic box).
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
    worst = 0.0
    for i in range(a.shape[0]):
        d = np.abs(a[i, fluid] - b[i, fluid]).max()
        s = np.abs(b[i, fluid]).max()
        worst = max(worst, d / s)
    return worst


def build_pair(mcb, dims, tau, T, shapes, phi=None, q_override=None, precision="f64", rho_ref=0.0):
    P = oracle.make_params(3, *dims, tau=tau, T=T)
    solid = oracle.classify(P, shapes)
    node, d, cls, q = oracle.links(P, shapes, solid)
    lat = mcb.Lattice(3, dims, tau, T, precision=precision, rho_ref=rho_ref)
    nl, nb, nw = lat.set_geometry(shapes)
    walls = oracle.wall_nodes(P, solid)
    assert nl == len(node) and nw == len(walls)
    got = lat.links()
    assert np.array_equal(got["node"], node) and np.array_equal(got["dir"], d)
    assert np.array_equal(got["q_fixed"], q) and np.array_equal(got["cls"], cls)
    assert np.array_equal(lat.wall_nodes(), walls)
    if q_override is not None:
        q = q_override(q).astype(np.uint32)
        links = lat.links()
        links["q_fixed"] = q
        lat.set_links(links)
    sim = oracle.Sim(P, solid, node, d, q)
    if phi is not None:
        phi = np.broadcast_to(np.asarray(phi, np.float64), (nw,)).copy()
        sim.set_phi(phi)
        lat.set_wettability(phi)
    return sim, lat, solid == 0


def random_state(rng, rho_field):
    N = len(rho_field)
    u = rng.uniform(-0.02, 0.02, (N, 3))
    f = np.stack([oracle.equilibrium(3, rho_field[x], u[x]) for x in range(N)], axis=1)
    return f * (1.0 + 0.01 * rng.standard_normal(f.shape))


CASES = [
    # name, dims, seed, q override
    ("7x8x6-wrapped-tile", (7, 8, 6), 11, None),
    ("45x30x13-ragged", (45, 30, 13), 12, None),
    ("31x27x19-random-q", (31, 27, 19), 13, "random"),
    ("29x14x12-half-q", (29, 14, 12), 14, "half"),
]


@pytest.mark.parametrize("name,dims,seed,qmode", CASES, ids=[c[0] for c in CASES])
def test_step3d_parity_small(mcb, name, dims, seed, qmode):
    banner(f"D3Q19 step parity {name}")
    rng = np.random.default_rng(seed)
    nballs = max(2, dims[0] * dims[1] * dims[2] // 2500)
    shapes = W.random_links_case(rng, dims, 3, nballs, 1.5, 4.5)
    rv, rl = W.MAXWELL[0.7]
    drops = [(tuple(rng.uniform(0, n) for n in dims), rng.uniform(2.5, 5.0)) for _ in range(3)]
    rho = W.drop_field(dims, 3, drops, rv, rl, 4.0)
    qo = None
    if qmode == "random":
        qo = lambda q: rng.integers(0, 65537, len(q))
    elif qmode == "half":
        qo = lambda q: np.full(len(q), 32768)
    phi = rng.uniform(0.85, 1.15)
    sim, lat, fluid = build_pair(mcb, dims, 0.8, 0.7 * TC, shapes, phi=phi, q_override=qo)
    f0 = random_state(rng, rho)
    sim.set_f(f0)
    lat.set_f(f0)
    assert rel_err(lat.get_f(), sim.get_f(), fluid) < 1e-13
    for k in range(1, 11):
        sim.step(1)
        lat.step(1)
        e = rel_err(lat.get_f(), sim.get_f(), fluid)
        assert e < 1e-12 * k, (k, e)
    rep = lat.mass()
    assert abs(rep.dM_last - sim.dm_last()) < 1e-12 * max(1.0, abs(sim.dm_last()))
    if qmode == "half":
        assert rep.dM_last == 0.0
    lat.close()


def test_step3d_init_and_moments(mcb):
    banner("D3Q19 equilibrium start and moments, 33x26x9")
    dims = (33, 26, 9)
    rng = np.random.default_rng(15)
    shapes = W.random_links_case(rng, dims, 3, 3, 2.0, 4.0)
    rv, rl = W.MAXWELL[0.7]
    rho = W.drop_field(dims, 3, [((16.0, 13.0, 4.5), 5.0)], rv, rl, 4.0)
    sim, lat, fluid = build_pair(mcb, dims, 0.8, 0.7 * TC, shapes, phi=1.1)
    sim.init_eq(rho)
    lat.init_equilibrium(rho)
    assert rel_err(lat.get_f(), sim.get_f(), fluid) < 1e-13
    sim.step(30)
    lat.step(30)
    assert rel_err(lat.get_f(), sim.get_f(), fluid) < 1e-11
    rho_g, v_g = lat.moments()
    rho_o, v_o, _ = sim.moments()
    assert np.abs(rho_g - rho_o)[fluid].max() / rho_o[fluid].max() < 1e-11
    assert np.abs(v_g - v_o)[:, fluid].max() < 1e-11 * max(1e-3, np.abs(v_o).max()) + 1e-14
    assert abs(lat.mass().M - sim.mass()) / sim.mass() < 1e-13


def test_c4_geometry_bitexact(mcb):
    banner("geometry workload c4 (256^3)")
    wl = W.make("c4")
    P = oracle.make_params(3, *wl.dims)
    solid = oracle.classify(P, wl.shapes)
    node, d, cls, q = oracle.links(P, wl.shapes, solid)
    walls = oracle.wall_nodes(P, solid)
    lat = mcb.Lattice(3, wl.dims, wl.tau, wl.T)
    nl, nb, nw = lat.set_geometry(wl.shapes)
    assert (nl, nw) == (len(node), len(walls))
    got = lat.links()
    assert np.array_equal(got["node"], node) and np.array_equal(got["dir"], d)
    assert np.array_equal(got["q_fixed"], q) and np.array_equal(got["cls"], cls)
    assert np.array_equal(lat.wall_nodes(), walls)
    lat.close()


@pytest.mark.parametrize("prec,tol", [("f32s", 2e-6), ("f16s", 2e-3)])
def test_step3d_shifted_storage(mcb, prec, tol):
    banner(f"D3Q19 {prec} against the FP64 oracle, 45x30x13")
    dims = (45, 30, 13)
    rng = np.random.default_rng(16)
    shapes = W.random_links_case(rng, dims, 3, 6, 1.5, 4.5)
    rv, rl = W.MAXWELL[0.7]
    rho = W.drop_field(dims, 3, [((20.0, 15.0, 6.0), 5.0)], rv, rl, 4.0)
    T = 0.7 * TC
    P = oracle.make_params(3, *dims, tau=0.8, T=T)
    sim, (solid, *_r) = oracle.sim_from_shapes(P, shapes)
    sim.set_phi(1.05)
    lat = mcb.Lattice(3, dims, 0.8, T, precision=prec, rho_ref=rv)
    lat.set_geometry(shapes)
    lat.set_wettability(1.05)
    sim.init_eq(rho)
    lat.init_equilibrium(rho)
    fluid = solid == 0
    assert rel_err(lat.get_f(), sim.get_f(), fluid) < tol
    for k in range(1, 11):
        sim.step(1)
        lat.step(1)
        e = rel_err(lat.get_f(), sim.get_f(), fluid)
        assert e < tol * (k + 1), (k, e)
    lat.close()
