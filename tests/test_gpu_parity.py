"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the same seeded inputs.

Bars (FP64): link lists and wall-node lists bit-exact; post-collision populations within 1e-12
relative per step and 1e-9 after 1000 steps, the relative error of a direction plane being
max|f_gpu - f_oracle| / max|f_oracle| over fluid nodes; relative mass drift <= 1e-12.
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
    """max over direction planes of max|a - b| / max|b| on fluid nodes"""
    worst = 0.0
    for i in range(a.shape[0]):
        d = np.abs(a[i, fluid] - b[i, fluid]).max()
        s = np.abs(b[i, fluid]).max()
        worst = max(worst, d / s)
    return worst


def build_pair(mcb, dim, dims, tau, T, shapes, phi=None, q_override=None, precision="f64", rho_ref=0.0):
    P = oracle.make_params(dim, *dims, tau=tau, T=T)
    solid = oracle.classify(P, shapes)
    node, d, cls, q = oracle.links(P, shapes, solid)
    lat = mcb.Lattice(dim, dims, tau, T, precision=precision, rho_ref=rho_ref)
    nl, nb, nw = lat.set_geometry(shapes)
    walls = oracle.wall_nodes(P, solid)
    assert nl == len(node) and nw == len(walls)
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


# ------------------------------------------------------------------ geometry, bit-exact
GEOM_CASES = [
    ("2d-balls-13x11", 2, (13, 11, 1), [W.ball((4.3, 5.1), 2.7, 0), W.ball((9.6, 3.3), 1.9, 1), W.ball((12.5, 9.9), 2.2, 2)]),
    ("2d-band-12x14", 2, (12, 14, 1), [W.band_y(-0.5, 2.35, 0), W.ball((5.2, 2.35), 2.3, 0), W.ball((10.7, 2.35), 1.6, 0)]),
    ("2d-on-node", 2, (11, 11, 1), [W.ball((5.0, 5.0), 3.0, 0)]),
    ("3d-balls", 3, (7, 8, 6), [W.ball((3.2, 3.9, 2.7), 2.1, 0), W.ball((6.1, 0.4, 4.8), 1.7, 1)]),
]


def _compare_geometry(mcb, dim, dims, shapes):
    P = oracle.make_params(dim, *dims)
    solid = oracle.classify(P, shapes)
    node, d, cls, q = oracle.links(P, shapes, solid)
    walls = oracle.wall_nodes(P, solid)
    lat = mcb.Lattice(dim, dims, 1.0, 0.066)
    nl, nb, nw = lat.set_geometry(shapes)
    assert (nl, nw) == (len(node), len(walls))
    assert nb == len(np.unique(node))
    got = lat.links()
    assert np.array_equal(got["node"], node)
    assert np.array_equal(got["dir"], d)
    assert np.array_equal(got["q_fixed"], q)
    assert np.array_equal(got["cls"], cls)
    assert np.array_equal(lat.wall_nodes(), walls)
    lat.close()


@pytest.mark.parametrize("name,dim,dims,shapes", GEOM_CASES, ids=[c[0] for c in GEOM_CASES])
def test_geometry_bitexact_small(mcb, name, dim, dims, shapes):
    banner(f"geometry {name}")
    _compare_geometry(mcb, dim, dims, np.array(shapes, np.int64))


@pytest.mark.parametrize("name", ["c0", "c1", "c3"])
def test_geometry_bitexact_workloads(mcb, name):
    banner(f"geometry workload {name}")
    wl = W.make(name)
    _compare_geometry(mcb, wl.dim, wl.dims, wl.shapes)


# ------------------------------------------------------------------ step parity
def _random_state(rng, sim_dims, rho_field, dim=2):
    Q = 9 if dim == 2 else 19
    N = len(rho_field)
    f = np.zeros((Q, N))
    for x in range(N):
        f[:, x] = oracle.equilibrium(dim, rho_field[x], rng.uniform(-0.02, 0.02, dim))
    return f * (1.0 + 0.01 * rng.standard_normal(f.shape))


TINY = [
    # name, dims, seed, q override
    ("300x70-ragged", (300, 70, 1), 1, None),
    ("37x29-random-q", (37, 29, 1), 2, "random"),
    ("40x34-half-q", (40, 34, 1), 3, "half"),
    # the ends of the two branches of the boundary condition, set on purpose: q = 0 (eq. 16 with
    # c1 = 0), q = 1/2 - 2^-16 (eq. 16 next to the switch), q = 1/2 (eq. 17, bounce-back), q = 1
    # (eq. 17 with weights 1/2), and q = 2^-16
    ("41x31-q-endpoints", (41, 31, 1), 4, "endpoints"),
]


@pytest.mark.parametrize("name,dims,seed,qmode", TINY, ids=[c[0] for c in TINY])
def test_step_parity_small(mcb, name, dims, seed, qmode):
    banner(f"step parity {name}")
    rng = np.random.default_rng(seed)
    nballs = max(3, dims[0] * dims[1] // 900)
    shapes = W.random_links_case(rng, dims, 2, nballs, 2.0, 6.0)
    rv, rl = W.MAXWELL[0.7]
    drops = [((rng.uniform(0, dims[0]), rng.uniform(0, dims[1])), rng.uniform(4, 9)) for _ in range(3)]
    rho = W.drop_field(dims, 2, drops, rv, rl, 2.0)
    qo = None
    if qmode == "random":
        qo = lambda q: rng.integers(0, 65537, len(q))
    elif qmode == "half":
        qo = lambda q: np.full(len(q), 32768)
    elif qmode == "endpoints":
        qo = lambda q: rng.choice(np.array([0, 1, 32767, 32768, 65536]), len(q))
    phi = rng.uniform(0.8, 1.15)
    sim, lat, fluid = build_pair(mcb, 2, dims, 0.8, 0.7 * TC, shapes, phi=phi, q_override=qo)
    f0 = _random_state(rng, dims, rho)
    sim.set_f(f0)
    lat.set_f(f0)
    e0 = rel_err(lat.get_f(), sim.get_f(), fluid)
    assert e0 < 1e-13, e0
    for k in range(1, 21):
        sim.step(1)
        lat.step(1)
        e = rel_err(lat.get_f(), sim.get_f(), fluid)
        assert e < 1e-12 * k, (k, e)
    rep = lat.mass()
    assert abs(rep.dM_last - sim.dm_last()) < 1e-12 * max(1.0, abs(sim.dm_last()))
    if qmode == "half":
        assert rep.dM_last == 0.0
    if qmode == "endpoints":
        cls = lat.links()["cls"]
        assert set(cls.tolist()) >= {0, 2}, "both branches present"
    # the monitor's mass and momentum against the oracle's state (FP64 reductions)
    fo = sim.get_f()
    e, *_ = oracle.lattice(2)
    J_o = (fo[:, fluid].T @ e[:, :2].astype(float)).sum(0)
    scale = (np.abs(fo[:, fluid]).T @ np.abs(e[:, :2]).astype(float)).sum()
    assert abs(rep.M - sim.mass()) <= 1e-13 * sim.mass()
    assert np.abs(np.array(rep.J[:2]) - J_o).max() <= 1e-13 * scale, (rep.J[:2], J_o)
    assert rep.J[2] == 0.0


def test_c0_parity_1000_steps_and_mass(mcb):
    banner("c0 parity, 1000 steps")
    wl = W.make("c0")
    P = oracle.make_params(2, *wl.dims, tau=wl.tau, T=wl.T)
    solid = oracle.classify(P, wl.shapes)
    phi = W.phi_for_walls(wl, oracle.wall_nodes(P, solid))
    sim, lat, fluid = build_pair(mcb, 2, wl.dims, wl.tau, wl.T, wl.shapes, phi=phi)
    rho0 = wl.rho0()
    sim.init_eq(rho0)
    lat.init_equilibrium(rho0)
    M0 = lat.mass().M
    assert abs(M0 - sim.mass()) / sim.mass() < 1e-14
    assert rel_err(lat.get_f(), sim.get_f(), fluid) < 1e-13
    sim.step(1)
    lat.step(1)
    assert rel_err(lat.get_f(), sim.get_f(), fluid) < 1e-12
    sim.step(999)
    lat.step(999)
    e = rel_err(lat.get_f(), sim.get_f(), fluid)
    assert e < 1e-9, e
    rho_g, v_g = lat.moments()
    rho_o, v_o, _ = sim.moments()
    assert np.abs(rho_g - rho_o)[fluid].max() / rho_o[fluid].max() < 1e-9
    assert np.abs(v_g - v_o)[:, fluid].max() < 1e-9 * max(1e-3, np.abs(v_o).max()) + 1e-13
    lat.step(1000)
    rep = lat.mass()
    assert abs(rep.M - M0) / M0 < 1e-12, (rep.M - M0) / M0


def test_c1_full_size_one_step_parity(mcb):
    banner("c1 full size (1024^2), 1 + 9 steps")
    wl = W.make("c1")
    P = oracle.make_params(2, *wl.dims, tau=wl.tau, T=wl.T)
    solid = oracle.classify(P, wl.shapes)
    phi = W.phi_for_walls(wl, oracle.wall_nodes(P, solid))
    sim, lat, fluid = build_pair(mcb, 2, wl.dims, wl.tau, wl.T, wl.shapes, phi=phi)
    rho0 = wl.rho0()
    sim.init_eq(rho0)
    lat.init_equilibrium(rho0)
    assert rel_err(lat.get_f(), sim.get_f(), fluid) < 1e-13
    sim.step(1)
    lat.step(1)
    assert rel_err(lat.get_f(), sim.get_f(), fluid) < 1e-12
    sim.step(9)
    lat.step(9)
    assert rel_err(lat.get_f(), sim.get_f(), fluid) < 1e-11


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32s", 3e-6), ("f16s", 3e-3)])
def test_wide_strip_path_parity(mcb, prec, tol):
    """Lattices above 2^21 nodes take the cache-line-aligned wide strips (224 output columns, 192
    with FP16 storage; ragged last strip) and, with FP32 storage, 16-row segments with a ragged last
    one of 6 rows; one oracle-checked run of three steps."""
    banner(f"wide-strip path, 2100x1030, {prec}")
    dims = (2100, 1030, 1)
    rng = np.random.default_rng(77)
    shapes = W.random_links_case(rng, dims, 2, 40, 6.0, 20.0)
    rv, rl = W.MAXWELL[0.7]
    drops = [((rng.uniform(0, dims[0]), rng.uniform(0, dims[1])), rng.uniform(15, 40)) for _ in range(12)]
    rho = W.drop_field(dims, 2, drops, rv, rl, 2.0)
    T = 0.7 * TC
    P = oracle.make_params(2, *dims, tau=0.9, T=T)
    sim, (solid, *_r) = oracle.sim_from_shapes(P, shapes)
    phi = rng.uniform(0.9, 1.1, sim.n_wall)
    sim.set_phi(phi)
    lat = mcb.Lattice(2, dims, 0.9, T, precision=prec, rho_ref=0.0 if prec == "f64" else rv)
    lat.set_geometry(shapes)
    lat.set_wettability(phi)
    sim.init_eq(rho)
    lat.init_equilibrium(rho)
    fluid = solid == 0
    for k in range(1, 4):
        sim.step(1)
        lat.step(1)
        e = rel_err(lat.get_f(), sim.get_f(), fluid)
        assert e < tol * (k + 1), (k, e)
    lat.close()


def test_half_q_gives_zero_compensation_on_gpu(mcb):
    banner("q = 1/2 everywhere: dM == 0 exactly")
    wl = W.make("c0")
    lat = mcb.Lattice(2, wl.dims, wl.tau, wl.T)
    lat.set_geometry(wl.shapes)
    links = lat.links()
    links["q_fixed"] = 32768
    lat.set_links(links)
    assert np.all(lat.links()["cls"] == 2)
    lat.set_wettability(1.05)
    lat.init_equilibrium(wl.rho0())
    M0 = lat.mass().M
    for _ in range(5):
        lat.step(40)
        rep = lat.mass()
        assert rep.dM_last == 0.0
    assert abs(rep.M - M0) / M0 < 1e-13


def test_deterministic_bitwise(mcb):
    banner("two identical runs are bit-identical")
    wl = W.make("c0")
    out = []
    for _ in range(2):
        lat = mcb.Lattice(2, wl.dims, wl.tau, wl.T)
        lat.set_geometry(wl.shapes)
        lat.set_wettability(0.95)
        lat.init_equilibrium(wl.rho0())
        lat.step(300)
        out.append((lat.get_f(), lat.mass().M))
        lat.close()
    assert np.array_equal(out[0][0], out[1][0]) and out[0][1] == out[1][1]


def test_nan_population_reported(mcb):
    banner("a non-finite population passed to mcb_set_f -> MCB_ENAN")
    wl = W.make("c0")
    P = oracle.make_params(2, *wl.dims, tau=wl.tau, T=wl.T)
    sim, (solid, *_r) = oracle.sim_from_shapes(P, wl.shapes)
    lat = mcb.Lattice(2, wl.dims, wl.tau, wl.T)
    lat.set_geometry(wl.shapes)
    lat.set_wettability(1.0)
    lat.init_equilibrium(wl.rho0())
    f = lat.get_f()
    x = int(np.nonzero(solid == 0)[0][100])
    f[3, x] = np.nan
    with pytest.raises(mcb.MCBError) as ei:
        lat.set_f(f)
    assert ei.value.code == mcb.MCB_ENAN
    # an infinite one as well, and the report counts the node after a step
    f[3, x] = np.inf
    with pytest.raises(mcb.MCBError) as ei:
        lat.set_f(f)
    assert ei.value.code == mcb.MCB_ENAN
    lat.close()


def test_domain_error_reported(mcb):
    banner("psi domain error -> MCB_EDOMAIN")
    wl = W.make("c0")
    lat = mcb.Lattice(2, wl.dims, wl.tau, wl.T)
    lat.set_geometry(wl.shapes)
    lat.set_wettability(1.6)
    with pytest.raises(mcb.MCBError) as ei:
        lat.init_equilibrium(wl.rho0())
        lat.step(20)
        lat.sync()
    assert ei.value.code == mcb.MCB_EDOMAIN


@pytest.mark.parametrize("dim,dims", [(2, (37, 29, 1)), (3, (13, 11, 9))], ids=["2d-37x29", "3d-13x11x9"])
def test_dm_cum_is_the_sum_of_the_steps_corrections(mcb, dim, dims):
    """track_dm: dM_cum equals the oracle's eq. 18 totals summed over the steps (Sec. 3.2), restarts
    with a new state, and is NaN when not tracked."""
    banner(f"running Delta M sum {dims}")
    rng = np.random.default_rng(77 + dim)
    shapes = W.random_links_case(rng, dims, dim, 3, 2.0 if dim == 2 else 1.5, 6.0 if dim == 2 else 3.5)
    rv, rl = W.MAXWELL[0.7]
    drops = [(tuple(rng.uniform(0, n) for n in dims[:dim]), rng.uniform(3, 6)) for _ in range(2)]
    rho = W.drop_field(dims, dim, drops, rv, rl, 2.0)
    P = oracle.make_params(dim, *dims, tau=0.8, T=0.7 * TC)
    solid = oracle.classify(P, shapes)
    node, d, cls, q = oracle.links(P, shapes, solid)
    walls = oracle.wall_nodes(P, solid)
    phi = rng.uniform(0.85, 1.15, len(walls))
    sim = oracle.Sim(P, solid, node, d, q)
    sim.set_phi(phi)
    lat = mcb.Lattice(dim, dims, 0.8, 0.7 * TC, track_dm=True)
    plain = mcb.Lattice(dim, dims, 0.8, 0.7 * TC)
    for L in (lat, plain):
        L.set_geometry(shapes)
        L.set_wettability(phi)
        L.init_equilibrium(rho)
    sim.init_eq(rho)
    assert lat.mass().dM_cum == 0.0 and np.isnan(plain.mass().dM_cum)
    total, scale = 0.0, 0.0
    for k in range(25):
        sim.step(1)
        lat.step(1)
        total += sim.dm_last()
        scale += abs(sim.dm_last())
    rep = lat.mass()
    assert scale > 0.0
    assert abs(rep.dM_cum - total) <= 1e-12 * scale, (rep.dM_cum, total)
    plain.step(3)
    assert np.isnan(plain.mass().dM_cum)
    # a new state starts the sum again
    lat.init_equilibrium(rho)
    assert lat.mass().dM_cum == 0.0
    lat.step(1)
    rep = lat.mass()
    assert abs(rep.dM_cum - rep.dM_last) <= 1e-13 * max(abs(rep.dM_last), 1e-300), (rep.dM_cum, rep.dM_last)
    lat.close()
    plain.close()
    sim.close()
