"""Host checks of the seeded input recipes (paper_2203_04508_amd/workloads.py): the geometry
generator's spacing guarantees, determinism, the drop profile and the chemical-potential inputs."""
import numpy as np
import pytest
from scipy.spatial import cKDTree

from paper_2203_04508_amd import workloads as W


def surface_gaps(wl, reach=60.0):
    """Smallest surface-to-surface distances between the balls of a 2-D workload (periodic)."""
    S = wl.shapes.astype(np.float64)
    c = S[:, 1:3] / W.ONE
    r = S[:, 4] / W.ONE
    L = np.array(wl.dims[:2], np.float64)
    tree = cKDTree(np.mod(c, L), boxsize=L)
    out = []
    for a, b in tree.query_pairs(reach):
        d = c[a] - c[b]
        d -= L * np.round(d / L)
        out.append(np.sqrt((d ** 2).sum()) - r[a] - r[b])
    return np.array(out)


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_min_gap_keeps_the_balls_apart(name):
    wl = W.make(name, min_gap=W.CP_MIN_GAP)
    g = surface_gaps(wl)
    assert len(wl.shapes) == (300 if name == "c1" else 4800)
    assert g.min() > W.CP_MIN_GAP
    assert wl.extra["min_gap"] == W.CP_MIN_GAP


def test_without_gap_the_balls_only_avoid_overlap():
    # the default recipe lets balls nearly touch: the sub-lattice gaps the chemical-potential runs avoid
    g = surface_gaps(W.make("c1"))
    assert g.min() > 0.0
    assert (g < 1.0).sum() > 0


def test_recipes_are_deterministic():
    a, b = W.make("c1"), W.make("c1")
    assert np.array_equal(a.shapes, b.shapes) and a.drops == b.drops
    assert np.array_equal(a.phi_group, b.phi_group)
    c = W.make("c1", min_gap=W.CP_MIN_GAP)
    assert not np.array_equal(a.shapes, c.shapes)


def test_drop_profile_and_chempot_inputs():
    wl = W.make("c0")
    rv, rl = W.PR_MAXWELL[0.80]
    rho = W.drop_field(wl.dims, 2, wl.drops, rv, rl, W.CP_WIDTH)
    assert rho.min() >= rv - 1e-12 and rho.max() <= rl + 1e-12
    (cx, cy), rd = wl.drops[0]
    nx = wl.dims[0]
    # eq. 19 at a node near the centre and at one beyond the drop, written out
    for x, y in ((int(round(cx)), int(round(cy))), (int(round(cx)), int(round(cy - rd - 4)))):
        r = np.hypot(x - cx, y - cy)
        want = 0.5 * (rv + rl) - 0.5 * (rl - rv) * np.tanh(2.0 * (r - rd) / W.CP_WIDTH)
        assert abs(rho[y * nx + x] - want) < 1e-12 * rl
    from oracle import oracle
    P = oracle.make_params(2, *wl.dims, tau=wl.tau, T=wl.T)
    walls = oracle.wall_nodes(P, oracle.classify(P, wl.shapes))
    rho0, mu_s, rv0 = W.chempot_inputs(wl, walls)
    assert np.array_equal(rho0, rho) and rv0 == rv
    mu_coex = W.CP_K ** 2 * W.MU_PR_COEX[0.80]
    assert mu_s.shape == (len(walls),) and len(walls) > 0
    assert np.allclose(mu_s, mu_coex * W.phi_for_walls(wl, walls), rtol=0, atol=0)


def test_stored_thermodynamic_constants_match_the_eos():
    """The Carnahan-Starling critical temperature and Maxwell densities the workloads store, recomputed
    from the EOS (critical point from p' = p'' = 0; equal areas)."""
    from oracle import thermo

    rc, Tc = thermo.critical_point()
    assert abs(W.CS_TC / Tc - 1) < 1e-13
    for tr, (rv, rl) in W.MAXWELL.items():
        v, l = thermo.maxwell(tr * Tc)
        assert abs(rv / v - 1) < 1e-9 and abs(rl / l - 1) < 1e-9, (tr, rv, v, rl, l)
