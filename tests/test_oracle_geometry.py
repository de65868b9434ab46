"""Pins of the oracle's exact geometry: node classes, the fluid-solid link list and q.

Definition (units of 2^-16 lattice spacings, periodic minimum image):
  * a node is solid iff it lies strictly inside some shape;
  * a link (x1, i) joins a fluid node x1 to a solid node x1 + e_i (Sec. 3.1, Figs. 1-2);
  * q_fixed = the first n in [0, 2^16] for which x1 + n e_i / 2^16 lies inside or on some shape,
    q = q_fixed / 2^16 in [0, 1];
  * class: eq. 16 if q < 1/2 and x2 = x1 - e_i is fluid, bounce-back if q < 1/2 and x2 is solid,
    eq. 17 if q >= 1/2.
The brute-force checks below enumerate every n with Python integers.
"""
import numpy as np
import pytest

from oracle import oracle
from paper_2203_04508_amd import workloads as W

ONE = 65536


def _min_image(d, L):
    d = d % L
    return np.where(d >= L // 2, d - L, d)


def brute_solid(dims, dim, shapes):
    nx, ny, nz = dims
    N = nx * ny * nz
    ids = np.arange(N, dtype=np.int64)
    c = [ids % nx, (ids // nx) % ny, ids // (nx * ny)]
    solid = np.zeros(N, bool)
    for s in shapes:
        if s[0] == W.KIND_BALL:
            acc = np.zeros(N, dtype=object)
            for k in range(dim):
                d = _min_image(c[k] * ONE - int(s[1 + k]), dims[k] * ONE).astype(object)
                acc = acc + d * d
            solid |= np.array([a < int(s[4]) ** 2 for a in acc])
        else:
            solid |= ((c[1] * ONE - int(s[5])) % (ny * ONE)) < (int(s[6]) - int(s[5]))
    return solid.astype(np.uint8)


def brute_q(dims, dim, shapes, x1, e):
    nx, ny, nz = dims
    c1 = [x1 % nx, (x1 // nx) % ny, x1 // (nx * ny)]
    n = np.arange(ONE + 1, dtype=np.int64)
    best = None
    for s in shapes:
        if s[0] == W.KIND_BALL:
            acc = np.zeros(ONE + 1, np.int64)
            for k in range(dim):
                d = int(_min_image(np.int64(c1[k] * ONE - int(s[1 + k])), dims[k] * ONE))
                acc += (d + n * e[k]) ** 2
            hit = np.nonzero(acc <= int(s[4]) ** 2)[0]
        else:
            Ly = ny * ONE
            hit = np.nonzero(((c1[1] * ONE + n * e[1] - int(s[5])) % Ly) <= (int(s[6]) - int(s[5])))[0]
        if len(hit):
            best = hit[0] if best is None else min(best, hit[0])
    return best


def brute_links(dims, dim, shapes, solid):
    e, w, wf, opp = oracle.lattice(dim)
    nx, ny, nz = dims
    N = nx * ny * nz
    out = []
    for x in range(N):
        if solid[x]:
            continue
        c = [x % nx, (x // nx) % ny, x // (nx * ny)]
        for i in range(1, len(e)):
            y = [(c[k] + e[i][k]) % dims[k] for k in range(3)]
            yid = y[0] + nx * (y[1] + ny * y[2])
            if solid[yid]:
                q = brute_q(dims, dim, shapes, x, e[i])
                b = [(c[k] - e[i][k]) % dims[k] for k in range(3)]
                bid = b[0] + nx * (b[1] + ny * b[2])
                cls = 2 if q >= ONE // 2 else (1 if solid[bid] else 0)
                out.append((x, i, cls, q))
    return out


def _params(dims, dim):
    return oracle.make_params(dim, dims[0], dims[1], dims[2])


CASES = [
    ("2d-balls", 2, (13, 11, 1), [W.ball((4.3, 5.1), 2.7, 0), W.ball((9.6, 3.3), 1.9, 1), W.ball((12.5, 9.9), 2.2, 2)]),
    ("2d-band+balls", 2, (12, 14, 1), [W.band_y(-0.5, 2.35, 0), W.ball((5.2, 2.35), 2.3, 0), W.ball((10.7, 2.35), 1.6, 0)]),
    ("2d-on-node", 2, (11, 11, 1), [W.ball((5.0, 5.0), 3.0, 0)]),
    ("3d-balls", 3, (7, 8, 6), [W.ball((3.2, 3.9, 2.7), 2.1, 0), W.ball((6.1, 0.4, 4.8), 1.7, 1)]),
]


@pytest.mark.parametrize("name,dim,dims,shapes", CASES, ids=[c[0] for c in CASES])
def test_geometry_matches_brute_force(name, dim, dims, shapes):
    shapes = np.array(shapes, np.int64)
    P = _params(dims, dim)
    solid = oracle.classify(P, shapes)
    assert np.array_equal(solid, brute_solid(dims, dim, shapes))
    node, d, cls, q = oracle.links(P, shapes, solid)
    ref = brute_links(dims, dim, shapes, solid)
    assert len(ref) == len(node) > 0
    for k, (x, i, c, qq) in enumerate(ref):
        assert (node[k], d[k], cls[k], q[k]) == (x, i, c, qq), (k, (node[k], d[k], cls[k], q[k]), (x, i, c, qq))
    # wall nodes: solid nodes with at least one fluid neighbour, ascending
    walls = oracle.wall_nodes(P, solid)
    e, *_ = oracle.lattice(dim)
    nx, ny, nz = dims
    expect = []
    for x in range(len(solid)):
        if not solid[x]:
            continue
        c = [x % nx, (x // nx) % ny, x // (nx * ny)]
        for i in range(1, len(e)):
            y = [(c[k] + e[i][k]) % dims[k] for k in range(3)]
            if not solid[y[0] + nx * (y[1] + ny * y[2])]:
                expect.append(x)
                break
    assert np.array_equal(walls, np.array(expect, np.int64))


def test_circle_centred_on_node_has_eightfold_symmetry():
    dims = (21, 21, 1)
    shapes = np.array([W.ball((10.0, 10.0), 6.3, 0)], np.int64)
    P = _params(dims, 2)
    solid = oracle.classify(P, shapes)
    node, d, cls, q = oracle.links(P, shapes, solid)
    e, *_ = oracle.lattice(2)
    table = {}
    for x, i, qq in zip(node, d, q):
        cx, cy = x % 21 - 10, x // 21 - 10
        table[(cx, cy, e[i][0], e[i][1])] = qq
    # the symmetry group of the square acting on (position, direction)
    for (cx, cy, ex, ey), qq in table.items():
        images = [(cy, cx, ey, ex), (-cx, cy, -ex, ey), (cx, -cy, ex, -ey), (-cy, cx, -ey, ex)]
        for im in images:
            assert table[im] == qq


def test_flat_wall_gives_equal_q_on_axis_and_diagonal_links():
    """q is the wall distance measured along the link as a fraction of its length; for a flat
    horizontal wall at height h above a node row, vertical and diagonal links share q."""
    for top in [2.1, 2.35, 2.5, 2.8, 3.0]:
        dims = (8, 12, 1)
        shapes = np.array([W.band_y(-0.5, top, 0)], np.int64)
        P = _params(dims, 2)
        solid = oracle.classify(P, shapes)
        node, d, cls, q = oracle.links(P, shapes, solid)
        down = [qq for x, i, qq in zip(node, d, q) if i in (4, 7, 8)]
        assert len(down) == 3 * 8 and len(set(down)) == 1
        first_fluid = int(np.ceil(top))
        assert down[0] == first_fluid * ONE - W.fx(top)


def test_integer_translation_invariance():
    rng = np.random.default_rng(11)
    dims = (24, 20, 1)
    shapes = W.random_links_case(rng, dims, 2, 5, 1.5, 4.0)
    P = _params(dims, 2)
    solid = oracle.classify(P, shapes)
    node, d, cls, q = oracle.links(P, shapes, solid)
    sx, sy = 7, 13
    sh = shapes.copy()
    sh[:, 1] += sx * ONE
    sh[:, 2] += sy * ONE
    solid2 = oracle.classify(P, sh)
    node2, d2, cls2, q2 = oracle.links(P, sh, solid2)
    moved = ((node % 24 + sx) % 24) + 24 * ((node // 24 + sy) % 20)
    order = np.lexsort((d, moved))
    assert np.array_equal(moved[order], node2)
    assert np.array_equal(d[order], d2) and np.array_equal(q[order], q2) and np.array_equal(cls[order], cls2)


def test_c0_link_census():
    wl = W.make("c0")
    P = _params(wl.dims, 2)
    solid = oracle.classify(P, wl.shapes)
    node, d, cls, q = oracle.links(P, wl.shapes, solid)
    # the cylinder of radius 12.3 covers about pi r^2 = 475 nodes
    assert 440 < solid.sum() < 510
    assert np.all(q <= ONE)
    assert np.all((q < ONE // 2) == (cls != 2))
