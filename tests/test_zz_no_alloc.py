"""mcb_mass_static, the entry point that allocates nothing (its reduction works in a static device
array of the library), against mcb_mass through the C ABI: the same kernels in the same order, so
every field of the report must be bit-identical; two calls in a row on one device, the second on a
smaller lattice, and a repeated call (the array keeps the last call's contents, which must not
leak into the next)."""
import sys

import numpy as np
import pytest

from paper_2203_04508_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mcb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_04508_amd import mcb as m
    m.load()
    return m


def _fields(r):
    return (r.M, r.J[0], r.J[1], r.J[2], r.dM_last, r.n_nan, r.n_domain, r.t)


def _lattice(mcb, dims, seed, precision):
    rng = np.random.default_rng(seed)
    shapes = W.random_links_case(rng, dims, 2, max(3, dims[0] * dims[1] // 2500), 4.0, 12.0)
    rv, rl = W.MAXWELL[0.7]
    drops = [((rng.uniform(0, dims[0]), rng.uniform(0, dims[1])), rng.uniform(6, 20)) for _ in range(4)]
    lat = mcb.Lattice(2, dims, 0.9, 0.7 * W.CS_TC, precision=precision, rho_ref=0.0 if precision == "f64" else rv)
    lat.set_geometry(shapes)
    lat.set_wettability(rng.uniform(0.9, 1.1, lat.n_wall))
    lat.init_equilibrium(W.drop_field(dims, 2, drops, rv, rl, 2.0))
    lat.step(37)
    return lat


@pytest.mark.parametrize("precision", ["f64", "f32s"])
def test_mass_static_matches_mass(mcb, precision):
    for dims, seed in (((640, 384, 1), 5), ((96, 80, 1), 6)):  # the second call on a smaller lattice
        print(f"\n[case] mcb_mass_static vs mcb_mass, {dims[0]}x{dims[1]}, {precision}", flush=True)
        sys.stdout.flush()
        lat = _lattice(mcb, dims, seed, precision)
        ref = _fields(lat.mass())
        got = _fields(lat.mass_static())
        assert got == ref, (got, ref)
        assert _fields(lat.mass_static()) == ref  # again, over the previous call's contents
        assert ref[0] > 0 and ref[4] != 0.0
        lat.close()
