"""Host side of the flat-substrate q-sweep: the geometry gives every link into the substrate the
chosen q on a fixed set of solid rows, and the contact-angle fit recovers the angle of a synthetic
circular cap."""
import math

import numpy as np
import pytest

from oracle import oracle
from paper_2203_04508_amd import qsweep as Q, workloads as W


@pytest.mark.parametrize("q", [0.0, 0.2, 0.5, 0.8])
def test_substrate_links_share_q(q):
    shapes, rho0, yw, rv, rl = Q.setup(q)
    P = oracle.make_params(2, Q.NX, Q.NY, 1, tau=1.0, T=0.7 * W.CS_TC)
    solid = oracle.classify(P, shapes)
    assert np.array_equal(np.nonzero(solid.reshape(Q.NY, Q.NX).all(1))[0], np.arange(Q.Y1))
    node, d, cls, qq = oracle.links(P, shapes, solid)
    upper = node // Q.NX == Q.Y1
    assert upper.sum() == 3 * Q.NX  # three links down from every node of the first fluid row
    assert np.all(np.abs(qq[upper] / W.ONE - q) <= 0.5 / W.ONE)
    assert np.all(qq[~upper] == W.ONE // 2)  # the band's underside


@pytest.mark.parametrize("theta", [45.0, 60.0, 90.0, 120.0, 140.0])
def test_contact_angle_of_a_circular_cap(theta):
    yw, R = 10.7, 50.0
    yc = yw - R * math.cos(math.radians(theta))
    yy, xx = np.mgrid[0:Q.NY, 0:Q.NX]
    r = np.sqrt((xx - 250.3) ** 2 + (yy - yc) ** 2)
    rv, rl = W.MAXWELL[0.7]
    rho = 0.5 * (rv + rl) + 0.5 * (rv - rl) * np.tanh(2.0 * (r - R) / 2.0)
    rho[yy < yw] = 0.0
    assert abs(Q.contact_angle(rho.reshape(-1), yw, rv, rl) - theta) < 0.05
