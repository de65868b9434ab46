"""Byte counts per step that bench.py and the precision study divide by the step time
(paper_2203_04508_amd/roofline.py): the method's bytes, each node's Q populations read and written
once in the stored format plus one byte of tag and about 20 bytes per fluid-solid link, and the
layout's bytes.  Pinned against the figures written out by hand; no GPU."""
import sys
import types

sys.path.insert(0, ".")
from paper_2203_04508_amd import roofline  # noqa: E402


def lattice(N, Q, dim):
    return types.SimpleNamespace(N=N, Q=Q, dim=dim)


def test_method_bytes_per_node_and_link():
    c2 = lattice(4096 * 4096, 9, 2)
    c4 = lattice(256 ** 3, 19, 3)
    # 2 Q s + 1 bytes per node: D2Q9 145 / 73 / 37, D3Q19 305 / 153 / 77 (FP64 / FP32 / FP16)
    for wl, per_node in ((c2, {"f64": 145, "f32s": 73, "f16s": 37}), (c4, {"f64": 305, "f32s": 153, "f16s": 77})):
        for prec, b in per_node.items():
            assert roofline.algorithmic_bytes(wl, prec, 0) == wl.N * b
            assert roofline.algorithmic_bytes(wl, prec, 1000) - roofline.algorithmic_bytes(wl, prec, 0) == 20 * 1000
    # the 4096^2 workload with 1 409 166 links in shifted FP32: 1 252 920 088 bytes per step
    assert roofline.algorithmic_bytes(c2, "f32s", 1409166) == 1252920088


def test_layout_bytes():
    from paper_2203_04508_amd import mcb

    c2 = lattice(4096 * 4096, 9, 2)
    c4 = lattice(256 ** 3, 19, 3)
    nb = 1000
    # populations and a 4-byte tag per node; FP16 storage keeps population 0 in FP32 (one more
    # half-plane pair); each boundary node's record read and written, its link coefficients read
    assert roofline.layout_bytes(c2, "f32s", nb) == c2.N * (2 * 9 * 4 + 4) + nb * (2 * mcb.REC2 + mcb.Q2_LINKS) * 4
    assert roofline.layout_bytes(c2, "f16s", nb) == c2.N * (2 * 10 * 2 + 4) + nb * (2 * mcb.REC2 + mcb.Q2_LINKS) * 4
    assert roofline.layout_bytes(c2, "f64", nb) == c2.N * (2 * 9 * 8 + 4) + nb * (2 * mcb.REC2 + mcb.Q2_LINKS) * 8
    assert roofline.layout_bytes(c4, "f32s", nb) == c4.N * (2 * 19 * 4 + 4) + nb * (2 * mcb.REC3 + mcb.Q3_LINKS) * 4
    # the layout never moves fewer bytes than the method needs once the tags are counted
    for prec in ("f64", "f32s", "f16s"):
        assert roofline.layout_bytes(c2, prec, 0) > roofline.algorithmic_bytes(c2, prec, 0)


def test_peak():
    assert roofline.HBM_PEAK_GBS == 8000.0
