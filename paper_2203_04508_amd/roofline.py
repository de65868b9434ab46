"""Byte counts per step that the HBM-roofline figures divide by the step time.

algorithmic_bytes is what the method must move (the roofline's numerator); layout_bytes is what
this implementation's data layout moves at least, which also counts the node tags and boundary
records it chose.
"""
from __future__ import annotations

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
STORAGE_BYTES = {"f64": 8, "f32s": 4, "f16s": 2}


def algorithmic_bytes(wl, precision, nl):
    """Each node's populations read once and written once (2 Q s, s the bytes of a stored
    population) plus one byte of node tag, and about 20 bytes per fluid-solid link (its index,
    direction and class, q, the incoming value and the eq. 18 term)."""
    s = STORAGE_BYTES[precision]
    return wl.N * (2 * wl.Q * s + 1) + 20 * nl


def layout_bytes(wl, precision, nb):
    """Populations (FP16 storage keeps population 0 in FP32), the 4-byte node tag, and each boundary
    node's record read and written once plus its link coefficients, once each (halo re-reads and
    partial lines not counted)."""
    from paper_2203_04508_amd import mcb

    s = STORAGE_BYTES[precision]
    cb = 8 if precision == "f64" else 4
    rec, nlk = (mcb.REC2, mcb.Q2_LINKS) if wl.dim == 2 else (mcb.REC3, mcb.Q3_LINKS)
    planes = wl.Q + 1 if precision == "f16s" else wl.Q
    return wl.N * (2 * planes * s + 4) + nb * (2 * rec + nlk) * cb
