"""The C-ABI library loads on a machine without a GPU, exports every entry point that
include/mcb.h declares, and its structs have the layouts the Python binding assumes.
No compute calls are made here."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mcb.h")
LIB = os.path.join(ROOT, "paper_2203_04508_amd", "libmcb.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mcb_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libmcb.so not built (python paper_2203_04508_amd/build.py)")
    return C.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_header():
    from paper_2203_04508_amd import mcb
    assert sorted(mcb.EXPORTS) == declared_functions()


def test_struct_layouts_match_header(tmp_path):
    from paper_2203_04508_amd import mcb
    src = tmp_path / "sz.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "mcb.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu\\n\", sizeof(mcb_params), sizeof(mcb_shape),"
        " sizeof(mcb_link), sizeof(mcb_sizes), sizeof(mcb_buffers), sizeof(mcb_mass_report),"
        " offsetof(mcb_params, cp_kappa)); return 0;}\n")
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    want = [C.sizeof(mcb.mcb_params), C.sizeof(mcb.mcb_shape), C.sizeof(mcb.mcb_link), C.sizeof(mcb.mcb_sizes),
            C.sizeof(mcb.mcb_buffers), C.sizeof(mcb.mcb_mass_report), mcb.mcb_params.cp_kappa.offset]
    assert got == want
    assert mcb.LINK_DTYPE.itemsize == C.sizeof(mcb.mcb_link)


def test_host_side_argument_checks(lib):
    """Parameter validation and sizing run on the host only."""
    from paper_2203_04508_amd import mcb
    mcb.load(LIB)
    good = mcb.mcb_params(2, 64, 64, 1, 1.0, -1.0, 1.0, 4.0, 1.0, 0.066, mcb.MCB_F64, 0, 0.0)
    sz = mcb.mcb_required_sizes(good, 1)
    assert sz.lattice_bytes >= 2 * 9 * 64 * 64 * 8 and sz.links_bytes == 0
    sz2 = mcb.mcb_required_sizes(good, 1, 100, 40, 30)
    assert sz2.links_bytes > 0
    for bad in [dict(tau=0.5), dict(G=1.0), dict(nx=2), dict(dim=4), dict(precision=7), dict(nz=5),
                dict(bc_mode=4), dict(bc_mode=-1)]:
        p = mcb.mcb_params(2, 64, 64, 1, 1.0, -1.0, 1.0, 4.0, 1.0, 0.066, mcb.MCB_F64, 0, 0.0)
        for k, v in bad.items():
            setattr(p, k, v)
        with pytest.raises(mcb.MCBError) as ei:
            mcb.mcb_create(p)
        assert ei.value.code == mcb.MCB_EINVAL
    # every boundary scheme in 2-D and 3-D
    for mode in (mcb.MCB_BC_PRESENT, mcb.MCB_BC_IBC, mcb.MCB_BC_MIBC, mcb.MCB_BC_HBBC):
        p = mcb.mcb_params(2, 64, 64, 1, 1.0, -1.0, 1.0, 4.0, 1.0, 0.066, mcb.MCB_F64, mode, 0.0)
        mcb.mcb_destroy(mcb.mcb_create(p))
        p3 = mcb.mcb_params(3, 16, 16, 16, 1.0, -1.0, 1.0, 4.0, 1.0, 0.066, mcb.MCB_F64, mode, 0.0)
        mcb.mcb_destroy(mcb.mcb_create(p3))
    # MRT: D2Q9 only, rates in (0, 2)
    pm = mcb.mcb_params(2, 64, 64, 1, 1.0, -1.0, 1.0, 4.0, 1.0, 0.066, mcb.MCB_F64, 0, 0.0, mcb.MCB_COLL_MRT, 0,
                        *mcb.MRT_RATES_PAPER)
    mcb.mcb_destroy(mcb.mcb_create(pm))
    for k, v in (("s_e", 2.0), ("s_q", 0.0), ("collision", 2)):
        bad = mcb.mcb_params(2, 64, 64, 1, 1.0, -1.0, 1.0, 4.0, 1.0, 0.066, mcb.MCB_F64, 0, 0.0, mcb.MCB_COLL_MRT, 0,
                             *mcb.MRT_RATES_PAPER)
        setattr(bad, k, v)
        with pytest.raises(mcb.MCBError) as ei:
            mcb.mcb_create(bad)
        assert ei.value.code == mcb.MCB_EINVAL
    # gravity: finite, no z component in 2-D
    for gz in ((0.0, 0.0, 1e-5), (float("nan"), 0.0, 0.0)):
        bad = mcb.mcb_params(2, 64, 64, 1, 1.0, -1.0, 1.0, 4.0, 1.0, 0.066, mcb.MCB_F64, 0, 0.0)
        bad.gravity[:] = gz
        with pytest.raises(mcb.MCBError) as ei:
            mcb.mcb_create(bad)
        assert ei.value.code == mcb.MCB_EINVAL
    # chemical-potential model: D2Q9 only, k > 0, kappa >= 0; G is not used
    pc = mcb.mcb_params(2, 64, 64, 1, 1.0, 0.0, 2 / 49, 2 / 21, 1.0, 0.058, mcb.MCB_F64, 0, 0.0)
    pc.model, pc.pr_omega, pc.cp_k, pc.cp_kappa = mcb.MCB_MODEL_CHEMPOT, 0.344, 0.2, 0.01
    mcb.mcb_destroy(mcb.mcb_create(pc))
    for k, v in (("cp_k", 0.0), ("cp_kappa", -1.0), ("model", 2)):
        bad = mcb.mcb_params(2, 64, 64, 1, 1.0, 0.0, 2 / 49, 2 / 21, 1.0, 0.058, mcb.MCB_F64, 0, 0.0)
        bad.model, bad.pr_omega, bad.cp_k, bad.cp_kappa = mcb.MCB_MODEL_CHEMPOT, 0.344, 0.2, 0.01
        setattr(bad, k, v)
        with pytest.raises(mcb.MCBError) as ei:
            mcb.mcb_create(bad)
        assert ei.value.code == mcb.MCB_EINVAL
    pc3 = mcb.mcb_params(3, 16, 16, 16, 1.0, 0.0, 2 / 49, 2 / 21, 1.0, 0.058, mcb.MCB_F64, 0, 0.0)
    pc3.model, pc3.pr_omega, pc3.cp_k, pc3.cp_kappa = mcb.MCB_MODEL_CHEMPOT, 0.344, 0.2, 0.01
    with pytest.raises(mcb.MCBError) as ei:
        mcb.mcb_create(pc3)
    assert ei.value.code == mcb.MCB_ENOTSUP
    p3.bc_mode, p3.collision, p3.s_e, p3.s_eps, p3.s_q = 0, mcb.MCB_COLL_MRT, 1.64, 1.54, 1.7
    with pytest.raises(mcb.MCBError) as ei:
        mcb.mcb_create(p3)
    assert ei.value.code == mcb.MCB_ENOTSUP
    h = mcb.mcb_create(good)
    # calls out of order are refused before any device work
    with pytest.raises(mcb.MCBError) as ei:
        mcb.mcb_step(h, 1)
    assert ei.value.code == mcb.MCB_ESTATE
    with pytest.raises(mcb.MCBError) as ei:
        mcb.mcb_set_geometry(h, [[1, 0, 0, 0, 65536, 0, 0, 0]])
    assert ei.value.code == mcb.MCB_ESTATE
    mcb.mcb_destroy(h)
