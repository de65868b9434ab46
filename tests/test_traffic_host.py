"""Host logic of the traffic summary (paper_2203_04508_amd/traffic.py): the FETCH_SIZE and
WRITE_SIZE counters (KiB) averaged per dispatch of the pulling kernels, each scaled by what the same
counter reads for the plain 1 GiB copy (scale = copy bytes / copy counter bytes), the per-step total,
and the kernel-source digest.  Synthetic counter databases in the schema rocprofv3 writes; no GPU."""
import json
import sqlite3
import sys
import types

import pytest

sys.path.insert(0, ".")
from paper_2203_04508_amd import traffic  # noqa: E402


def make_db(path, rows):
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (kernel_name text, dispatch_id integer, counter_name text, value real)")
    con.executemany("insert into counters_collection values (?, ?, ?, ?)", rows)
    con.commit()
    con.close()


STEP = "void mcb::(anonymous namespace)::k_step2d<float, float, 256, 224, true, false>(mcb::Args2<float, float>)"
FIRST = "void mcb::(anonymous namespace)::k_step2d<float, float, 256, 224, false, false>(mcb::Args2<float, float>)"
COPY = "__amd_rocclr_copyBuffer"


def test_summary_scales_each_counter_by_the_copy(tmp_path):
    # values in KiB.  FETCH_SIZE reads the 1 GiB copy as 512 MiB (scale 2), WRITE_SIZE whole (scale
    # 1); dispatch 1 of the step reports two instances (summed), the first collision (PULL = false)
    # and the small copies are not counted
    fetch = [(STEP, 1, "FETCH_SIZE", 100.0), (STEP, 1, "FETCH_SIZE", 100.0), (STEP, 2, "FETCH_SIZE", 300.0),
             (FIRST, 0, "FETCH_SIZE", 9e9), (COPY, 3, "FETCH_SIZE", 512.0 * 1024), (COPY, 4, "FETCH_SIZE", 1.0)]
    write = [(STEP, 1, "WRITE_SIZE", 50.0), (STEP, 2, "WRITE_SIZE", 150.0), (FIRST, 0, "WRITE_SIZE", 9e9),
             (COPY, 3, "WRITE_SIZE", 1024.0 * 1024)]
    make_db(tmp_path / "f.db", fetch)
    make_db(tmp_path / "w.db", write)
    args = types.SimpleNamespace(fetch_db=str(tmp_path / "f.db"), write_db=str(tmp_path / "w.db"), workload="c0",
                                 precision="f32s", model="pseudo", collision="bgk", commands="cmd",
                                 out_dir=str(tmp_path / "out"))
    traffic.summarize(args)
    out = json.load(open(tmp_path / "out" / "traffic_c0_f32s.json"))
    assert out["read_scale"] == pytest.approx(2.0)
    assert out["write_scale"] == pytest.approx(1.0)
    k = out["kernels"]["k_step2d"]
    assert k["read_counter_kib_per_dispatch"] == pytest.approx(250.0)
    assert k["read_bytes_per_launch"] == pytest.approx(250.0 * 1024 * 2.0)
    assert k["write_bytes_per_launch"] == pytest.approx(100.0 * 1024)
    assert out["bytes_per_launch"] == pytest.approx(k["read_bytes_per_launch"] + k["write_bytes_per_launch"])
    assert out["bytes_per_step"] == out["bytes_per_launch"]  # one pulling kernel per 2-D step
    assert out["kernel_digest"] == traffic.kernel_digest(2)
    assert (tmp_path / "out" / "traffic_c0_f32s.txt").read_text().startswith("HBM traffic of the step kernels")


def test_names_and_digest():
    assert traffic.out_name("c2", "f32s") == "traffic_c2_f32s"
    assert traffic.out_name("c2", "f32s", "chempot", "mrt") == "traffic_c2_f32s_chempot_mrt"
    assert traffic._pull_kernel("void k_cp_march<float, float, 256, 224, true, true>(x)")
    assert not traffic._pull_kernel("void k_cp_march<float, float, 256, 224, false, true>(x)")
    assert traffic._pull_kernel("void k_rho3d<float, float, true>(x)")
    assert not traffic._pull_kernel("void k_speed2d<float, float>(x)")
    assert traffic.kernel_digest(2) != traffic.kernel_digest(3)
