"""The counter summaries bench.py reads back: HBM bytes per launch from FETCH_SIZE / WRITE_SIZE
scaled by a copy of known size, and SQ instruction counts per lattice update, from rocprofv3
databases (here small sqlite files of the same `counters_collection` shape)."""
import json
import os
import sqlite3

import pytest

from paper_1812_05401_amd import counters as C
from paper_1812_05401_amd import inputs as I


def db(folder, rows):
    os.makedirs(os.path.join(folder, "host", "123"), exist_ok=True)
    con = sqlite3.connect(os.path.join(folder, "host", "123", "run_results.db"))
    con.execute("create table counters_collection (kernel_name text, counter_name text, "
                "value real, grid_size integer)")
    con.executemany("insert into counters_collection values (?, ?, ?, 0)", rows)
    con.commit()
    con.close()
    return str(folder)


S2 = "vplbm::step2_kernel<1, 128, 8, true, false>(vplbm::StepArgs)"
S1 = "vplbm::step_kernel<1, true>(vplbm::StepArgs)"
CP = "__amd_rocclr_copyBuffer(char*, char*)"


def test_traffic_scales_by_the_copy_and_compares_with_the_algorithmic_bytes(tmp_path):
    gib = 1 << 30
    cf = db(tmp_path / "cf", [(CP, "FETCH_SIZE", 524288.0)] * 3)           # reads half of 1 GiB
    cw = db(tmp_path / "cw", [(CP, "WRITE_SIZE", 1048576.0)] * 3)
    case = I.oscillating_cylinder_8192x2048()
    n = case.nodes
    # a two-step launch: the planes and both masks read once (74 B per node with moving bodies
    # in all, 37 + 1 read), the planes written once; the median over dispatches is taken
    rd2, wr2 = (36 + 2) * n, 36 * n
    f = db(tmp_path / "f", [(S2, "FETCH_SIZE", rd2 / 2048.0)] * 5 + [(S2, "FETCH_SIZE", 1.0)]
           + [(S1, "FETCH_SIZE", 37 * n / 2048.0)] * 4 + [(CP, "FETCH_SIZE", 9.0)])
    w = db(tmp_path / "w", [(S2, "WRITE_SIZE", wr2 / 1024.0)] * 6
           + [(S1, "WRITE_SIZE", 36 * n / 1024.0)] * 4)
    table, lines = C.traffic([f"oscillating_cylinder_8192x2048:f32={f},{w}"], [cf, cw], gib)
    two = table["oscillating_cylinder_8192x2048/f32/2"]
    one = table["oscillating_cylinder_8192x2048/f32/1"]
    assert two["fetch_scale"] == 2.0 and two["write_scale"] == 1.0
    assert two["dispatches"] == 6 and two["lattice_updates_per_launch"] == 2
    assert two["algorithmic_bytes_per_launch"] == 74 * n
    assert two["bytes_per_launch"] == 74 * n and two["ratio_to_algorithmic"] == 1.0
    assert two["bytes_per_lattice_update"] == 37.0
    assert one["algorithmic_bytes_per_launch"] == 73 * n and one["ratio_to_algorithmic"] == 1.0
    assert two["source_digest"] == C.source_digest() and two["kernel"] == S2.split("(")[0]
    assert any("step2_kernel" in ln for ln in lines)


def test_valu_counts_per_lattice_update(tmp_path):
    case = I.cylinder_wake_2048x512()
    n = case.nodes
    waves = 2 * n // 64
    rows = []
    for name, spl, valu in ((S2, 2, 204.0), (S1, 1, 264.0)):
        u = n * spl
        rows += [(name, "SQ_INSTS_VALU", valu * u / 64), (name, "SQ_WAVES", waves),
                 (name, "SQ_INSTS_SALU", 367.5 * waves), (name, "SQ_INSTS_VMEM_RD", 7.15 * u / 64),
                 (name, "SQ_INSTS_VMEM_WR", 4.5 * u / 64), (name, "SQ_INSTS_LDS", 11.5 * u / 64)]
    d = db(tmp_path / "v", rows * 3)
    table, _ = C.valu([f"cylinder_wake_2048x512:f32={d}"])
    e = table["cylinder_wake_2048x512/f32/2"]
    assert e["valu_per_lattice_update"] == 204.0 and e["lds_per_lattice_update"] == 11.5
    assert e["vmem_rd_per_lattice_update"] == 7.15 and e["salu_per_wave"] == 367.5
    assert e["valu_lane_instr_per_launch"] == 204 * 2 * n and e["dispatches"] == 3
    assert table["cylinder_wake_2048x512/f32/1"]["valu_per_lattice_update"] == 264.0


def test_cli_writes_the_table_bench_reads(tmp_path, monkeypatch):
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    n = I.cylinder_wake_2048x512().nodes
    cf = db(tmp_path / "cf", [(CP, "FETCH_SIZE", 524288.0)])
    cw = db(tmp_path / "cw", [(CP, "WRITE_SIZE", 1048576.0)])
    f = db(tmp_path / "f", [(S2, "FETCH_SIZE", 37 * n / 2048.0)])
    w = db(tmp_path / "w", [(S2, "WRITE_SIZE", 36 * n / 1024.0)])
    (tmp_path / "profiles").mkdir()
    out = tmp_path / "profiles" / "traffic.json"
    assert C.main(["traffic", "--out", str(out), "--copy", f"{cf},{cw}",
                   f"cylinder_wake_2048x512:f32={f},{w}"]) == 0
    assert json.loads(out.read_text())["cylinder_wake_2048x512/f32/2"]["bytes_per_launch"] == 73 * n
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("cylinder_wake_2048x512", "f32", 2) == 73 * n


def test_a_missing_database_is_an_error(tmp_path):
    with pytest.raises(FileNotFoundError):
        C.dispatch_values(str(tmp_path))


def test_source_digest_ignores_comments_and_layout(tmp_path):
    """A counter summary stays valid across an edit of a comment or of whitespace, not across an
    edit of code."""
    import shutil
    src = os.path.join(os.path.dirname(C.__file__), "csrc")
    for f in C.KERNEL_SOURCES:
        shutil.copy(os.path.join(src, f), tmp_path / f)
    base = C.source_digest(str(tmp_path))
    assert base == C.source_digest()
    k = tmp_path / "kernels.hpp"
    text = k.read_text()
    k.write_text(text.replace("//", "//  (edited)", 1) + "\n/* a block\n   comment */\n")
    assert C.source_digest(str(tmp_path)) == base
    k.write_text(text.replace(";", ";\n\n    ", 1))
    assert C.source_digest(str(tmp_path)) == base
    k.write_text(text + "\nstatic const int vplbm_digest_probe = 1;\n")
    assert C.source_digest(str(tmp_path)) != base
