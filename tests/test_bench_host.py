"""Host-side logic of bench.py (no GPU): the rocprofv3 summaries behind the committed profiles, the
traffic record's source check, and the one-GPU guard."""
import csv
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def write_csv(path, header, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_kernel_base_name():
    assert bench.kernel_base_name("void jet::(anonymous namespace)::k_apply<1, unsigned short>(int4 const*, long)") \
        == "k_apply"
    assert bench.kernel_base_name("jet::k_rb_select") == "k_rb_select"
    assert bench.kernel_base_name("k_ab_chunks") == "k_ab_chunks"


def test_family_table_counts_head_kernels_and_merges_templates(tmp_path, capsys):
    # apply: head k_apply (two template instances, 3 + 1 calls), rest k_apply_chunks and k_apply_nets
    write_csv(tmp_path / "t_kernel_stats.csv", ["Name", "Calls", "TotalDurationNs", "AverageNs"], [
        ["void jet::k_apply<1, unsigned short>(int*)", 3, 300e6, 100e6],
        ["void jet::k_apply<2, int>(int*)", 1, 100e6, 100e6],
        ["void jet::k_apply_chunks<1, unsigned short>(int*)", 4, 80e6, 20e6],
        ["void jet::k_apply_nets<1, unsigned short, 128>(int*)", 8, 40e6, 5e6],
        ["jet::k_rb_select", 2, 50e6, 25e6],
        ["jet::k_rb_sel_hist", 1, 10e6, 10e6],
    ])
    bench.summarize(str(tmp_path), 0)
    out = capsys.readouterr().out.splitlines()
    apply = next(line for line in out if line.startswith("apply "))
    f = apply.split()
    assert f[1] == "4"                                 # launches: calls of the head kernel
    assert float(f[2]) == pytest.approx(520.0)         # ms: 400 + 80 + 40
    assert float(f[3]) == pytest.approx(130000.0)      # us per launch
    assert "k_apply 4x100000.0us" in apply
    sel = next(line for line in out if line.startswith("rebalance_select "))
    assert sel.split()[1] == "2" and float(sel.split()[2]) == pytest.approx(60.0)


def test_counter_table_scales_by_the_copy_calibration(tmp_path, capsys):
    # five calibration copies of 16 MiB that read as 8192 KiB each: 2048 bytes per counted unit
    rows = [["void jet::k_apply<1, unsigned short>(int*)", "FETCH_SIZE", 100_000.0],
            ["void jet::k_apply<1, unsigned short>(int*)", "FETCH_SIZE", 300_000.0]]
    rows += [["__amd_rocclr_copyBuffer", "FETCH_SIZE", 8192.0]] * 5
    write_csv(tmp_path / "f_counter_collection.csv", ["Kernel_Name", "Counter_Name", "Counter_Value"], rows)
    bench.summarize(str(tmp_path), 16)
    out = capsys.readouterr().out.splitlines()
    assert any("2048.00 bytes per unit" in line for line in out)
    apply = next(line for line in out if line.startswith("apply "))
    f = apply.split()
    assert f[1] == "2"
    assert float(f[2]) == pytest.approx(400_000 * 2048 / 1e6, abs=0.05)
    assert float(f[3]) == pytest.approx(200_000 * 2048 / 1e6, abs=0.0005)


def test_level_table_groups_by_state_build(tmp_path):
    # set-up, then two level refinements (coarsest first), each opened by k_build_ns
    seq = [("k_fill_incidence", 50_000), ("k_build_ns", 5_000), ("k_apply", 20_000), ("k_apply", 30_000),
           ("k_build_ns", 5_000), ("k_rb_select", 100_000)]
    rows, t = [], 1_000_000
    for name, us in seq:
        rows.append([f"void jet::{name}<1>(int*)", t, t + us * 1000])
        t += us * 1000 + 500
    path = tmp_path / "x_kernel_trace.csv"
    write_csv(path, ["Kernel_Name", "Start_Timestamp", "End_Timestamp"], rows)
    lines = bench.summarize_levels(str(path))
    assert lines[1].split()[0] == "set-up" and "k_fill_incidence 1x50000us" in lines[1]
    assert lines[2].split()[:2] == ["level", "1"]      # coarsest of two levels
    assert float(lines[2].split()[2]) == pytest.approx(55.0)
    assert "k_apply 2x25000us" in lines[2]
    assert lines[3].split()[:2] == ["level", "0"]      # finest
    assert float(lines[3].split()[2]) == pytest.approx(105.0)
    assert "k_rb_select 1x100000us" in lines[3]


def test_traffic_record_is_keyed_by_the_kernel_sources():
    # the committed counter figures apply only to the kernel sources they were measured on (the
    # bench reports no traffic once those sources change)
    for rec in bench.TRAFFIC_RECORDS:
        assert rec["family"] in bench.FAMILIES
        assert len(rec["sources_sha256"]) == 64 and rec["bytes_per_step"] > 0
        assert len(bench.kernel_sources_sha256(rec["sources"])) == 64
    assert bench.traffic_per_launch("apply", "no such workload", 10) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
