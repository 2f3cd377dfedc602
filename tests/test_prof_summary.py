"""The profile summariser on small synthetic rocprofv3 CSVs (the column layout of rocprofv3's csv output):
dispatch counts and durations of a kernel trace, the copy-calibrated HBM bytes per dispatch, and the
instruction counts per cell with their VALU issue floor."""
import csv
import json
import os
import subprocess
import sys

import pytest

from paper_2202_08778_amd import prof_summary

APPLY = "void vr::k_apply_tiled<float, float, true, false, false, true, 1, 0>(vr::Grid, vr::TileGeom)"
COARSE = APPLY
RESID = "void vr::k_residual_tiled<float, float, float, false, 0, 1>(vr::Grid, vr::TileGeom, int)"
COPY = "__amd_rocclr_copyBuffer"
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _write(path, header, rows):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh, quoting=csv.QUOTE_NONNUMERIC)
        w.writerow(header)
        w.writerows(rows)


def _run(*args):
    r = subprocess.run([sys.executable, "-m", "paper_2202_08778_amd.prof_summary", *map(str, args)],
                       capture_output=True, text=True, cwd=ROOT)
    assert r.returncode == 0, r.stderr


def test_trace_counts_and_durations(tmp_path):
    hdr = ["Kind", "Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp", "Grid_Size_X"]
    rows = [["KERNEL_DISPATCH", 1, APPLY, 1000, 301000, 524288],     # 300 us
            ["KERNEL_DISPATCH", 2, APPLY, 400000, 710000, 524288],   # 310 us
            ["KERNEL_DISPATCH", 3, APPLY, 800000, 815000, 65536]]    # 15 us, a coarse level
    _write(tmp_path / "t.csv", hdr, rows)
    _run("trace", tmp_path / "t.csv", tmp_path / "t.md", "--cmd", "CMD", "--title", "T")
    md = (tmp_path / "t.md").read_text()
    assert "Kernel time in the run: 0.6 ms over 3 dispatches." in md
    line = next(l for l in md.splitlines() if "| 524288 |" in l)
    cells = [c.strip() for c in line.strip("|").split("|")]
    assert cells[0] == "k_apply_tiled<float, float, true, false, false, true, 1, 0>"
    assert cells[2:] == ["2", "0.61", "97.6%", "305.0", "300.0", "310.0"]


def test_hbm_scaled_by_the_calibration_copies(tmp_path):
    hdr = ["Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name", "Counter_Value"]
    mib256 = 256 * 1024   # KiB in 256 MiB
    fetch = [[1, 524288, APPLY, "FETCH_SIZE", 100.0], [2, 524288, APPLY, "FETCH_SIZE", 300.0],
             [3, 65536, COARSE, "FETCH_SIZE", 10.0]]
    write = [[1, 524288, APPLY, "WRITE_SIZE", 50.0], [2, 524288, APPLY, "WRITE_SIZE", 50.0],
             [3, 65536, COARSE, "WRITE_SIZE", 5.0]]
    # an early copy of another size, then the four calibration copies (the run's last): FETCH_SIZE reads
    # half of a copy's bytes, WRITE_SIZE all of them
    fetch.append([4, 65536, COPY, "FETCH_SIZE", 1.0])
    write.append([4, 65536, COPY, "WRITE_SIZE", 1.0])
    for d in range(10, 14):
        fetch.append([d, 65536, COPY, "FETCH_SIZE", mib256 / 2])
        write.append([d, 65536, COPY, "WRITE_SIZE", float(mib256)])
    _write(tmp_path / "f.csv", hdr, fetch)
    _write(tmp_path / "w.csv", hdr, write)
    _run("hbm", tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "h.md", tmp_path / "h.json", "--n", 256,
         "--title", "H", "--cmds", "A", "B")
    rec = json.loads((tmp_path / "h.json").read_text())
    assert rec["read_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    a = rec["classes"]["apply_fp32"]
    assert a["dispatches"] == 2
    assert a["read_bytes"] == pytest.approx(2.0 * 1024 * 200.0)   # mean 200 KiB raw, x 2
    assert a["write_bytes"] == pytest.approx(1024 * 50.0)
    m = rec["classes"]["multigrid_levels"]
    assert m["read_bytes"] == pytest.approx(2.0 * 1024 * 10.0) and m["write_bytes"] == pytest.approx(1024 * 5.0)
    assert len(rec["source_sha256"]) == 64 and rec["commands"] == ["A", "B"]


def test_insts_per_cell_and_issue_floor(tmp_path):
    hdr = ["Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name", "Counter_Value"]
    cells = 16777216
    rows = []
    for d, valu in ((1, 8.0e7), (2, 9.0e7)):        # mean 8.5e7 VALU per dispatch
        rows += [[d, 524288, APPLY, "SQ_INSTS_VALU", valu], [d, 524288, APPLY, "SQ_INSTS_LDS", 1.6e7],
                 [d, 524288, APPLY, "SQ_WAVES", 8192.0]]
    rows += [[3, 524288, RESID, "SQ_INSTS_VALU", 1.2e8], [3, 524288, RESID, "SQ_WAVES", 8192.0],
             [4, 65536, COARSE, "SQ_INSTS_VALU", 5.0e6],      # a coarse level: not listed
             [5, 524288, COPY, "SQ_INSTS_VALU", 1.0e6]]       # not a stencil kernel: not listed
    _write(tmp_path / "i.csv", hdr, rows)
    _run("insts", tmp_path / "i.csv", tmp_path / "i.md", "--cells", cells, "--cmd", "CMD", "--title", "I")
    lines = [l for l in (tmp_path / "i.md").read_text().splitlines() if l.startswith("| k_")]
    assert len(lines) == 2
    assert lines[0].startswith("| k_residual_tiled")   # by VALU per dispatch, largest first
    c = [x.strip() for x in lines[1].strip("|").split("|")]
    assert c[1] == "2" and c[2] == "8192"
    assert float(c[4]) == pytest.approx(8.5e7 * 64 / cells, abs=0.05)           # VALU per cell
    assert float(c[5]) == pytest.approx(1.6e7 * 64 / cells, abs=0.05)           # LDS per cell
    assert float(c[9]) == pytest.approx(8.5e7 / (256 * 2.4e9) * 1e6, abs=0.05)  # floor, us


def test_kernel_class_names():
    assert prof_summary.kernel_class("k_apply_tiled<float>", 100, 100) == "apply_fp32"
    assert prof_summary.kernel_class("k_apply_tiled<float>", 50, 100) == "multigrid_levels"
    assert prof_summary.kernel_class("k_residual_tiled<double>", 100, 100) == "residual_fp64"
    assert prof_summary.kernel_class("at::native::foo", 100, 100) is None
    assert prof_summary.short_name(APPLY) == "k_apply_tiled<float, float, true, false, false, true, 1, 0>"
