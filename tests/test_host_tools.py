"""Host-side tools without a GPU: the bench's command line contract and the
profile summaries (on small synthetic rocprofv3-style CSV files)."""
import csv
import json
import os
import subprocess
import sys

from paper_1901_07993_amd import prof_summary as PS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def _write(path, header, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def _trace(path):
    # dispatch, name, start, end (ns): a first factorization, then a second one
    rows = [(1, "__amd_rocclr_copyBuffer", 0, 100),
            (2, "lif::(anonymous namespace)::k_chol_scatter(int)", 1000, 1100),
            (3, "void lif::(anonymous namespace)::k_numeric_f64<64, false, false, true>(long)", 1100, 2100),
            (4, "lif::(anonymous namespace)::k_chol_scatter(int)", 5000, 5100),
            (5, "void lif::(anonymous namespace)::k_numeric_f64<64, false, false, true>(long)", 5100, 7100),
            (6, "void lif::(anonymous namespace)::k_numeric_f64<64, false, false, true>(long)", 7100, 9100)]
    _write(path, ["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"], rows)


def _counters(path, name, per_kib):
    # the probe copy (4 MiB) counts half its size; kernels count per_kib KiB
    rows = [(1, "__amd_rocclr_copyBuffer", name, 2048.0),
            (2, "lif::(anonymous namespace)::k_chol_scatter(int)", name, 1.0),
            (3, "void lif::(anonymous namespace)::k_numeric_f64<64, false, false, true>(long)", name, per_kib),
            (4, "lif::(anonymous namespace)::k_chol_scatter(int)", name, 1.0),
            (5, "void lif::(anonymous namespace)::k_numeric_f64<64, false, false, true>(long)", name, per_kib),
            (6, "void lif::(anonymous namespace)::k_numeric_f64<64, false, false, true>(long)", name, per_kib)]
    _write(path, ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"], rows)


def test_profile_summaries(tmp_path):
    tr, fe, wr = tmp_path / "t.csv", tmp_path / "f.csv", tmp_path / "w.csv"
    _trace(tr)
    _counters(fe, "FETCH_SIZE", 1000.0)
    _counters(wr, "WRITE_SIZE", 500.0)
    # stats: the last factorization only (3 kernels from the second k_chol_scatter)
    PS.stats(str(tr), str(tmp_path / "s.md"), "T", "C", groups=("k_numeric_f64", "k_none"))
    text = (tmp_path / "s.md").read_text()
    assert "3 kernels" in text and "| `k_numeric_f64<64, false, false, true>` | 2 | 0.004 |" in text
    # a group's totals: 2 calls of 2 us each, 4 of the 4.1 us summed; an empty group is left out
    assert "All `k_numeric_f64*` kernels together: 2 calls, 0.004 ms, average 2.0 us per call, 97.6 %" in text
    assert "k_none" not in text
    # traffic: counts scaled by the probe's factor 2 (4 MiB counted as 2 MiB)
    PS.traffic(str(fe), str(wr), str(tmp_path / "x.json"), "k_numeric_f64", 4.0, "C", "h")
    t = json.load(open(tmp_path / "x.json"))
    assert t["fetch_calibration"] == 2.0 and t["fetch_dispatches"] == 3
    assert t["bytes_per_launch"] == 2.0 * 1000.0 * 1024 + 2.0 * 500.0 * 1024
    # hbm: bytes per dispatch / mean duration over the last factorization
    PS.hbm(str(tr), str(fe), str(wr), str(tmp_path / "h.md"), 4.0, 8000.0, "T", "C")
    row = [ln for ln in (tmp_path / "h.md").read_text().splitlines() if "k_numeric_f64" in ln][0]
    cells = [c.strip() for c in row.strip("|").split("|")]
    mb, us, gbps = float(cells[3]), float(cells[4]), float(cells[5])
    assert abs(mb - 3.072) < 0.006 and us == 2.0 and abs(gbps - 3.072e6 / 2e3) < 1.0
