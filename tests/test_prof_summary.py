"""Host checks of the rocprofv3 summary helper (no GPU): the kernel table, the
copy-calibrated traffic figure and its invalidation when the kernel's sources
change."""
import csv
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _load():
    spec = importlib.util.spec_from_file_location(
        "prof_summary", os.path.join(ROOT, "paper_2301_04259_amd", "prof_summary.py")
    )
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


P = _load()


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_stats_table_sorted_by_total(tmp_path):
    _write(
        str(tmp_path / "kt" / "run_kernel_stats.csv"),
        ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"],
        [
            ["void soap::k_small(int)", 2, 2000, 1000, 10.0, 900, 1100, 1],
            ["void soap::k_apply<float, 4>(soap::Args)", 3, 18000, 6000, 90.0, 5900, 6100, 1],
        ],
    )
    out = P.stats(str(tmp_path / "kt")).splitlines()
    assert out[1].startswith("soap::k_apply<float, 4>")
    assert "6.00" in out[1] and "18.0" in out[1]
    assert out[2].startswith("soap::k_small")


def _counters(path, counter, rows):
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    _write(path, hdr, [[d, k, counter, v] for d, k, v in rows])


def test_traffic_scales_by_copy_calibration(tmp_path):
    calib = 1 << 20
    # the copy reads calib bytes but FETCH_SIZE reports half of them; two
    # counter instances per dispatch are summed
    _counters(
        str(tmp_path / "f" / "run_counter_collection.csv"),
        "FETCH_SIZE",
        [
            (1, "void at::native::neg_kernel_cuda(x)", calib / 2048 / 2),
            (1, "void at::native::neg_kernel_cuda(x)", calib / 2048 / 2),
            (2, "void soap::k_apply<float>(a)", 100.0),
            (2, "void soap::k_apply<float>(a)", 100.0),
            (3, "void soap::k_apply<float>(a)", 200.0),
            (3, "void soap::k_apply<float>(a)", 200.0),
        ],
    )
    _counters(
        str(tmp_path / "w" / "run_counter_collection.csv"),
        "WRITE_SIZE",
        [
            (1, "void at::native::neg_kernel_cuda(x)", calib / 1024),
            (2, "void soap::k_apply<float>(a)", 50.0),
            (3, "void soap::k_apply<float>(a)", 50.0),
        ],
    )
    txt = P.traffic(str(tmp_path / "f"), str(tmp_path / "w"), "k_apply", "neg_kernel", calib)
    vals = dict(ln.split(": ", 1) for ln in txt.splitlines() if ln.count(":") == 1 and "bytes" in ln)
    # fetch: mean 300 KiB per dispatch, factor 2; write: 50 KiB, factor 1
    assert float(vals["read_bytes_per_launch"]) == pytest.approx(300 * 1024 * 2)
    assert float(vals["write_bytes_per_launch"]) == pytest.approx(50 * 1024)
    assert float(vals["traffic_bytes_per_launch"]) == pytest.approx(300 * 1024 * 2 + 50 * 1024)


def test_read_traffic_and_source_hash(tmp_path):
    f = tmp_path / "t.txt"
    f.write_text("# comment\ntraffic_bytes_per_launch: 123\nkernel_source_sha256: abc\n")
    assert P.read_traffic(str(f)) == (123.0, "abc")
    assert P.read_traffic(str(tmp_path / "missing.txt")) is None
    h = P.sources_sha256()
    assert len(h) == 64 and h == P.sources_sha256()


def test_committed_traffic_summary_parses():
    path = os.path.join(ROOT, "profiles", "k_apply_full_visible_r115000_traffic.txt")
    tr = P.read_traffic(path)
    assert tr is not None and tr[0] > 0 and len(tr[1]) == 64
