"""Host logic of the profile summaries: counter calibration and the byte model (CPU)."""

import csv

import pytest

from paper_2602_14016_amd import profile_summary as ps
from paper_2602_14016_amd.roofline import algorithmic_bytes, field_bytes, read_traffic


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (name, val) in enumerate(rows):
            w.writerow([i, name, counter, val])


def test_field_bytes_and_classes_at_256():
    Yb, Cb = field_bytes(256)
    assert Yb == 256 * 86 * 16 and Cb == 171 * 86 * 16
    assert algorithmic_bytes(2, 256) == 8 * Yb
    r, w = ps.kernel_rw_bytes("row_adj_kernel<256, 2>", 256)
    assert r + w == algorithmic_bytes(2, 256)
    r, w = ps.kernel_rw_bytes("row_nl_pipe_kernel<256>", 256)
    assert r + w == algorithmic_bytes(0, 256)
    modes = [ps.kernel_rw_bytes(f"col_kernel<256, 1, {m}>", 256) for m in (1, 2, 3, 4)]
    assert sum(a + b for a, b in modes) / 4 == pytest.approx(algorithmic_bytes(1, 256))
    modes = [ps.kernel_rw_bytes(f"col_kernel<256, 1, {m}>", 256) for m in (7, 8, 9, 10)]
    assert sum(a + b for a, b in modes) / 4 == pytest.approx(algorithmic_bytes(3, 256))


def test_traffic_record_calibrates_and_round_trips(tmp_path, monkeypatch):
    # the copy of 512 MiB reads as half its size on FETCH_SIZE and as its size on WRITE_SIZE
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    _counter_csv(fetch, "FETCH_SIZE", [("__amd_rocclr_copyBuffer", 262144.0), ("__amd_rocclr_copyBuffer", 4.0),
                                       ("void pa::row_adj_kernel<256, 2>(pa::Dims, pa::RowArgs)", 50000.0),
                                       ("void pa::row_adj_kernel<256, 2>(pa::Dims, pa::RowArgs)", 52000.0)])
    _counter_csv(write, "WRITE_SIZE", [("__amd_rocclr_copyBuffer", 524288.0),
                                       ("void pa::row_adj_kernel<256, 2>(pa::Dims, pa::RowArgs)", 44032.0)])
    out = tmp_path / "traffic.txt"
    ps.main(["traffic", str(fetch), str(write), "--command", "cmd", "--members", "64", "--N", "256", "--cls", "2",
             "--kernel", "row_adj_kernel<256, 2>", "--calib-mib", "512", "--out", str(out)])
    text = out.read_text()
    assert "scale_fetch: 2.0000" in text and "scale_write: 1.0000" in text
    expect = int(round(1024 * (2.0 * 51000.0 + 1.0 * 44032.0)))
    assert f"hbm_bytes_per_launch: {expect}" in text
    assert read_traffic(2, 256, 64, kernel="row_adj_kernel<256, 2>", path=str(out)) == expect
    assert read_traffic(2, 256, 64, kernel="row_adj_kernel<256, 1>", path=str(out)) is None
    assert read_traffic(0, 256, 64, path=str(out)) is None
    stale = tmp_path / "stale.txt"
    stale.write_text(text.replace("source_sha: ", "source_sha: 0"))
    assert read_traffic(2, 256, 64, path=str(stale)) is None


def test_counter_summary_means_and_shares(tmp_path):
    k = "void pa::row_adj_kernel<256, 2>(pa::Dims, pa::RowArgs)"
    a, b = tmp_path / "a.csv", tmp_path / "b.csv"
    _counter_csv(a, "SQ_WAVE_CYCLES", [(k, 1000.0), (k, 3000.0), ("other", 5.0)])
    _counter_csv(b, "SQ_WAIT_INST_LDS", [(k, 400.0), (k, 400.0)])
    out = tmp_path / "c.txt"
    text = ps.main(["counters", str(a), str(b), "--command", "cmd", "--title", "t",
                    "--kernels", "row_adj_kernel<256, 2>", "--out", str(out)]) or out.read_text()
    assert "kernel: row_adj_kernel<256, 2>" in text
    lines = {l.split()[0]: l.split() for l in text.splitlines() if l.startswith("  SQ_")}
    assert float(lines["SQ_WAVE_CYCLES"][1]) == 2000.0           # mean over the two dispatches
    share = [l for l in text.splitlines() if "share SQ_WAIT_INST_LDS" in l][0]
    assert float(share.split()[-1]) == pytest.approx(0.2)         # 400 / 2000
    with pytest.raises(SystemExit):
        ps.main(["counters", str(a), "--command", "c", "--title", "t", "--kernels", "missing", "--out", str(out)])
