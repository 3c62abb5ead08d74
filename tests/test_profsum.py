"""The rocprofv3 summary tool on small synthetic CSV files (CPU only).

profsum turns kernel traces and counter runs into the tables under profiles/; these checks fix
its grouping, the template-instance selection, the counter scaling by the calibration copies,
the live-dispatch filter and the timeline's busy fraction on hand-computed values.
"""
import csv

import pytest

from paper_2502_08034_amd import profsum

COPY = ('"void at::native::elementwise_kernel_manual_unroll<128, 4, at::native::'
        'direct_copy_kernel_cuda(at::TensorIteratorBase&)>(int)"')
REFRESH = '"void socfv::k_march64<2, 1, true, true>(socfv::March64Args, int, int, int)"'
SWEEP = '"void socfv::k_march64<2, 0, false, false>(socfv::March64Args, int, int, int)"'


def write_trace(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z",
                    "Start_Timestamp", "End_Timestamp"])
        for name, grid, t0, t1 in rows:
            w.writerow([name.strip('"'), *grid, t0, t1])


def write_counters(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Grid_Size", "Start_Timestamp",
                    "End_Timestamp", "Counter_Name", "Counter_Value"])
        for d, (name, grid, dur_ns, value) in enumerate(rows):
            # two rows per dispatch (per-XCD parts of one counter) that the tool must add up
            for part in (0.25, 0.75):
                w.writerow([d, name.strip('"'), grid, 1000, 1000 + dur_ns, counter,
                            value * part])


def test_short_names_and_instances():
    assert profsum.short(REFRESH) == "socfv::k_march64<2, 1, true, true>"
    assert profsum._is_kernel(REFRESH, "k_march64")
    assert profsum._is_kernel(REFRESH, "k_march64<2, 1, true, true>")
    assert not profsum._is_kernel(REFRESH, "k_march64<2, 0, false, false>")
    assert not profsum._is_kernel(SWEEP, "k_sweep2")


def test_trace_groups_by_kernel_and_grid(tmp_path, capsys):
    p = tmp_path / "t.csv"
    write_trace(p, [(SWEEP, (256, 4, 1), 0, 10_000), (SWEEP, (256, 4, 1), 0, 30_000),
                    (SWEEP, (128, 4, 1), 0, 5_000), (REFRESH, (256, 4, 1), 0, 2_000),
                    (COPY, (64, 1, 1), 0, 1_000)])
    profsum.trace(str(p), "socfv", split_us=8)
    out = capsys.readouterr().out
    # two 256-wide sweeps: 40 us in total, 20 us on average; the copy is not a socfv kernel
    assert "| socfv::k_march64<2, 0, false, false> | 256x4x1 | 2 | 0.0 | 20.00 |" in out
    assert "| socfv::k_march64<2, 0, false, false> (< 8 us) | 128x4x1 | 1 |" in out
    assert "| socfv::k_march64<2, 1, true, true> (< 8 us) | 256x4x1 | 1 |" in out
    assert "direct_copy" not in out


def test_pmc_scales_by_the_calibration_copies(tmp_path, capsys):
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    cal_f = profsum.CAL_READ / 1024 / 2.0          # the counter reads half the copy's bytes
    cal_w = profsum.CAL_WRITE / 1024 / 1.0
    cells = 1000
    f_rows = [(COPY, 1 << 28, 500_000, cal_f)] * 4 + [
        (REFRESH, 1024, 2_000, 10.0), (REFRESH, 1024, 4_000, 30.0),   # 20 KiB on average
        (SWEEP, 1024, 1_000, 99.0)]
    w_rows = [(COPY, 1 << 28, 500_000, cal_w)] * 4 + [
        (REFRESH, 1024, 2_000, 4.0), (REFRESH, 1024, 4_000, 8.0), (SWEEP, 1024, 1_000, 1.0)]
    write_counters(fetch, "FETCH_SIZE", f_rows)
    write_counters(write, "WRITE_SIZE", w_rows)
    profsum.pmc(str(fetch), str(write), None, "k_march64<2, 1, true, true>", cells, 1, None)
    out = capsys.readouterr().out
    assert "| FETCH_SIZE | 524,288 KiB | 1,048,576 KiB | 2.0000 |" in out
    assert "| WRITE_SIZE | 2,097,152 KiB | 2,097,152 KiB | 1.0000 |" in out
    # read 20 KiB x 2 = 40,960 B = 40.96 B per cell; written 6 KiB = 6.14 B per cell
    assert "= 40.96 B/cell update" in out
    assert "| WRITE_SIZE (raw, x 1.000) | 6 KiB = 6.14 B/cell update |" in out
    assert "| traffic per launch | 0.0000 GB = 47.10 B/cell update |" in out
    assert "| duration under counters | 3.0 us |" in out
    # the live-dispatch filter keeps the 4 us dispatch only: 30 KiB read, 8 KiB written
    profsum.pmc(str(fetch), str(write), None, "k_march64<2, 1, true, true>", cells, 1, None,
                min_us=3.0)
    out = capsys.readouterr().out
    assert "= 61.44 B/cell update" in out and "| duration under counters | 4.0 us |" in out


def test_pmc_needs_the_calibration(tmp_path):
    fetch = tmp_path / "f.csv"
    write_counters(fetch, "FETCH_SIZE", [(REFRESH, 1024, 2_000, 10.0)])
    with pytest.raises(SystemExit):
        profsum.pmc(str(fetch), str(fetch), None, "k_march64", 1000, 1, None)


def test_timeline_busy_fraction(tmp_path, capsys):
    p = tmp_path / "t.csv"
    # window 0..100 us from the first to the last batch launch; 60 us of it busy
    write_trace(p, [("socfv::k_batch_sweep2<false>(int)", (1024, 16, 1), 0, 20_000),
                    ("socfv::k_batch_reduce(int)", (256, 1, 1), 30_000, 50_000),
                    ("socfv::k_batch_sweep2<false>(int)", (1024, 16, 1), 80_000, 100_000)])
    profsum.timeline(str(p), "batch_sweep2", bins=2)
    out = capsys.readouterr().out
    assert "window 0.000 s from the first to the last batch_sweep2 launch: 3 launches, " \
           "GPU busy 0.600" in out
    assert "| 0 | 1 | 20.0 | 0.80 |" in out
