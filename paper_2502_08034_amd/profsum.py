"""Summaries of rocprofv3 CSV output for this library's kernels (a profiling aid: it only
reads CSV files and prints markdown).

``trace CSV [--split-us T]``: dispatch count and duration statistics per (kernel, grid size)
from a ``--kernel-trace`` CSV, so that launches of one kernel on differently sized problems are
not averaged together; with ``--split-us`` each group is split into dispatches of at least T us
and shorter ones (kernels that return at once once a device-side stop is set).

``timeline CSV --window NAME [--bins B]``: GPU busy fraction and the launches of kernels
whose name contains NAME, per time bin over the window from that kernel's first launch to
its last (how a batched solve's launches shrink as problems finish, and whether the host
leaves the GPU idle between them).

``pmc --fetch CSV --write CSV [--sq CSV] --kernel NAME --cells N --updates U``: HBM bytes per
launch of the kernel at its largest grid (NAME with template arguments selects one instance), from ``--pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE``
runs of ``bench.py --profile-sweeps``.  Each counter is scaled by what it reads for the
calibration copies that run launches first (four converting copies of 2^28 FP32 values to
FP64: 1 GiB read and 2 GiB written each), which fixes the counters' unit on this device.
"""
import argparse
import collections
import csv
import hashlib
import os
import statistics
import sys

CAL_ELEMS = 1 << 28
CAL_READ = CAL_ELEMS * 4
CAL_WRITE = CAL_ELEMS * 8


def short(name):
    name = name.strip('"')
    if name.startswith("void "):
        name = name[5:]
    name = name.replace("(anonymous namespace)::", "")
    return name.split("(")[0]


def grid_of(row):
    if "Grid_Size" in row:
        return (int(row["Grid_Size"]),)
    return tuple(int(row[k]) for k in ("Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z") if k in row)


def trace(path, match, split_us=None):
    groups = collections.defaultdict(list)
    with open(path) as f:
        for r in csv.DictReader(f):
            if match not in r["Kernel_Name"]:
                continue
            dur = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
            key = (short(r["Kernel_Name"]), grid_of(r))
            if split_us is not None:
                key += ("" if dur >= split_us * 1e3 else f"< {split_us:g} us",)
            groups[key].append(dur)
    print("| kernel | grid | calls | total ms | avg us | median us | min us | max us |")
    print("|---|---|---|---|---|---|---|---|")
    for key, v in sorted(groups.items(), key=lambda kv: -sum(kv[1])):
        k, g = key[0], key[1]
        if len(key) > 2 and key[2]:
            k = f"{k} ({key[2]})"
        print(f"| {k} | {'x'.join(map(str, g))} | {len(v)} | {sum(v) / 1e6:.1f} | "
              f"{sum(v) / len(v) / 1e3:.2f} | {statistics.median(v) / 1e3:.2f} | "
              f"{min(v) / 1e3:.2f} | {max(v) / 1e3:.2f} |")


def timeline(path, window, bins=20):
    rows = []
    with open(path) as f:
        for r in csv.DictReader(f):
            rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]),
                         short(r["Kernel_Name"])))
    rows.sort()
    sel = [(s, e) for s, e, k in rows if window in k]
    if not sel:
        raise SystemExit(f"no launch of {window} in the trace")
    w0, w1 = sel[0][0], sel[-1][1]
    inwin = [(s, e, k) for s, e, k in rows if s >= w0 and e <= w1]
    busy = sum(e - s for s, e, _ in inwin)
    print(f"window {(w1 - w0) / 1e9:.3f} s from the first to the last {window} launch: "
          f"{len(inwin)} launches, GPU busy {busy / (w1 - w0):.3f}\n")
    print(f"| bin | {window} launches | their average us | busy fraction |")
    print("|---|---|---|---|")
    step = (w1 - w0) / bins
    for i in range(bins):
        a, z = w0 + i * step, w0 + (i + 1) * step
        part = [(s, e, k) for s, e, k in inwin if a <= s < z]
        mine = [e - s for s, e, k in part if window in k]
        frac = sum(e - s for s, e, _ in part) / step
        avg = sum(mine) / len(mine) / 1e3 if mine else 0.0
        print(f"| {i} | {len(mine)} | {avg:.1f} | {frac:.2f} |")


def _counters(path):
    """{dispatch id: (kernel, grid, {counter: value}, duration ns)} in dispatch order."""
    out = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            d = int(r["Dispatch_Id"])
            if d not in out:
                out[d] = (r["Kernel_Name"], int(r["Grid_Size"]), {},
                          int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
            c = out[d][2]
            c[r["Counter_Name"]] = c.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return [out[d] for d in sorted(out)]


def _calibration(rows, counter):
    cal = [c[counter] for name, _, c, _ in rows if "direct_copy" in name][:4]
    if len(cal) < 4:
        raise SystemExit("fewer than four calibration copies in the counter CSV")
    return sum(cal) / len(cal)


def _is_kernel(name, kernel):
    # a NAME with template arguments ("k_march64<2, 1, true, true>") picks that instance,
    # a plain NAME every instance
    s = short(name)
    return s.endswith(kernel) if "<" in kernel else s.split("<")[0].endswith(kernel)


def _kernel_rows(rows, kernel, min_us=None):
    mine = [r for r in rows if _is_kernel(r[0], kernel)]
    if min_us is not None:
        mine = [r for r in mine if r[3] >= min_us * 1e3]
    if not mine:
        raise SystemExit(f"no dispatch of {kernel} in the counter CSV")
    g = max(r[1] for r in mine)
    return [r for r in mine if r[1] == g], g


def pmc(fetch, write, sq, kernel, cells, updates, source, min_us=None):
    fr = _counters(fetch)
    wr = _counters(write)
    f_cal = _calibration(fr, "FETCH_SIZE")
    w_cal = _calibration(wr, "WRITE_SIZE")
    f_fac = CAL_READ / 1024 / f_cal
    w_fac = CAL_WRITE / 1024 / w_cal
    kf, grid = _kernel_rows(fr, kernel, min_us)
    kw, _ = _kernel_rows(wr, kernel, min_us)
    f_kib = statistics.mean(c["FETCH_SIZE"] for _, _, c, _ in kf)
    w_kib = statistics.mean(c["WRITE_SIZE"] for _, _, c, _ in kw)
    rd = f_kib * 1024 * f_fac
    wb = w_kib * 1024 * w_fac
    per = cells * updates
    dur = statistics.mean(d for _, _, _, d in kf)
    if source:
        digest = hashlib.sha256(open(source, "rb").read()).hexdigest()
        print(f"{os.path.basename(source)} sha256 at measurement: {digest}\n")
    print("## Calibration (plain copy of known size)\n")
    print("| counter | reads for the copy | expected | factor |")
    print("|---|---|---|---|")
    print(f"| FETCH_SIZE | {f_cal:,.0f} KiB | {CAL_READ // 1024:,} KiB | {f_fac:.4f} |")
    print(f"| WRITE_SIZE | {w_cal:,.0f} KiB | {CAL_WRITE // 1024:,} KiB | {w_fac:.4f} |")
    print(f"\n## {kernel} per launch (grid {grid}; {cells:,} cells x {updates} update(s); "
          f"{len(kf)} dispatches averaged)\n")
    print("| quantity | value |")
    print("|---|---|")
    print(f"| FETCH_SIZE (raw) | {f_kib:,.0f} KiB |")
    print(f"| DRAM read bytes (x {f_fac:.3f}) | {rd / 1e9:.4f} GB = {rd / per:.2f} B/cell update |")
    print(f"| WRITE_SIZE (raw, x {w_fac:.3f}) | {w_kib:,.0f} KiB = {wb / per:.2f} B/cell update |")
    print(f"| traffic per launch | {(rd + wb) / 1e9:.4f} GB = {(rd + wb) / per:.2f} B/cell update |")
    print(f"| duration under counters | {dur / 1e3:.1f} us |")
    if sq:
        sr = _counters(sq)
        ks, _ = _kernel_rows(sr, kernel, min_us)
        names = sorted(ks[0][2])
        for n in names:
            v = statistics.mean(c[n] for _, _, c, _ in ks)
            extra = ""
            if n == "SQ_INSTS_VALU":
                extra = f" wave instructions = {v * 64 / per:.1f} lane instructions per cell update"
            print(f"| {n} | {v:.4e}{extra} |")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("csv")
    t.add_argument("--match", default="socfv")
    t.add_argument("--split-us", type=float, default=None)
    tl = sub.add_parser("timeline")
    tl.add_argument("csv")
    tl.add_argument("--window", required=True)
    tl.add_argument("--bins", type=int, default=20)
    p = sub.add_parser("pmc")
    p.add_argument("--fetch", required=True)
    p.add_argument("--write", required=True)
    p.add_argument("--sq")
    p.add_argument("--kernel", required=True)
    p.add_argument("--cells", type=int, required=True)
    p.add_argument("--updates", type=int, default=1)
    p.add_argument("--min-us", type=float, default=None,
                   help="average only dispatches lasting at least this long")
    p.add_argument("--source", default=os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                    "csrc", "kernels.hip"))
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        trace(a.csv, a.match, a.split_us)
    elif a.cmd == "timeline":
        timeline(a.csv, a.window, a.bins)
    else:
        pmc(a.fetch, a.write, a.sq, a.kernel, a.cells, a.updates, a.source, a.min_us)


if __name__ == "__main__":
    sys.exit(main())
