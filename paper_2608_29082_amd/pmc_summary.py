"""Summaries of rocprofv3 output: per-kernel statistics and calibrated HBM traffic.

    python -m paper_2608_29082_amd.pmc_summary stats  STATS_CSV [--top N]
    python -m paper_2608_29082_amd.pmc_summary traffic FETCH_CSV WRITE_CSV COPY_FETCH_CSV COPY_WRITE_CSV
           [--copy-mib 256] [--kernel NAME] [--json OUT] [--workload TEXT]
    python -m paper_2608_29082_amd.pmc_summary counters CSV [CSV ...] --kernel NAME [--kernel NAME ...]

`stats` prints a markdown table (calls, total ms, average us, share) from a
`--kernel-trace --stats` run's `*_kernel_stats.csv`.

`counters` prints, for each named kernel, the mean per dispatch of every
counter in the given `--pmc` passes (one table row per counter).

`traffic` reads two counter passes (`--pmc FETCH_SIZE`, then `--pmc
WRITE_SIZE`; KiB per dispatch) of the same program and the same passes of a
plain device copy of --copy-mib MiB (paper_2608_29082_amd.copycal), which
reads and writes exactly that many bytes per dispatch.  The copy fixes one
scale factor per counter; the table gives each kernel's mean calibrated MB
read and written per dispatch.  With --kernel and --json it also writes that
kernel's calibrated bytes per dispatch, tagged with the SHA-256 of the kernel
sources, which the benchmark reports as `roofline.traffic` while the sources
are unchanged.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))


def kernel_sources_sha256() -> str:
    """SHA-256 over the kernel and tiling sources (csrc/kernels.hpp, csrc/tiles.hpp)."""
    h = hashlib.sha256()
    for name in ("kernels.hpp", "tiles.hpp"):
        with open(os.path.join(HERE, "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def short_name(name: str) -> str:
    """Kernel symbol without the leading return type and the parameter list."""
    s = name.strip()
    if s.startswith("void "):
        s = s[5:]
    depth = 0
    for i, ch in enumerate(s):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return s[:i]
    return s


def read_stats(path: str):
    rows = []
    with open(path, newline="") as fh:
        for r in csv.DictReader(fh):
            rows.append((short_name(r["Name"]), int(r["Calls"]), float(r["TotalDurationNs"]),
                         float(r["AverageNs"]), float(r["Percentage"])))
    rows.sort(key=lambda t: -t[2])
    return rows


def stats_table(path: str, top: int = 25) -> str:
    out = ["| kernel | calls | total ms | avg us | % |", "|---|---:|---:|---:|---:|"]
    for name, calls, tot, avg, pct in read_stats(path)[:top]:
        out.append(f"| `{name}` | {calls} | {tot / 1e6:.2f} | {avg / 1e3:.2f} | {pct:.1f} |")
    return "\n".join(out)


def read_counter(path: str, counter: str):
    """kernel -> list of per-dispatch values of one counter."""
    vals = defaultdict(list)
    with open(path, newline="") as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] == counter:
                vals[short_name(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return vals


def mean(v):
    return sum(v) / len(v) if v else 0.0


def calibration(copy_fetch: str, copy_write: str, mib: int):
    """Scale factors that turn FETCH_SIZE / WRITE_SIZE KiB into bytes read / written,
    from a copy kernel that reads and writes mib MiB per dispatch."""
    kib = mib * 1024.0
    f = read_counter(copy_fetch, "FETCH_SIZE")
    w = read_counter(copy_write, "WRITE_SIZE")
    fk = max(f, key=lambda k: len(f[k]))      # the copy kernel: the most dispatched one
    wk = max(w, key=lambda k: len(w[k]))
    fm, wm = mean(f[fk]), mean(w[wk])
    if fm <= 0 or wm <= 0:
        raise ValueError("copy calibration counters are zero")
    return kib / fm, kib / wm, fm, wm


def traffic(fetch: str, write: str, copy_fetch: str, copy_write: str, mib: int = 256, top: int = 12):
    ff, fw, fm, wm = calibration(copy_fetch, copy_write, mib)
    f = read_counter(fetch, "FETCH_SIZE")
    w = read_counter(write, "WRITE_SIZE")
    rows = []
    for k in set(f) | set(w):
        rd = mean(f.get(k, [])) * ff * 1024.0
        wr = mean(w.get(k, [])) * fw * 1024.0
        n = max(len(f.get(k, [])), len(w.get(k, [])))
        rows.append((k, n, mean(f.get(k, [])), mean(w.get(k, [])), rd, wr))
    rows.sort(key=lambda t: -(t[1] * (t[4] + t[5])))
    table = ["| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | calibrated MB read | calibrated MB written |",
             "|---|---:|---:|---:|---:|---:|"]
    for k, n, fk, wk, rd, wr in rows[:top]:
        table.append(f"| `{k}` | {n} | {fk:.0f} | {wk:.0f} | {rd / 1e6:.1f} | {wr / 1e6:.1f} |")
    cal = (f"Calibration (KiB per dispatch of a {mib * 1024} KiB read + {mib * 1024} KiB write copy): "
           f"FETCH_SIZE {fm:.0f}, WRITE_SIZE {wm:.0f} -> factors fetch x{ff:.3f}, write x{fw:.3f}.")
    return "\n".join(table), cal, {k: (rd, wr) for k, n, fk, wk, rd, wr in rows}, (ff, fw)


def counters_table(paths, kernels) -> str:
    """Mean per dispatch of every counter in the CSV files, for each kernel."""
    vals = defaultdict(lambda: defaultdict(list))
    for path in paths:
        with open(path, newline="") as fh:
            for r in csv.DictReader(fh):
                vals[short_name(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    names = sorted({c for k in kernels for c in vals.get(k, {})})
    out = ["| counter | " + " | ".join(f"`{k}`" for k in kernels) + " |",
           "|---|" + "---:|" * len(kernels)]
    for c in names:
        out.append(f"| {c} | " + " | ".join(f"{mean(vals[k][c]):.4g}" if vals[k].get(c) else "" for k in kernels)
                   + " |")
    out.append("| dispatches | " + " | ".join(str(max((len(v) for v in vals[k].values()), default=0))
                                                for k in kernels) + " |")
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--top", type=int, default=25)
    cs = sub.add_parser("counters")
    cs.add_argument("csv", nargs="+")
    cs.add_argument("--kernel", action="append", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("fetch")
    t.add_argument("write")
    t.add_argument("copy_fetch")
    t.add_argument("copy_write")
    t.add_argument("--copy-mib", type=int, default=256)
    t.add_argument("--kernel", default=None, help="kernel symbol (without parameters) for --json")
    t.add_argument("--json", default=None)
    t.add_argument("--workload", default="")
    t.add_argument("--source", default="")
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        print(stats_table(a.csv, a.top))
        return
    if a.cmd == "counters":
        print(counters_table(a.csv, a.kernel))
        return
    table, cal, per, (ff, fw) = traffic(a.fetch, a.write, a.copy_fetch, a.copy_write, a.copy_mib)
    print(cal)
    print()
    print(table)
    if a.kernel and a.json:
        if a.kernel not in per:
            raise SystemExit(f"kernel {a.kernel!r} not in the counter files")
        rd, wr = per[a.kernel]
        rec = {"kernel": a.kernel, "workload": a.workload, "bytes_per_dispatch": rd + wr, "read_bytes": rd,
               "written_bytes": wr,
               "counters": f"FETCH_SIZE x{ff:.3f} and WRITE_SIZE x{fw:.3f} (KiB per dispatch, calibrated on a "
                           f"{a.copy_mib} MiB device copy)",
               "source": a.source, "kernel_sources_sha256": kernel_sources_sha256()}
        with open(a.json, "w") as fh:
            json.dump(rec, fh, indent=1)
            fh.write("\n")
        print(f"\nwrote {a.json}: {(rd + wr) / 1e6:.1f} MB per dispatch")


if __name__ == "__main__":
    main()
