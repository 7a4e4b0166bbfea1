"""Summaries of rocprofv3 output as short Markdown files.

  stats:   python paper_1708_03621_amd/profile_summary.py stats KERNEL_STATS.csv --command "..." > out.md
  traffic: python paper_1708_03621_amd/profile_summary.py traffic --kernel NAME_PREFIX \
               --fetch FETCH.csv --write WRITE.csv --cal-fetch CAL_FETCH.csv --cal-write CAL_WRITE.csv \
               --cal-bytes BYTES --command "..." > out.md

The traffic summary scales the per-dispatch FETCH_SIZE and WRITE_SIZE (KiB)
of the kernel by the ratio of known bytes to the same counter's reading for a
plain device copy of known size, and records a hash of the kernel's source so
that a reader can tell whether the kernel changed since the counters were
taken (`kernel_source_hash`).
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import os
import statistics

HERE = os.path.dirname(os.path.abspath(__file__))


def xz_reg_source_hash() -> str:
    """Hash of the register x pass: its kernel text and the register FFT header."""
    src = open(os.path.join(HERE, "csrc", "fft.hip")).read()
    a = src.index("k_xz_reg(const FftItem*")
    b = src.index("// Register x pass lengths", a)
    h = hashlib.sha256(src[a:b].encode())
    h.update(open(os.path.join(HERE, "csrc", "fft_reg.h")).read().encode())
    h.update(open(os.path.join(HERE, "csrc", "fft_engine.h")).read().encode())
    return h.hexdigest()[:16]


def _counters(path):
    d = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        d[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return d


def _full_launch_avg(trace_csv):
    """Per kernel: mean duration (us) and count of the launches longer than
    half the kernel's median, i.e. without the launches masked to a few
    items (line-search retries), which return almost at once."""
    d = collections.defaultdict(list)
    for r in csv.DictReader(open(trace_csv)):
        d[r["Kernel_Name"]].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    out = {}
    for k, v in d.items():
        med = statistics.median(v)
        full = [x for x in v if x > 0.5 * med]
        out[k] = (statistics.mean(full), len(full))
    return out


def stats(args):
    rows = list(csv.DictReader(open(args.csv)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    trace = os.path.join(os.path.dirname(args.csv), os.path.basename(args.csv).replace("kernel_stats", "kernel_trace"))
    full = _full_launch_avg(trace) if os.path.exists(trace) else {}
    print(f"# Kernel statistics: {args.title}\n")
    print(f"Command: `{args.command}`\n")
    print(f"Total kernel time {tot / 1e6:.3f} ms. \"full\" = launches longer than half the kernel's median "
          f"(launches masked to a few items return almost at once).\n")
    print("| total ms | calls | avg us | avg us (full) | full calls | % | kernel |\n|---:|---:|---:|---:|---:|---:|---|")
    for r in rows[: args.top]:
        name = r["Name"].split("(")[0]
        fa, fc = full.get(r["Name"], (float("nan"), 0))
        print(f"| {float(r['TotalDurationNs']) / 1e6:.3f} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
              f"{fa:.2f} | {fc} | {float(r['Percentage']):.1f} | `{name}` |")


def traffic(args):
    f, w = _counters(args.fetch), _counters(args.write)
    cf, cw = _counters(args.cal_fetch), _counters(args.cal_write)
    cal = [k for k in cf if "copyBuffer" in k][0]
    kib = args.cal_bytes / 1024.0
    ffac = kib / statistics.mean(cf[cal])
    wfac = kib / statistics.mean(cw[cal])
    names = [k for k in f if k.startswith(args.kernel)]
    if not names:
        raise SystemExit(f"no kernel starting with {args.kernel}")
    k = names[0]
    # launches masked to a few items (line-search retries) move almost nothing:
    # the figure is the mean over full launches
    full_f = [v for v in f[k] if v > 0.05 * max(f[k])]
    full_w = [v for v in w[k] if v > 0.05 * max(w[k])]
    fk, wk = statistics.mean(full_f), statistics.mean(full_w)
    tb = fk * 1024 * ffac + wk * 1024 * wfac
    print(f"# HBM traffic: `{k.split('(')[0]}`\n")
    print(f"Command (two passes, FETCH_SIZE then WRITE_SIZE): `{args.command}`\n")
    print(f"Calibration: `{cal}` copying {args.cal_bytes} bytes reads FETCH_SIZE "
          f"{statistics.mean(cf[cal]):.1f} KiB and WRITE_SIZE {statistics.mean(cw[cal]):.1f} KiB per dispatch: "
          f"factors {ffac:.4f} (fetch) and {wfac:.4f} (write).\n")
    print(f"| dispatches (full / all) | FETCH_SIZE KiB | WRITE_SIZE KiB | scaled read bytes | scaled write bytes |\n"
          f"|---:|---:|---:|---:|---:|\n| {len(full_f)} / {len(f[k])} | {fk:.1f} | {wk:.1f} | {fk * 1024 * ffac:.4g} | "
          f"{wk * 1024 * wfac:.4g} |\n")
    print(f"traffic_bytes_per_launch: {tb:.6g}")
    print(f"kernel_source_hash: {xz_reg_source_hash()}")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--command", required=True)
    s.add_argument("--title", default="")
    s.add_argument("--top", type=int, default=30)
    t = sub.add_parser("traffic")
    t.add_argument("--kernel", required=True)
    for a in ("fetch", "write", "cal_fetch", "cal_write"):
        t.add_argument("--" + a.replace("_", "-"), dest=a, required=True)
    t.add_argument("--cal-bytes", type=float, required=True)
    t.add_argument("--command", required=True)
    args = ap.parse_args()
    (stats if args.cmd == "stats" else traffic)(args)


if __name__ == "__main__":
    main()
