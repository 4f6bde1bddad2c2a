"""Summaries of rocprofv3 CSV output, in the short text form kept under profiles/.

  python -m paper_2208_14703_amd.profsum stats <dir> [--top N] [--cmd "..."]
      Per-kernel calls, total and average duration from <dir>/*_kernel_stats.csv,
      plus the traced span and busy time from *_kernel_trace.csv.

  python -m paper_2208_14703_amd.profsum levels <dir> [--per NAME] [--top N] [--cmd "..."]
      Kernel time grouped by (kernel, grid size) from *_kernel_trace.csv, i.e. per
      level of the hierarchy; with --per, also per call of kernel NAME (for
      instance the once-per-V-cycle norm kernel: time per V-cycle).

  python -m paper_2208_14703_amd.profsum traffic --fetch <dir> --write <dir> --kernel NAME
          --copy NAME --copy-bytes B --cells N --bytes-per-cell K [--cmd "..."]
      Turns FETCH_SIZE and WRITE_SIZE (KiB per dispatch, from two separate
      --pmc runs) into bytes per launch of the kernel.  Each counter is scaled
      by the factor that makes it read the known size of a plain copy kernel
      run in the same process.  The bench reads `traffic_bytes_per_launch`,
      `cells` and `sources_sha256` from the output.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = ["m1_kernels.hip", "m1_cells.hpp", "m1_device.hpp", "m1_internal.hpp", "m1_mixed.hip", "m1_transfer.hip",
                  "m1_mixed.hpp", "m1_transfer.hpp", "m1_kernels3.hip", "m1_3d.hpp"]


def code_only(text: str) -> str:
    """C++ source without comments and whitespace (what the compiler sees of the kernels)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return re.sub(r"\s+", "", text)


def sources_hash(read=None) -> str:
    """Hash of the kernel sources' code (comments and layout excluded)."""
    h = hashlib.sha256()
    for s in KERNEL_SOURCES:
        path = os.path.join(ROOT, "paper_2208_14703_amd", "csrc", s)
        text = read(s) if read else open(path, encoding="utf-8").read()
        h.update(code_only(text).encode())
    return h.hexdigest()[:16]


def _one(d: str, suffix: str) -> str:
    fs = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not fs:
        sys.exit(f"no *{suffix} under {d}")
    return fs[-1]


def short(name: str) -> str:
    name = name.replace("void ", "")
    return name.split("(")[0]


def stats(d: str, top: int, cmd: str):
    rows = list(csv.DictReader(open(_one(d, "_kernel_stats.csv"))))
    tr = list(csv.DictReader(open(_one(d, "_kernel_trace.csv"))))
    span = (max(int(r["End_Timestamp"]) for r in tr) - min(int(r["Start_Timestamp"]) for r in tr)) * 1e-6
    busy = sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in tr) * 1e-6
    print(f"command: {cmd}")
    print(f"dispatches: {len(tr)}   traced span: {span:.2f} ms   kernel busy: {busy:.2f} ms")
    print(f"{'calls':>8} {'total ms':>10} {'avg us':>9} {'min us':>8} {'max us':>8} {'%':>6}  kernel")
    for r in rows[:top]:
        print(f"{int(r['Calls']):8d} {float(r['TotalDurationNs']) * 1e-6:10.2f} {float(r['AverageNs']) * 1e-3:9.2f} "
              f"{float(r['MinNs']) * 1e-3:8.2f} {float(r['MaxNs']) * 1e-3:8.2f} {float(r['Percentage']):6.2f}  "
              f"{short(r['Name'])}")


def levels(d: str, per: str, top: int, cmd: str):
    tr = list(csv.DictReader(open(_one(d, "_kernel_trace.csv"))))
    groups = collections.defaultdict(list)
    for r in tr:
        groups[(short(r["Kernel_Name"]), int(r["Grid_Size_X"]))].append(
            (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3)
    nper = sum(len(v) for (k, _), v in groups.items() if per and k.endswith(per)) if per else 0
    busy = sum(sum(v) for v in groups.values())
    print(f"command: {cmd}")
    head = f"kernel time by (kernel, grid threads); busy {busy * 1e-3:.2f} ms"
    if nper:
        head += f"; {nper} calls of {per}: {busy / nper:.2f} us per call"
    print(head)
    print(f"{'calls':>8} {'total ms':>10} {'avg us':>9} {'us/' + (per or '-'):>16} {'grid':>10}  kernel")
    out = sorted(groups.items(), key=lambda kv: -sum(kv[1]))
    for (name, grid), v in out[:top]:
        pc = f"{sum(v) / nper:16.2f}" if nper else f"{'':>16}"
        print(f"{len(v):8d} {sum(v) * 1e-3:10.2f} {sum(v) / len(v):9.2f} {pc} {grid:10d}  {name}")


def counter_per_dispatch(d: str, counter: str):
    """Average counter value per dispatch, keyed by short kernel name."""
    rows = list(csv.DictReader(open(_one(d, "_counter_collection.csv"))))
    per = collections.defaultdict(dict)
    for r in rows:
        if r["Counter_Name"] != counter:
            continue
        per[short(r["Kernel_Name"])][r["Dispatch_Id"]] = float(r["Counter_Value"])
    return {k: (sum(v.values()) / len(v), len(v)) for k, v in per.items()}


def pick(table: dict, name: str):
    hits = [k for k in table if name in k]
    if not hits:
        sys.exit(f"kernel {name!r} not in counters ({sorted(table)[:8]} ...)")
    return table[max(hits, key=lambda k: table[k][1])]


def traffic(a):
    fe = counter_per_dispatch(a.fetch, "FETCH_SIZE")
    wr = counter_per_dispatch(a.write, "WRITE_SIZE")
    kf, nkf = pick(fe, a.kernel)
    kw, nkw = pick(wr, a.kernel)
    cf, _ = pick(fe, a.copy)
    cw, _ = pick(wr, a.copy)
    half = a.copy_bytes / 2  # the copy reads and writes half of its bytes each
    sf, sw = half / (cf * 1024), half / (cw * 1024)
    fetch_b, write_b = kf * 1024 * sf, kw * 1024 * sw
    alg = a.cells * a.bytes_per_cell
    print(f"command (FETCH_SIZE run): {a.cmd_fetch}")
    print(f"command (WRITE_SIZE run): {a.cmd_write}")
    print(f"kernel: {a.kernel}")
    print(f"cells: {a.cells}")
    print(f"sources_sha256: {sources_hash()}")
    print(f"kernel FETCH_SIZE KiB per dispatch: {kf:.1f}   ({nkf} dispatches)")
    print(f"kernel WRITE_SIZE KiB per dispatch: {kw:.1f}   ({nkw} dispatches)")
    print(f"copy kernel ({a.copy}, {a.copy_bytes} B moved: half read, half written):")
    print(f"  FETCH_SIZE KiB {cf:.1f} -> scale {sf:.4f};  WRITE_SIZE KiB {cw:.1f} -> scale {sw:.4f}")
    print(f"fetch_bytes_per_launch: {fetch_b:.0f}")
    print(f"write_bytes_per_launch: {write_b:.0f}")
    print(f"traffic_bytes_per_launch: {fetch_b + write_b:.0f}")
    print(f"algorithmic_bytes_per_launch: {alg}")
    print(f"traffic / algorithmic: {(fetch_b + write_b) / alg:.3f}")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--top", type=int, default=25)
    s.add_argument("--cmd", default="")
    lv = sub.add_parser("levels")
    lv.add_argument("dir")
    lv.add_argument("--per", default="")
    lv.add_argument("--top", type=int, default=30)
    lv.add_argument("--cmd", default="")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--copy", required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--cells", type=int, required=True)
    t.add_argument("--bytes-per-cell", type=int, required=True)
    t.add_argument("--cmd-fetch", default="")
    t.add_argument("--cmd-write", default="")
    a = ap.parse_args()
    if a.what == "stats":
        stats(a.dir, a.top, a.cmd)
    elif a.what == "levels":
        levels(a.dir, a.per, a.top, a.cmd)
    else:
        traffic(a)


if __name__ == "__main__":
    main()
