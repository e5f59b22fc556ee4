"""Summaries of rocprofv3 output (CSV) for the profiles kept with the sources.

  python -m paper_1312_3062_amd.profiling trace RUN_kernel_trace.csv [--kernel REGEX --last N]
      per-kernel calls, average and total duration; with --kernel, the
      durations of its last N dispatches

  python -m paper_1312_3062_amd.profiling traffic --fetch FETCH.csv --write WRITE.csv \\
          --kernel REGEX --copy REGEX --copy-bytes B [--last N] [--per-launch M]
      HBM traffic of a kernel from two counter-collection runs (FETCH_SIZE,
      then WRITE_SIZE, KiB per dispatch).  Each counter is divided by what it
      reads for a copy-like kernel that moves a known B bytes in and B bytes
      out, which removes the counters' own scale.  Prints a markdown summary
      and one machine-readable line (an HTML comment) that bench.py reads.

  python -m paper_1312_3062_amd.profiling sq RUN_A.csv [RUN_B.csv] --kernel REGEX --last N --queries Q
      SQ counters of a kernel (averaged over its last N dispatches), per
      dispatch and per query, with the VALU / scalar / LDS busy shares.

The machine-readable line carries a hash of the search kernel's code
(comments aside): a figure taken on other code is not reported.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os
import re
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("csrc/search.hip", "csrc/common.hpp", "csrc/mseq.hpp")
TRAFFIC_TAG = "traffic-record"


def kernel_source_hash() -> str:
    """Hash of the search kernel's code: comments, indentation and blank
    lines are left out, so that only a change of the code itself retires a
    traffic record (the sources hold no string with `//` or `/*`)."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(PKG, rel), encoding="utf-8") as f:
            text = re.sub(r"/\*.*?\*/", "", f.read(), flags=re.S)
        code = [ln.split("//", 1)[0].strip() for ln in text.splitlines()]
        h.update(rel.encode() + b"\0" + "\n".join(c for c in code if c).encode())
    return h.hexdigest()[:16]


def short_name(name: str) -> str:
    m = re.search(r"(k_[A-Za-z0-9_]+)(<[^()]*>)?", name)
    if m:
        return m.group(1) + (m.group(2) or "")
    return name.split("(")[0].replace("void ", "")


def _rows(path: str):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def trace_table(path: str) -> str:
    rows = _rows(path)
    agg = collections.OrderedDict()
    for r in rows:
        k = short_name(r["Kernel_Name"])
        d = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        a = agg.setdefault(k, [0, 0, r.get("LDS_Block_Size", ""), r.get("VGPR_Count", ""),
                               r.get("Grid_Size_X", r.get("Grid_Size", "")), r.get("Workgroup_Size_X", "")])
        a[0] += 1
        a[1] += d
    tot = sum(v[1] for v in agg.values()) or 1
    out = ["| kernel | calls | avg ms | total ms | % | LDS B/WG | VGPR | grid x | WG |",
           "|---|---|---|---|---|---|---|---|---|"]
    for k, v in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        out.append(f"| `{k}` | {v[0]} | {v[1] / v[0] / 1e6:.3f} | {v[1] / 1e6:.1f} | {100 * v[1] / tot:.1f} | "
                   f"{v[2]} | {v[3]} | {v[4]} | {v[5]} |")
    return "\n".join(out)


def last_durations(path: str, kernel_re: str, last: int):
    rx = re.compile(kernel_re)
    rows = sorted(_rows(path), key=lambda r: int(r["Start_Timestamp"]))
    ds = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6 for r in rows
          if rx.search(short_name(r["Kernel_Name"]))]
    return ds[-last:]


def counter_values(path: str, counter: str, kernel_re: str):
    """Per-dispatch values (in dispatch order) of one counter for the kernels matching kernel_re."""
    rx = re.compile(kernel_re)
    by_dispatch = collections.OrderedDict()
    for r in _rows(path):
        if r.get("Counter_Name", counter) != counter:
            continue
        if not rx.search(short_name(r["Kernel_Name"])) and not rx.search(r["Kernel_Name"]):
            continue
        key = int(r.get("Dispatch_Id", len(by_dispatch)))
        by_dispatch[key] = by_dispatch.get(key, 0.0) + float(r["Counter_Value"])
    return [by_dispatch[k] for k in sorted(by_dispatch)]


def sq_table(csvs, kernel_re: str, last: int, queries: int) -> str:
    """SQ counters of a kernel's last `last` dispatches (averaged), per dispatch
    and per query.  Cycle counters of the SQ are in units of 4 cycles; the
    busy shares divide by the SIMDs' time (GRBM_GUI_ACTIVE per XCD x 32 CUs x
    4 SIMDs; the same for VALU and the scalar unit's issue slots)."""
    vals = {}
    for path in csvs:
        by = collections.OrderedDict()
        for r in _rows(path):
            if re.search(kernel_re, r["Kernel_Name"]):
                by.setdefault(int(r["Dispatch_Id"]), {})[r["Counter_Name"]] = float(r["Counter_Value"])
        for d in list(by)[-last:]:
            for k, v in by[d].items():
                vals.setdefault(k, []).append(v)
    avg = {k: sum(v) / len(v) for k, v in vals.items()}
    lines = ["| counter | per dispatch | per query |", "|---|---|---|"]
    for k in sorted(avg):
        lines.append(f"| {k} | {avg[k]:.4g} | {avg[k] / max(queries, 1):.4g} |")
    if "GRBM_GUI_ACTIVE" in avg:
        simd_quads = avg["GRBM_GUI_ACTIVE"] * 32 * 4 / 4.0  # per XCD cycles x SIMDs, in 4-cycle units
        for k in ("SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_SCA", "SQ_ACTIVE_INST_LDS", "SQ_INSTS_VALU", "SQ_INSTS_SALU"):
            if k in avg:
                lines.append(f"| {k} / SIMD time | {avg[k] / simd_quads:.3f} | |")
    if "SQ_WAVE_CYCLES" in avg:
        for k in ("SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_ANY"):
            if k in avg:
                lines.append(f"| {k} / SQ_WAVE_CYCLES | {avg[k] / avg['SQ_WAVE_CYCLES']:.3f} | |")
    return "\n".join(lines)


def traffic(fetch_csv: str, write_csv: str, kernel_re: str, copy_re: str, copy_bytes: int, last: int,
            per_launch: int = 1):
    kib = copy_bytes / 1024.0
    cf = counter_values(fetch_csv, "FETCH_SIZE", copy_re)
    cw = counter_values(write_csv, "WRITE_SIZE", copy_re)
    kf = counter_values(fetch_csv, "FETCH_SIZE", kernel_re)
    kw = counter_values(write_csv, "WRITE_SIZE", kernel_re)
    if not (cf and cw and kf and kw):
        raise SystemExit(f"missing dispatches: copy fetch {len(cf)} write {len(cw)}, kernel fetch {len(kf)} "
                         f"write {len(kw)}")
    f_scale = (sum(cf) / len(cf)) / kib
    w_scale = (sum(cw) / len(cw)) / kib
    kf, kw = kf[-last:], kw[-last:]
    # a launch may be several dispatches of the kernel (one per budget class)
    fetch_b = sum(kf) / len(kf) * per_launch / f_scale * 1024.0
    write_b = sum(kw) / len(kw) * per_launch / w_scale * 1024.0
    return {"fetch_bytes": fetch_b, "write_bytes": write_b, "bytes_per_launch": fetch_b + write_b,
            "fetch_scale": f_scale, "write_scale": w_scale, "copy_dispatches": [len(cf), len(cw)],
            "kernel_dispatches": [len(kf), len(kw)],
            "raw_kib": {"kernel_fetch": sum(kf) / len(kf), "kernel_write": sum(kw) / len(kw),
                        "copy_fetch": sum(cf) / len(cf), "copy_write": sum(cw) / len(cw)}}


def read_traffic_record(md_path: str):
    """The record a traffic summary carries, or None if absent or taken on other kernel sources."""
    try:
        text = open(md_path).read()
    except OSError:
        return None
    m = re.search(r"<!-- " + TRAFFIC_TAG + r" (\{.*?\}) -->", text)
    if not m:
        return None
    rec = json.loads(m.group(1))
    return rec if rec.get("kernel_sources") == kernel_source_hash() else None


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("csv")
    t.add_argument("--kernel", default="")
    t.add_argument("--last", type=int, default=6)
    c = sub.add_parser("traffic")
    c.add_argument("--fetch", required=True)
    c.add_argument("--write", required=True)
    c.add_argument("--kernel", required=True)
    c.add_argument("--copy", required=True)
    c.add_argument("--copy-bytes", type=int, required=True)
    c.add_argument("--last", type=int, default=1 << 30)
    c.add_argument("--algorithmic-bytes", type=float, default=0.0)
    c.add_argument("--workload", default="")
    c.add_argument("--per-launch", type=int, default=1, help="dispatches of the kernel per launch")
    q = sub.add_parser("sq")
    q.add_argument("csv", nargs="+")
    q.add_argument("--kernel", required=True)
    q.add_argument("--last", type=int, default=1)
    q.add_argument("--queries", type=int, default=1)
    a = ap.parse_args(argv)
    if a.cmd == "sq":
        print(sq_table(a.csv, a.kernel, a.last, a.queries))
        return
    if a.cmd == "trace":
        print(trace_table(a.csv))
        if a.kernel:
            ds = last_durations(a.csv, a.kernel, a.last)
            if ds:
                print(f"\nLast {len(ds)} `{a.kernel}` dispatches (ms): " + ", ".join(f"{d:.3f}" for d in ds) +
                      f" (mean {sum(ds) / len(ds):.3f} ms)")
        return
    r = traffic(a.fetch, a.write, a.kernel, a.copy, a.copy_bytes, a.last, a.per_launch)
    print(f"| quantity | value |\n|---|---|")
    print(f"| copy kernel: FETCH_SIZE / bytes read | {r['fetch_scale']:.4f} |")
    print(f"| copy kernel: WRITE_SIZE / bytes written | {r['write_scale']:.4f} |")
    print(f"| `{a.kernel}` FETCH_SIZE per dispatch (KiB, raw) | {r['raw_kib']['kernel_fetch']:.0f} |")
    print(f"| `{a.kernel}` WRITE_SIZE per dispatch (KiB, raw) | {r['raw_kib']['kernel_write']:.0f} |")
    print(f"| HBM bytes read per launch (scaled) | {r['fetch_bytes']:.4g} |")
    print(f"| HBM bytes written per launch (scaled) | {r['write_bytes']:.4g} |")
    print(f"| HBM bytes per launch | {r['bytes_per_launch']:.4g} |")
    if a.algorithmic_bytes:
        print(f"| algorithmic bytes per launch | {a.algorithmic_bytes:.4g} |")
        print(f"| traffic / algorithmic | {r['bytes_per_launch'] / a.algorithmic_bytes:.3f} |")
    rec = {"kernel": a.kernel, "workload": a.workload, "bytes_per_launch": round(r["bytes_per_launch"]),
           "fetch_bytes": round(r["fetch_bytes"]), "write_bytes": round(r["write_bytes"]),
           "kernel_sources": kernel_source_hash()}
    print(f"\n<!-- {TRAFFIC_TAG} {json.dumps(rec)} -->")


if __name__ == "__main__":
    main(sys.argv[1:])
