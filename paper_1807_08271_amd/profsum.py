"""Summarises rocprofv3 output of a bench run into the short text record
kept with the sources: per-kernel launch statistics (--kernel-trace --stats)
and per-dispatch counters (--pmc passes), the HBM counters scaled by what
the same counters read for a plain copy of known size.

    python -m paper_1807_08271_amd.profsum --stats kernel_stats.csv \\
        [--trace kernel_trace.csv] \\
        --pmc pmc1.csv pmc2.csv ... --copy cpy1.csv cpy2.csv ... \\
        --copy-bytes 1073741824 --cmd "<profiled command>" --workload "<text>" \\
        --out profiles/<name>.md

The fenced JSON block at the end of the output is what bench.py reads.
"""
from __future__ import annotations

import argparse
import collections
import csv
import json
import re

from .build import source_sha


def kernel_key(name: str):
    """('reduce', level) for k_reduce<F16, LOG2B, FUSED> etc. under the
    full-resolution warp (LOG2B = level); (name, None) otherwise."""
    m = re.search(r"\bk_(\w+?)(<([^>]*)>)?\(", name)
    if not m:
        return None
    k = m.group(1)
    args = [a.strip() for a in (m.group(3) or "").split(",")]
    lvl = int(args[1]) if k in ("reduce", "warp") and len(args) > 1 else None
    return k, lvl, (m.group(3) or "")


def load_pmc(path, keep):
    rows = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in csv.DictReader(open(path)):
        if not keep(r["Kernel_Name"]):
            continue
        rows[(r["Kernel_Name"], int(r["Grid_Size"]))][r["Counter_Name"]].append(
            float(r["Counter_Value"]))
    return rows


def load_trace(path):
    """Durations (us) per (kernel name, grid size) from a --kernel-trace CSV."""
    out = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if "Grid_Size" in r and r["Grid_Size"]:
            grid = int(r["Grid_Size"])
        else:
            grid = (int(r.get("Grid_Size_X") or 1) * int(r.get("Grid_Size_Y") or 1) *
                    int(r.get("Grid_Size_Z") or 1))
        out[(r["Kernel_Name"], grid)].append(
            (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--stats", required=True)
    ap.add_argument("--trace", default=None, help="kernel_trace.csv of the same run")
    ap.add_argument("--pmc", nargs="*", default=[])
    ap.add_argument("--copy", nargs="*", default=[])
    ap.add_argument("--copy-bytes", type=int, default=1 << 30)
    ap.add_argument("--cmd", required=True)
    ap.add_argument("--workload", required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--tune", default=None,
                    help="the launch-shape file passed to the profiled command (--tune-file): "
                         "its lines are recorded, so the command can be repeated")
    ap.add_argument("--roof-bytes", nargs="*", default=[], metavar="KERNEL=BYTES",
                    help="algorithmic bytes per launch of named kernels: adds a table of their "
                         "achieved GB/s against the 8 TB/s HBM roof")
    a = ap.parse_args(argv)

    lines = ["# rocprofv3: %s" % a.workload, "", "Command (from the repository root):", "",
             "```", a.cmd, "```", ""]
    if a.tune:
        lines += ["Launch shapes (the tune file; per batch shape: fused, waves, tiles per wave, "
                  "XCD remap, warp passes):", "", "```"]
        lines += [ln.rstrip("\n") for ln in open(a.tune) if ln.strip()]
        lines += ["```", ""]
    lines += ["## Kernel trace (`--kernel-trace --stats`), library kernels", "",
             "| kernel | template args | calls | average us | total ms |", "|---|---|---|---|---|"]
    for r in csv.DictReader(open(a.stats)):
        kk = kernel_key(r["Name"])
        if not kk or "rgbid" not in r["Name"]:
            continue
        lines.append("| k_%s | %s | %s | %.2f | %.3f |" % (kk[0], kk[2], r["Calls"],
                                                           float(r["AverageNs"]) / 1e3,
                                                           float(r["TotalDurationNs"]) / 1e6))
    if a.roof_bytes:
        want = {k: float(v) for k, v in (e.split("=", 1) for e in a.roof_bytes)}
        avg = {}
        for r in csv.DictReader(open(a.stats)):
            kk = kernel_key(r["Name"])
            if kk and "rgbid" in r["Name"] and ("k_" + kk[0]) in want:
                avg[("k_" + kk[0])] = float(r["AverageNs"]) / 1e3
        lines += ["", "## Against the HBM roof (8 TB/s): algorithmic bytes per launch / average "
                  "duration", "", "| kernel | bytes per launch | average us | GB/s | fraction |",
                  "|---|---|---|---|---|"]
        for k, b in want.items():
            if k in avg:
                gbs = b / (avg[k] * 1e-6) / 1e9
                lines.append("| %s | %.0f | %.2f | %.1f | %.4f |" % (k, b, avg[k], gbs, gbs / 8000.0))
    trace = {}
    if a.trace:
        lines += ["", "## Kernel trace per launch shape (`--kernel-trace`), library kernels", "",
                  "| kernel | template args | grid | calls | average us |", "|---|---|---|---|---|"]
        for (name, grid), d in sorted(load_trace(a.trace).items(),
                                      key=lambda x: (kernel_key(x[0][0]) or ("",))[0:1] + (x[0][1],)):
            kk = kernel_key(name)
            if not kk or "rgbid" not in name:
                continue
            avg = sum(d) / len(d)
            trace[(kk[0], kk[1], kk[2], grid)] = (avg, len(d))
            lines.append("| k_%s | %s | %d | %d | %.2f |" % (kk[0], kk[2], grid, len(d), avg))
    # copy calibration: counters of the copy kernel against the known bytes
    cal = {}
    for path in a.copy:
        for (_, _), d in load_pmc(path, lambda n: "copyBuffer" in n).items():
            for c, v in d.items():
                cal.setdefault(c, []).extend(v)
    factors = {}
    kib = a.copy_bytes / 1024.0
    if cal.get("FETCH_SIZE"):
        factors["FETCH_SIZE"] = kib / max(cal["FETCH_SIZE"])
    if cal.get("WRITE_SIZE"):
        factors["WRITE_SIZE"] = kib / max(cal["WRITE_SIZE"])
    per = collections.defaultdict(dict)
    for path in a.pmc:
        for (name, grid), d in load_pmc(path, lambda n: "rgbid" in n).items():
            kk = kernel_key(name)
            if not kk:
                continue
            for c, v in d.items():
                per[(kk[0], kk[1], kk[2], grid)][c] = (sum(v) / len(v), len(v))
    if not a.pmc:
        # a kernel trace only: no counter section, and nothing for bench.py
        with open(a.out, "w") as fh:
            fh.write("\n".join(lines + [""]))
        print("wrote", a.out)
        return
    lines += ["", "## Counters per dispatch (`--pmc`, one counter group per run)", "",
              "Copy calibration: a copy of %d bytes reads FETCH_SIZE %s KiB and WRITE_SIZE %s KiB "
              "per dispatch; scale factors FETCH %.3f, WRITE %.3f." % (
                  a.copy_bytes, "%.0f" % max(cal.get("FETCH_SIZE", [0])),
                  "%.0f" % max(cal.get("WRITE_SIZE", [0])), factors.get("FETCH_SIZE", 0),
                  factors.get("WRITE_SIZE", 0)), "",
              "| kernel | args | grid | dispatches | FETCH KiB | WRITE KiB | HBM MB (scaled) | "
              "SQ_INSTS_VALU | SQ_WAVES |", "|---|---|---|---|---|---|---|---|---|"]
    kernels = {}
    for (k, lvl, targs, grid), d in sorted(per.items(), key=lambda x: (x[0][0], x[0][1] or 0, x[0][3])):
        f = d.get("FETCH_SIZE", (0, 0))[0]
        w = d.get("WRITE_SIZE", (0, 0))[0]
        hbm = (f * factors.get("FETCH_SIZE", 1.0) + w * factors.get("WRITE_SIZE", 1.0)) * 1024.0
        valu = d.get("SQ_INSTS_VALU", (0, 0))[0]
        lines.append("| k_%s | %s | %d | %d | %.1f | %.1f | %.2f | %.0f | %.0f |" % (
            k, targs, grid, d.get("FETCH_SIZE", (0, 0))[1], f, w, hbm / 1e6, valu,
            d.get("SQ_WAVES", (0, 0))[0]))
        if lvl is not None:
            key = "%s_l%d" % (k, lvl)
            # keep the largest dispatch (the whole batch in one launch)
            if key not in kernels or grid > kernels[key]["grid"]:
                kernels[key] = {"grid": grid, "hbm_bytes_per_launch": round(hbm),
                                "fetch_kib": round(f, 1), "write_kib": round(w, 1),
                                "valu_insts_per_launch": round(valu), "template_args": targs}
                if (k, lvl, targs, grid) in trace:
                    kernels[key]["trace_avg_us"] = round(trace[(k, lvl, targs, grid)][0], 2)
                    kernels[key]["trace_calls"] = trace[(k, lvl, targs, grid)][1]
    blob = {"source_sha": source_sha(), "fetch_factor": round(factors.get("FETCH_SIZE", 0), 4),
            "write_factor": round(factors.get("WRITE_SIZE", 0), 4), "kernels": kernels}
    lines += ["", "Machine-readable (read by bench.py; valid only while the kernel sources "
              "hash to source_sha):", "", "```json", json.dumps(blob, indent=1), "```", ""]
    with open(a.out, "w") as fh:
        fh.write("\n".join(lines))
    print("wrote", a.out)


if __name__ == "__main__":
    main()
