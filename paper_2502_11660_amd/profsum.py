"""Summaries of rocprofv3 CSV output for this library's kernels.

  python -m paper_2502_11660_amd.profsum stats KERNEL_STATS_CSV
      markdown table: kernel, calls, total ms, average us, share of time
  python -m paper_2502_11660_amd.profsum traffic --fetch CSV --write CSV
          --calib-fetch CSV --calib-write CSV --copy-bytes N --kernel NAME
          [--entries E]
      HBM bytes per launch of one kernel from FETCH_SIZE / WRITE_SIZE counter
      runs (KiB per dispatch), each scaled by the factor that maps the same
      counter on the copy microbenchmark (k_mb_copy, N bytes read and N bytes
      written per launch) onto its known size; prints JSON, including a
      SHA-256 of the accumulation kernel's sources so that a reader can tell
      whether the counters still describe the current kernel, and with
      --entries the bytes per digit entry of the profiled launches.
  python -m paper_2502_11660_amd.profsum valu CSV [--kernel NAME ...]
      VALU counters per dispatch of the named kernels (averaged over their
      dispatches): instructions issued (SQ_INSTS_VALU and its 32/64-bit
      integer parts), SQ_ACTIVE_INST_VALU, GRBM_GUI_ACTIVE summed over the
      XCDs and the dispatch time, hence the mean engine clock and the share
      of SIMD cycles that issue VALU work (4 cycles per wave64 instruction).
  python -m paper_2502_11660_amd.profsum clusters KERNEL_TRACE_CSV [--gap-ms G]
      the kernel dispatches of a trace grouped into clusters separated by idle
      gaps longer than G ms; per cluster the dispatch count, the wall time
      from its first start to its last end, the union of the intervals in
      which at least one kernel runs (busy), the sum of the kernel durations
      and their ratio to busy (above 1 where kernels of several streams
      overlap).
"""

import argparse
import csv
import hashlib
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ACCUM_SOURCES = ["paper_2502_11660_amd/csrc/k_accum.hip", "paper_2502_11660_amd/csrc/curve.hpp",
                 "paper_2502_11660_amd/csrc/field.hpp", "paper_2502_11660_amd/csrc/fe28.hpp",
                 "paper_2502_11660_amd/csrc/curve28.hpp"]


def short_name(name):
    s = name.replace("msm::(anonymous namespace)::", "").replace("(anonymous namespace)::", "")
    s = re.sub(r"\(.*", "", s)
    return re.sub(r"^void ", "", s)


def sources_sha256(paths=ACCUM_SOURCES):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def stats_table(path):
    rows = list(csv.DictReader(open(path)))
    out = ["| kernel | calls | total ms | avg us | % |", "|---|---|---|---|---|"]
    for r in rows:
        name = short_name(r.get("Name") or r.get("KernelName"))
        out.append("| %s | %d | %.3f | %.1f | %.1f |" % (
            name[:60], int(r["Calls"]), float(r["TotalDurationNs"]) / 1e6,
            float(r["AverageNs"]) / 1e3, float(r["Percentage"])))
    return "\n".join(out)


def counter_per_dispatch(path, kernel, counter):
    """The counter's value per dispatch of the kernel, for the dispatches of
    its largest grid (smaller launches of the same kernel in the profiled
    program, such as a small MSM before the measured one, are left out)."""
    per = {}
    grid = {}
    for r in csv.DictReader(open(path)):
        if short_name(r["Kernel_Name"]) == kernel and r["Counter_Name"] == counter:
            d = r["Dispatch_Id"]
            per[d] = per.get(d, 0.0) + float(r["Counter_Value"])
            grid[d] = int(r.get("Grid_Size") or 0)
    if not per:
        raise SystemExit("no %s samples of %s in %s" % (counter, kernel, path))
    top = max(grid.values())
    return [v for d, v in per.items() if grid[d] == top]


def traffic(args):
    """HBM bytes per launch of one kernel, or summed over several kernels
    (one launch each, e.g. the kernels of one phase)."""
    kib = 1024.0
    cf = counter_per_dispatch(args.calib_fetch, "k_mb_copy", "FETCH_SIZE")
    cw = counter_per_dispatch(args.calib_write, "k_mb_copy", "WRITE_SIZE")
    f_fac = args.copy_bytes / (sum(cf) / len(cf) * kib)
    w_fac = args.copy_bytes / (sum(cw) / len(cw) * kib)
    fetch = write = 0.0
    launches = []
    for k in args.kernel:
        kf = counter_per_dispatch(args.fetch, k, "FETCH_SIZE")
        kw = counter_per_dispatch(args.write, k, "WRITE_SIZE")
        fetch += sum(kf) / len(kf) * kib * f_fac
        write += sum(kw) / len(kw) * kib * w_fac
        launches.append([len(kf), len(kw)])
    sources = ACCUM_SOURCES if args.kernel == ["k_accum"] else args.sources
    return {
        "kernel": args.kernel[0] if len(args.kernel) == 1 else args.kernel,
        "fetch_bytes_per_launch": fetch,
        "write_bytes_per_launch": write,
        "bytes_per_launch": fetch + write,
        "launches": launches[0] if len(launches) == 1 else launches,
        "copy_calibration": {"bytes_each_way": args.copy_bytes, "fetch_factor": f_fac,
                             "write_factor": w_fac},
        "sources": sources,
        "sources_sha256": sources_sha256(sources),
    }


def valu(args, xcds=8, simds=1024):
    rows = list(csv.DictReader(open(args.csv)))
    out = {}
    for name in args.kernel:
        per = {}
        for r in rows:
            if short_name(r["Kernel_Name"]) != name:
                continue
            d = per.setdefault(r["Dispatch_Id"], {"ns": int(r["End_Timestamp"]) - int(r["Start_Timestamp"])})
            d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        if not per:
            raise SystemExit("no dispatches of %s in %s" % (name, args.csv))
        big = max(per.values(), key=lambda d: d.get("SQ_INSTS_VALU", 0.0))
        keep = [d for d in per.values() if d.get("SQ_INSTS_VALU", 0.0) >= 0.5 * big.get("SQ_INSTS_VALU", 0.0)]
        avg = {k: sum(d[k] for d in keep) / len(keep) for k in keep[0]}
        cyc = avg.get("GRBM_GUI_ACTIVE", 0.0) / xcds
        ent = {"dispatches": len(keep), "ns": avg["ns"]}
        ent.update({k: avg[k] for k in sorted(avg) if k != "ns"})
        if cyc:
            ent["engine_clock_GHz"] = cyc / avg["ns"]
            if "SQ_INSTS_VALU" in avg:
                ent["valu_issue_share"] = 4.0 * avg["SQ_INSTS_VALU"] / (simds * cyc)
        out[name] = ent
    return out


def clusters(path, gap_ms):
    rows = [(int(r["Start_Timestamp"]), int(r["End_Timestamp"]), short_name(r["Kernel_Name"]))
            for r in csv.DictReader(open(path))]
    rows.sort()
    groups, cur, end = [], [], None
    for s_ns, e_ns, name in rows:
        if cur and s_ns - end > gap_ms * 1e6:
            groups.append(cur)
            cur = []
        cur.append((s_ns, e_ns, name))
        end = e_ns if end is None or not cur[:-1] else max(end, e_ns)
    if cur:
        groups.append(cur)
    out = []
    for g in groups:
        busy, run_s, run_e = 0, None, None
        for s_ns, e_ns, _ in g:
            if run_e is None or s_ns > run_e:
                if run_e is not None:
                    busy += run_e - run_s
                run_s, run_e = s_ns, e_ns
            else:
                run_e = max(run_e, e_ns)
        busy += run_e - run_s
        total = sum(e - s for s, e, _ in g)
        wall = max(e for _, e, _ in g) - g[0][0]
        out.append({"dispatches": len(g), "wall_ms": wall / 1e6, "busy_ms": busy / 1e6,
                    "busy_share": busy / wall if wall else 1.0,
                    "kernel_sum_ms": total / 1e6, "overlap": total / busy if busy else 1.0})
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(prog="profsum")
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    t = sub.add_parser("traffic")
    for k in ("fetch", "write", "calib_fetch", "calib_write"):
        t.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--kernel", action="append", default=None,
                   help="kernel (repeat to sum several); default k_accum")
    t.add_argument("--sources", nargs="*", default=[],
                   help="source files the figure describes (default: the accumulation kernel's)")
    t.add_argument("--entries", type=float, default=0.0,
                   help="digit entries per profiled launch (adds bytes per entry)")
    v = sub.add_parser("valu")
    v.add_argument("csv")
    v.add_argument("--kernel", action="append", required=True)
    c = sub.add_parser("clusters")
    c.add_argument("csv")
    c.add_argument("--gap-ms", type=float, default=5.0)
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        print(stats_table(a.csv))
    elif a.cmd == "clusters":
        print(json.dumps(clusters(a.csv, a.gap_ms), indent=1))
    elif a.cmd == "valu":
        print(json.dumps(valu(a), indent=1))
    else:
        a.kernel = a.kernel or ["k_accum"]
        rec = traffic(a)
        if a.entries:
            rec["entries_per_launch"] = a.entries
            rec["bytes_per_entry"] = rec["bytes_per_launch"] / a.entries
        print(json.dumps(rec, indent=1))


if __name__ == "__main__":
    sys.exit(main())
