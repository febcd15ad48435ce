"""Summaries of rocprofv3 CSV output for this library's kernels.

  python -m paper_2502_11660_amd.profsum stats KERNEL_STATS_CSV
      markdown table: kernel, calls, total ms, average us, share of time
  python -m paper_2502_11660_amd.profsum traffic --fetch CSV --write CSV
          --calib-fetch CSV --calib-write CSV --copy-bytes N --kernel NAME
      HBM bytes per launch of one kernel from FETCH_SIZE / WRITE_SIZE counter
      runs (KiB per dispatch), each scaled by the factor that maps the same
      counter on the copy microbenchmark (k_mb_copy, N bytes read and N bytes
      written per launch) onto its known size; prints JSON, including a
      SHA-256 of the accumulation kernel's sources so that a reader can tell
      whether the counters still describe the current kernel.
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
                 "paper_2502_11660_amd/csrc/field.hpp"]


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
    vals = []
    for r in csv.DictReader(open(path)):
        if short_name(r["Kernel_Name"]) == kernel and r["Counter_Name"] == counter:
            vals.append(float(r["Counter_Value"]))
    if not vals:
        raise SystemExit("no %s samples of %s in %s" % (counter, kernel, path))
    return vals


def traffic(args):
    kib = 1024.0
    cf = counter_per_dispatch(args.calib_fetch, "k_mb_copy", "FETCH_SIZE")
    cw = counter_per_dispatch(args.calib_write, "k_mb_copy", "WRITE_SIZE")
    f_fac = args.copy_bytes / (sum(cf) / len(cf) * kib)
    w_fac = args.copy_bytes / (sum(cw) / len(cw) * kib)
    kf = counter_per_dispatch(args.fetch, args.kernel, "FETCH_SIZE")
    kw = counter_per_dispatch(args.write, args.kernel, "WRITE_SIZE")
    fetch = sum(kf) / len(kf) * kib * f_fac
    write = sum(kw) / len(kw) * kib * w_fac
    return {
        "kernel": args.kernel,
        "fetch_bytes_per_launch": fetch,
        "write_bytes_per_launch": write,
        "bytes_per_launch": fetch + write,
        "launches": [len(kf), len(kw)],
        "copy_calibration": {"bytes_each_way": args.copy_bytes, "fetch_factor": f_fac,
                             "write_factor": w_fac},
        "sources": ACCUM_SOURCES,
        "sources_sha256": sources_sha256(),
    }


def main(argv=None):
    ap = argparse.ArgumentParser(prog="profsum")
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    t = sub.add_parser("traffic")
    for k in ("fetch", "write", "calib_fetch", "calib_write"):
        t.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--kernel", default="k_accum")
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        print(stats_table(a.csv))
    else:
        print(json.dumps(traffic(a), indent=1))


if __name__ == "__main__":
    sys.exit(main())
