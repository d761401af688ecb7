"""Summaries of rocprofv3 output for the roofline report (measurement only).

  python -m paper_2509_15948_amd.profiling stats DIR CMD...
      markdown table of a `--kernel-trace --stats --output-format csv` run
  python -m paper_2509_15948_amd.profiling counters DIR CMD...
      markdown table of a `--pmc` run: every counter per dispatch, by kernel
      (demangled name without its argument list) and grid, largest first
  python -m paper_2509_15948_amd.profiling traffic FETCH_DIR WRITE_DIR OUT_DIR WORKLOAD CMD...
      HBM bytes per launch of every kernel class from two `--pmc` runs
      (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by what the
      same counter reads for the calibration copy that bench.py --pmc-run
      performs first (a device-to-device copy of CALIB_BYTES)

The kernel classes are those of mg_profile_enable; the traffic records carry
the sha256 of the kernel sources they were taken on, so bench.py reports them
only while the kernels are unchanged.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CALIB_BYTES = 256 << 20

# kernel name patterns of each class (demangled names as rocprofv3 prints them)
CLASSES = {
    "conv_cols": r"mg::k_cols<",
    "conv_rows": r"mg::k_rows_(spec|conv|bwd|firspec)<",
    "conv_icols": r"mg::k_icols<",
    "eq_conv": r"mg::k_eq_(fwd|bwd)\b",
    "eq_spec": r"mg::k_eq_spec\b",
    "dyn": r"mg::k_dyn_",
    "pointwise": r"mg::k_(pointwise_|pw_chain_)",
    "sum": r"mg::k_sum\b",
    "loss": r"mg::k_loss_",
    "reverb_fir": r"mg::k_rv_",
    "fir": r"mg::k_(eq_synth|eq_adjoint|delay_synth|delay_adjoint)\b",
}


def kernel_sources():
    d = os.path.join(ROOT, "paper_2509_15948_amd", "csrc")
    return sorted(os.path.relpath(p, ROOT) for p in glob.glob(os.path.join(d, "*.hip")) + glob.glob(os.path.join(d, "*.h")))


def sources_sha256(files):
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()


def _find(dirpath, suffix):
    hits = glob.glob(os.path.join(dirpath, "**", f"*{suffix}"), recursive=True)
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {dirpath}")
    return hits[0]


def stats_markdown(dirpath, command):
    path = _find(dirpath, "kernel_stats.csv")
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    out = ["Command: `" + command + "`", "",
           "| total ms | share | calls | avg us | kernel |", "|---:|---:|---:|---:|---|"]
    for r in rows[:30]:
        t = float(r["TotalDurationNs"])
        name = r["Name"].replace("|", "/")
        if len(name) > 90:
            name = name[:87] + "..."
        out.append(f"| {t / 1e6:.3f} | {100 * t / total:.1f}% | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"`{name}` |")
    return "\n".join(out) + "\n"


def counters_markdown(dirpath, command, top=16):
    """Per-dispatch averages of every counter of one --pmc run, by kernel and
    grid (dispatches of the same kernel and grid are averaged)."""
    path = _find(dirpath, "counter_collection.csv")
    acc, disp = {}, {}
    for r in csv.DictReader(open(path)):
        name = re.sub(r"\(.*", "", r["Kernel_Name"]).replace("void ", "").replace("mg::", "")
        key = (name, r["Grid_Size"])
        acc.setdefault(key, {})
        acc[key][r["Counter_Name"]] = acc[key].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        disp.setdefault(key, set()).add(r["Dispatch_Id"])
    names = sorted({c for v in acc.values() for c in v})
    keys = [k for k in acc if k[0].startswith("k_")]
    sort_by = "SQ_WAVE_CYCLES" if "SQ_WAVE_CYCLES" in names else names[0]
    keys.sort(key=lambda k: -acc[k].get(sort_by, 0.0) / len(disp[k]))
    out = ["Command: `" + command + "`", "", "Per dispatch (averaged over the dispatches of each kernel and grid):", "",
           "| kernel | grid | dispatches | " + " | ".join(names) + " |",
           "|---|---:|---:|" + "---:|" * len(names)]
    for k in keys[:top]:
        n = len(disp[k])
        out.append(f"| `{k[0]}` | {k[1]} | {n} | " + " | ".join(f"{acc[k].get(c, 0.0) / n:.3g}" for c in names) + " |")
    return "\n".join(out) + "\n"


def class_markdown(dirpath):
    """Average duration per kernel class over every dispatch of the trace
    (the classes of mg_profile_enable; bench.py times the same classes)."""
    rows = list(csv.DictReader(open(_find(dirpath, "kernel_trace.csv"))))
    out = ["| class | dispatches | avg us |", "|---|---:|---:|"]
    for cls, pat in CLASSES.items():
        rx = re.compile(pat)
        d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in rows if rx.search(r["Kernel_Name"])]
        if d:
            out.append(f"| {cls} | {len(d)} | {sum(d) / len(d):.1f} |")
    return "\n".join(out) + "\n"


def _counter_rows(dirpath):
    path = _find(dirpath, "counter_collection.csv")
    return list(csv.DictReader(open(path)))


def _per_dispatch(rows, counter):
    """dispatch id -> (kernel name, counter value summed over its dimensions)"""
    acc = {}
    for r in rows:
        if r.get("Counter_Name") != counter:
            continue
        d = r.get("Dispatch_Id") or r.get("Correlation_Id")
        name = r.get("Kernel_Name", "")
        v = float(r["Counter_Value"])
        if d in acc:
            acc[d] = (name, acc[d][1] + v)
        else:
            acc[d] = (name, v)
    return acc


def traffic_records(fetch_dir, write_dir, command):
    fetch = _per_dispatch(_counter_rows(fetch_dir), "FETCH_SIZE")
    write = _per_dispatch(_counter_rows(write_dir), "WRITE_SIZE")

    def calib(acc):
        # the calibration copy is the largest dispatch that is not ours: it
        # reads and writes CALIB_BYTES (its source fill writes as much)
        best = max(((v, n) for (n, v) in acc.values() if "mg::" not in n), default=None)
        if best is None:
            raise RuntimeError("calibration copy not found")
        return best[0] * 1024.0 / CALIB_BYTES, best[1]

    fr, fname = calib(fetch)
    wr, _ = calib(write)
    files = kernel_sources()
    sha = sources_sha256(files)
    out = {}
    for cls, pat in CLASSES.items():
        rx = re.compile(pat)
        f = [v for (n, v) in fetch.values() if rx.search(n)]
        w = [v for (n, v) in write.values() if rx.search(n)]
        if not f or not w:
            continue
        fb = sum(f) / len(f) * 1024.0 / fr
        wb = sum(w) / len(w) * 1024.0 / wr
        out[cls] = {"class": cls, "bytes_per_launch": round(fb + wb), "fetch_bytes_per_launch": round(fb),
                    "write_bytes_per_launch": round(wb), "launches": len(f),
                    "calibration": {"kernel": fname[:80], "bytes": CALIB_BYTES, "fetch_factor": round(fr, 4),
                                    "write_factor": round(wr, 4)},
                    "command": command, "sources": files, "sources_sha256": sha}
    return out


def traffic_markdown(recs, workload):
    any_rec = next(iter(recs.values()))
    cal = any_rec["calibration"]
    out = [f"# HBM traffic per launch by kernel class: {workload} console", "",
           "Two runs, one counter each (FETCH_SIZE, then WRITE_SIZE):", "",
           "`" + any_rec["command"] + "`", "",
           f"Calibration: a device copy of {cal['bytes']} bytes (`{cal['kernel']}`) reads as {cal['fetch_factor']} x "
           f"its size in FETCH_SIZE and {cal['write_factor']} x in WRITE_SIZE; the counters are divided by these "
           "factors.  The run covers target rendering, loss setup, one warm-up step and two steps.", "",
           "| class | launches | fetch MB/launch | write MB/launch | total MB/launch |", "|---|---:|---:|---:|---:|"]
    for cls in sorted(recs):
        r = recs[cls]
        out.append(f"| {cls} | {r['launches']} | {r['fetch_bytes_per_launch'] / 1e6:.1f} | "
                   f"{r['write_bytes_per_launch'] / 1e6:.1f} | {r['bytes_per_launch'] / 1e6:.1f} |")
    return "\n".join(out) + "\n"


def main(argv):
    if argv[0] == "stats":
        sys.stdout.write(stats_markdown(argv[1], " ".join(argv[2:])))
        sys.stdout.write("\nBy kernel class:\n\n" + class_markdown(argv[1]))
    elif argv[0] == "counters":
        sys.stdout.write(counters_markdown(argv[1], " ".join(argv[2:])))
    elif argv[0] == "traffic":
        # argv: traffic FETCH_DIR WRITE_DIR OUT_DIR WORKLOAD CMD...
        recs = traffic_records(argv[1], argv[2], " ".join(argv[5:]))
        os.makedirs(argv[3], exist_ok=True)
        for cls, rec in recs.items():
            rec["workload"] = argv[4]
            json.dump(rec, open(os.path.join(argv[3], f"{cls}_{argv[4]}_console_traffic.json"), "w"), indent=1)
            print(cls, rec["bytes_per_launch"], "bytes per launch over", rec["launches"], "launches")
        with open(os.path.join(argv[3], f"console_{argv[4]}_traffic.md"), "w") as f:
            f.write(traffic_markdown(recs, argv[4]))
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
