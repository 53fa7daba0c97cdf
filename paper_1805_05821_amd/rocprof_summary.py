"""Summaries of rocprofv3 output for the committed profiles.

  python -m paper_1805_05821_amd.rocprof_summary kernels DIR
      per-kernel statistics (from *kernel_stats.csv) plus the aggregate of the
      fused row-pass kernels (all k_pass instances).
  python -m paper_1805_05821_amd.rocprof_summary counter DIR COUNTER
      average value of COUNTER per dispatch for the row-pass kernels and for
      the copy kernel of a calibration run (from *counter_collection.csv).
"""

import csv
import glob
import os
import sys
from collections import defaultdict


def _find(d, suffix):
    hits = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return hits


def _col(row, *keys):
    for k in row:
        kl = k.lower().replace("_", "")
        for want in keys:
            if kl == want.lower().replace("_", ""):
                return row[k]
    raise KeyError(keys)


def is_row_pass(name):
    return "k_pass" in name


def kernel_stats(d):
    rows = []
    for f in _find(d, "kernel_stats.csv"):
        for r in csv.DictReader(open(f)):
            rows.append(dict(name=_col(r, "Name"), calls=int(_col(r, "Calls")),
                             total_ns=float(_col(r, "TotalDurationNs")), avg_ns=float(_col(r, "AverageNs"))))
    return rows


def summarize_kernels(d):
    rows = kernel_stats(d)
    rows.sort(key=lambda r: -r["total_ns"])
    tot = sum(r["total_ns"] for r in rows)
    lines = [f"{'calls':>7} {'total ms':>10} {'avg us':>10} {'share':>6}  kernel"]
    for r in rows[:25]:
        lines.append(f"{r['calls']:7d} {r['total_ns'] / 1e6:10.2f} {r['avg_ns'] / 1e3:10.2f} "
                     f"{100 * r['total_ns'] / tot:5.1f}%  {r['name'][:110]}")
    rp = [r for r in rows if is_row_pass(r["name"])]
    calls = sum(r["calls"] for r in rp)
    ns = sum(r["total_ns"] for r in rp)
    if calls:
        lines.append("")
        lines.append(f"row passes (all k_pass instances): {calls} launches, {ns / 1e6:.2f} ms total, "
                     f"average {ns / calls / 1e6:.4f} ms per launch, {100 * ns / tot:.1f}% of kernel time")
    return "\n".join(lines)


def counter_per_dispatch(d, counter):
    per = defaultdict(lambda: [0.0, set()])
    for f in _find(d, "counter_collection.csv"):
        for r in csv.DictReader(open(f)):
            if _col(r, "Counter_Name") != counter:
                continue
            name = _col(r, "Kernel_Name")
            disp = _col(r, "Dispatch_Id")
            per[name][0] += float(_col(r, "Counter_Value"))
            per[name][1].add(disp)
    out = {}
    for name, (v, ds) in per.items():
        out[name] = (v, len(ds))
    return out


def summarize_counter(d, counter):
    per = counter_per_dispatch(d, counter)
    lines = [f"{counter}: value per dispatch (as reported by rocprofv3)"]
    rp_v = rp_n = 0
    for name, (v, n) in sorted(per.items(), key=lambda kv: -kv[1][0]):
        lines.append(f"{n:7d} dispatches {v / max(n, 1):16.1f} per dispatch  {name[:100]}")
        if is_row_pass(name):
            rp_v += v
            rp_n += n
    if rp_n:
        lines.append(f"row passes: {rp_n} dispatches, {rp_v / rp_n:.1f} per dispatch")
    return "\n".join(lines)


def main(argv):
    if len(argv) >= 2 and argv[0] == "kernels":
        print(summarize_kernels(argv[1]))
    elif len(argv) >= 3 and argv[0] == "counter":
        print(summarize_counter(argv[1], argv[2]))
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
