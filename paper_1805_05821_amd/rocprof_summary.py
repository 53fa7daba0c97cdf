"""Summaries of rocprofv3 output for the committed profiles.

  python -m paper_1805_05821_amd.rocprof_summary kernels DIR
      per-kernel statistics (from *kernel_stats.csv) plus the aggregate of the
      fused row-pass kernels (all k_pass instances).
  python -m paper_1805_05821_amd.rocprof_summary window DIR PREFIX START COUNT [MIN_US]
      average duration of the dispatches START .. START+COUNT-1 (time order)
      of the kernels whose name starts with PREFIX (from *kernel_trace.csv):
      picks one run out of a trace that holds several.  With MIN_US, the
      dispatches shorter than MIN_US microseconds (kernels whose gate was
      closed, which return at once) are counted apart and left out of the
      average.
  python -m paper_1805_05821_amd.rocprof_summary counter DIR COUNTER
      average value of COUNTER per dispatch for the row-pass kernels and for
      the copy kernel of a calibration run (from *counter_collection.csv).
  python -m paper_1805_05821_amd.rocprof_summary traffic FETCH_DIR WRITE_DIR \
         FETCH_COPY_DIR WRITE_COPY_DIR COPY_BYTES BENCH_LOG OUT_JSON
      HBM bytes per row-pass launch: FETCH_SIZE and WRITE_SIZE (KiB per
      dispatch), each scaled by bytes-moved / counter-value of the plain copy
      of COPY_BYTES bytes, next to the algorithmic bytes per launch that the
      benchmark printed in BENCH_LOG (its JSON line); written to OUT_JSON with
      the SHA-256 of the kernel source it describes.
  python -m paper_1805_05821_amd.rocprof_summary batched FETCH_DIR WRITE_DIR \
         FETCH_SCALE WRITE_SCALE STEPS
      HBM bytes of the batched form's last timed run: FETCH_SIZE and
      WRITE_SIZE of every batched kernel dispatched from the STEPS-th last plan
      dispatch before the FP64-basis reference batch on, scaled by the
      calibration factors (bytes per counter unit), per kernel.
  python -m paper_1805_05821_amd.rocprof_summary kernel_traffic FETCH_DIR WRITE_DIR \
         FETCH_COPY_DIR WRITE_COPY_DIR COPY_BYTES NAME_PREFIX BENCH_LOG KEY
      the same per-launch HBM bytes for the kernels whose name starts with
      NAME_PREFIX, against the algorithmic bytes per launch that the
      benchmark's JSON line in BENCH_LOG holds under KEY.
  python -m paper_1805_05821_amd.rocprof_summary counter_window FETCH_DIR WRITE_DIR \
         FETCH_COPY_DIR WRITE_COPY_DIR COPY_BYTES PREFIX START COUNT
      HBM bytes per dispatch (FETCH_SIZE and WRITE_SIZE scaled by the copy
      calibration, as in kernel_traffic) averaged over the dispatches
      START .. START+COUNT-1, in dispatch order, of the kernels whose name
      starts with PREFIX: one kernel instance of one run in a counter pass
      over several.
  python -m paper_1805_05821_amd.rocprof_summary batched_run DIR OCCURRENCE STEPS
      per-kernel time of one batched run in a kernel trace: the STEPS plan
      dispatches (k_batch_plan) that precede the OCCURRENCE-th FP64-basis
      batch (the untimed reference batch bench.py builds after each timed
      batched leg, 1-based), with every dispatch from the first of them to
      the run's last finalize; also the span from the first dispatch's start
      to the last one's end.
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
    lines.append("")
    for label, key in (("all k_pass instances", "k_pass"), ("FP32 basis, k_pass<float, ...>", "k_pass<float"),
                       ("FP64 basis, k_pass<double, ...>", "k_pass<double")):
        rp = [r for r in rows if key in r["name"]]
        calls = sum(r["calls"] for r in rp)
        ns = sum(r["total_ns"] for r in rp)
        if calls:
            lines.append(f"row passes ({label}): {calls} launches, {ns / 1e6:.2f} ms total, "
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


def _copy_value(d, counter):
    per = counter_per_dispatch(d, counter)
    for name, (v, n) in per.items():
        if "copyBuffer" in name or "copy" in name.lower():
            return v / max(n, 1)
    raise RuntimeError(f"no copy kernel under {d}")


def _row_pass_avg(d, counter):
    """Average per launch of the FP32-basis row passes (the form the record describes)."""
    per = counter_per_dispatch(d, counter)
    sel = [(x, n) for name, (x, n) in per.items() if is_row_pass(name) and "k_pass<float" in name]
    return sum(x for x, _ in sel) / max(sum(n for _, n in sel), 1), sum(n for _, n in sel)


def _prefix_avg(d, counter, prefix):
    per = counter_per_dispatch(d, counter)
    v = sum(x for name, (x, n) in per.items() if name.startswith(prefix))
    n = sum(n for name, (x, n) in per.items() if name.startswith(prefix))
    return v / max(n, 1), n


def kernel_traffic(fetch_dir, write_dir, fetch_copy, write_copy, copy_bytes, prefix, bench_log, key):
    import json

    copy_bytes = float(copy_bytes)
    f_scale = copy_bytes / _copy_value(fetch_copy, "FETCH_SIZE")
    w_scale = copy_bytes / _copy_value(write_copy, "WRITE_SIZE")
    f_avg, nf = _prefix_avg(fetch_dir, "FETCH_SIZE", prefix)
    w_avg, nw = _prefix_avg(write_dir, "WRITE_SIZE", prefix)
    alg = None
    for line in open(bench_log):
        line = line.strip()
        if line.startswith("{") and f'"{key}"' in line:
            alg = json.loads(line)[key]
    fetch_b, write_b = f_avg * f_scale, w_avg * w_scale
    return {"kernels": prefix, "dispatches": [nf, nw], "fetch_bytes_per_launch": fetch_b,
            "write_bytes_per_launch": write_b, "traffic_bytes_per_launch": fetch_b + write_b,
            "alg_bytes_per_launch": alg, "traffic_over_alg": (fetch_b + write_b) / alg if alg else None,
            "fetch_scale": f_scale, "write_scale": w_scale}


def _prefix_window(d, counter, prefix, start, count):
    per = defaultdict(float)
    for f in _find(d, "counter_collection.csv"):
        for r in csv.DictReader(open(f)):
            if _col(r, "Counter_Name") == counter and _col(r, "Kernel_Name").startswith(prefix):
                per[int(_col(r, "Dispatch_Id"))] += float(_col(r, "Counter_Value"))
    ids = sorted(per)
    sel = ids[int(start):int(start) + int(count)]
    return sum(per[i] for i in sel) / max(len(sel), 1), len(sel), len(ids)


def counter_window(fetch_dir, write_dir, fetch_copy, write_copy, copy_bytes, prefix, start, count):
    copy_bytes = float(copy_bytes)
    f_scale = copy_bytes / _copy_value(fetch_copy, "FETCH_SIZE")
    w_scale = copy_bytes / _copy_value(write_copy, "WRITE_SIZE")
    f_avg, nf, tf = _prefix_window(fetch_dir, "FETCH_SIZE", prefix, start, count)
    w_avg, nw, tw = _prefix_window(write_dir, "WRITE_SIZE", prefix, start, count)
    return {"kernels": prefix, "window": [int(start), int(count)], "dispatches": [nf, nw],
            "of": [tf, tw], "fetch_bytes_per_launch": f_avg * f_scale, "write_bytes_per_launch": w_avg * w_scale,
            "traffic_bytes_per_launch": f_avg * f_scale + w_avg * w_scale,
            "fetch_scale": f_scale, "write_scale": w_scale}


ROW_PASS_SOURCES = ("foa_buffer.h", "foa_device.h", "foa_kernels.hip")


def row_pass_source_digest():
    """SHA-256 over the sources that define the single-stream row-pass
    kernels; a stored traffic measurement applies only while it matches."""
    import hashlib

    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    h = hashlib.sha256()
    for name in ROW_PASS_SOURCES:
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic(fetch_dir, write_dir, fetch_copy, write_copy, copy_bytes, bench_log, out_json):
    import json

    copy_bytes = float(copy_bytes)
    f_scale = copy_bytes / _copy_value(fetch_copy, "FETCH_SIZE")
    w_scale = copy_bytes / _copy_value(write_copy, "WRITE_SIZE")
    f_avg, nf = _row_pass_avg(fetch_dir, "FETCH_SIZE")
    w_avg, nw = _row_pass_avg(write_dir, "WRITE_SIZE")
    bench = None
    for line in open(bench_log):
        line = line.strip()
        if line.startswith("{") and '"roofline"' in line:
            bench = json.loads(line)
    alg = bench["roofline"]["alg_bytes_per_launch"] if bench else None
    fetch_b = f_avg * f_scale
    write_b = w_avg * w_scale
    rec = {
        "kernel_source_sha256": row_pass_source_digest(),
        "kernel_sources": list(ROW_PASS_SOURCES),
        "f32": {
            "traffic_bytes_per_launch": fetch_b + write_b,
            "fetch_bytes_per_launch": fetch_b,
            "write_bytes_per_launch": write_b,
            "alg_bytes_per_launch": alg,
            "traffic_over_alg": (fetch_b + write_b) / alg if alg else None,
            "dispatches": [nf, nw],
            "fetch_scale": f_scale,
            "write_scale": w_scale,
        },
    }
    with open(out_json, "w") as fh:
        json.dump(rec, fh, indent=1)
    return rec


def window(d, prefix, start, count, min_us=None):
    """Average duration of dispatches [start, start + count) in time order
    among the kernels whose name starts with prefix (without those shorter
    than min_us microseconds, when given)."""
    rows = []
    for path in _find(d, "kernel_trace.csv"):
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if _col(r, "Kernel_Name", "Kernel-Name").startswith(prefix):
                    rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
    rows.sort()
    sel = rows[int(start):int(start) + int(count)]
    ms = [(b - a) / 1e6 for a, b in sel]
    head = f"{prefix}*: dispatches {start}..{int(start) + len(sel) - 1} of {len(rows)} in time order: "
    if min_us is None:
        return head + f"{len(sel)} dispatches, total {sum(ms):.2f} ms, average {sum(ms) / max(len(ms), 1):.4f} ms"
    ran = [t for t in ms if t * 1e3 >= float(min_us)]
    short = len(ms) - len(ran)
    return (head + f"{len(ran)} ran, total {sum(ran):.2f} ms, average {sum(ran) / max(len(ran), 1):.4f} ms; "
            f"{short} under {float(min_us):g} us (returned at once), total {sum(ms) - sum(ran):.2f} ms")


def batched_run(d, occurrence, steps):
    """Per-kernel time of one batched run (see the module docstring)."""
    rows = []
    for path in _find(d, "kernel_trace.csv"):
        with open(path) as fh:
            for r in csv.DictReader(fh):
                rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]),
                             _col(r, "Kernel_Name", "Kernel-Name")))
    rows.sort()
    # an FP64-basis batch starts at its first row pass after FP32-basis
    # batched row passes or sweeps
    starts, last = [], None
    for i, (_, _, n) in enumerate(rows):
        if "k_pass_batch<double" in n:
            if last != "f64":
                starts.append(i)
            last = "f64"
        elif "k_pass_batch<float" in n or "k_ls_pass_batch<float" in n:
            last = "f32"
    end = starts[int(occurrence) - 1]
    plans = [i for i in range(end) if rows[i][2].startswith("foa::k_batch_plan")]
    first = plans[-int(steps)]
    # the run ends with its last step's finalize (the next batch's set-up follows)
    last = max(i for i in range(first, end) if "finalize_batch" in rows[i][2])
    per = defaultdict(lambda: [0, 0.0])
    for a, b, n in rows[first:last + 1]:
        k = n.split("(")[0]
        per[k][0] += 1
        per[k][1] += (b - a) / 1e6
    busy = sum(v[1] for v in per.values())
    span = (rows[last][1] - rows[first][0]) / 1e6
    lines = [f"dispatches {first}..{last} in time order: span {span:.2f} ms, kernel time {busy:.2f} ms"]
    for k, (c, ms) in sorted(per.items(), key=lambda kv: -kv[1][1]):
        lines.append(f"{c:6d} {ms:9.2f} ms {1e3 * ms / c:9.1f} us  {k}")
    return "\n".join(lines)


def batched_traffic(fetch_dir, write_dir, fetch_scale, write_scale, steps):
    """Per-kernel HBM bytes of the batched form's last run of STEPS steps."""
    lines, total = [], 0.0
    for d, counter, scale in ((fetch_dir, "FETCH_SIZE", float(fetch_scale)),
                              (write_dir, "WRITE_SIZE", float(write_scale))):
        per, name = defaultdict(float), {}
        for f in _find(d, "counter_collection.csv"):
            for r in csv.DictReader(open(f)):
                if _col(r, "Counter_Name") != counter:
                    continue
                di = int(_col(r, "Dispatch_Id"))
                per[di] += float(_col(r, "Counter_Value"))
                name[di] = _col(r, "Kernel_Name")
        # the timed FP32-basis run ends where the FP64-basis reference batch
        # that bench.py builds after it starts
        end, last = None, None
        for di in sorted(name):
            n = name[di]
            if "k_pass_batch<double" in n:
                if last == "f32":
                    end = di
                    break
                last = "f64"
            elif "k_pass_batch<float" in n or "k_ls_pass_batch<float" in n or "k_step_persist<float" in n:
                last = "f32"
        end = end if end is not None else max(name) + 1
        plans = sorted(di for di, n in name.items() if n.startswith("foa::k_batch_plan") and di < end)
        first = plans[-int(steps)]
        tot = defaultdict(float)
        for di, v in per.items():
            n = name[di]
            if first <= di < end and ("batch" in n.lower() or "persist" in n):
                tot[n.split("(")[0]] += v * scale
        sub = sum(tot.values())
        total += sub
        lines.append(f"{counter}: {sub / 1e9:.1f} GB")
        for k, v in sorted(tot.items(), key=lambda kv: -kv[1]):
            if v >= 1e8:
                lines.append(f"    {v / 1e9:9.1f} GB  {k}")
    lines.append(f"total: {total / 1e9:.1f} GB")
    return "\n".join(lines)


def main(argv):
    if len(argv) >= 2 and argv[0] == "kernels":
        print(summarize_kernels(argv[1]))
    elif len(argv) >= 5 and argv[0] == "window":
        print(window(argv[1], argv[2], argv[3], argv[4], argv[5] if len(argv) > 5 else None))
    elif len(argv) >= 3 and argv[0] == "counter":
        print(summarize_counter(argv[1], argv[2]))
    elif len(argv) >= 9 and argv[0] == "kernel_traffic":
        import json

        print(json.dumps(kernel_traffic(*argv[1:9]), indent=1))
    elif len(argv) >= 9 and argv[0] == "counter_window":
        import json

        print(json.dumps(counter_window(*argv[1:9]), indent=1))
    elif len(argv) >= 4 and argv[0] == "batched_run":
        print(batched_run(argv[1], argv[2], argv[3]))
    elif len(argv) >= 6 and argv[0] == "batched":
        print(batched_traffic(*argv[1:6]))
    elif len(argv) >= 8 and argv[0] == "traffic":
        import json

        print(json.dumps(traffic(*argv[1:8]), indent=1))
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
