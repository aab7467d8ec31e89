"""Summarise rocprofv3 output into the short text/JSON records kept in profiles/.

  python -m paper_2603_13190_amd.rocprof_summary stats  <kernel_stats.csv> <out.txt>
         [--tail "<kernel name>=N"]... <command...>
  python -m paper_2603_13190_amd.rocprof_summary pmc    <fetch_counter_collection.csv>
         <write_counter_collection.csv> <out.json> <calibration_bytes> <command...>
  python -m paper_2603_13190_amd.rocprof_summary counters <counter_collection.csv> <out.txt> <command...>

--tail adds, from the per-dispatch trace next to the stats file
(*_kernel_trace.csv), the average duration of the kernel's last N
dispatches: the steps a benchmark profiles at the end of a run, whose
average it reports from HIP events.

The PMC mode reads FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the facet
kernels and of the calibration copy kernel (a plain device-to-device copy of
a known number of bytes), scales the facet-kernel counters by
known_bytes / counter_of_copy, and records them with the SHA-1 of the kernel
sources, so that a later benchmark reports the traffic only while the kernel
is unchanged (the SHA-1 covers the step kernels' device sources and the
build flags).
"""
import csv
import hashlib
import json
import os
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
# the sources that define the step kernels' machine code (device code and
# compile flags); host-side changes elsewhere do not invalidate the counters
KERNEL_SOURCES = [os.path.join(HERE, "csrc", f) for f in ("step_kernels.hpp", "law.hpp", "mlp.hpp")] + \
    [os.path.join(HERE, "build.py")]


def source_sha1():
    h = hashlib.sha1()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _short(name):
    name = name.split("(")[0]
    return name[:90]


def tail_average(trace_csv, kernel, n):
    """Average duration (us) and count of the last n dispatches of kernel
    (by start time) in a rocprofv3 kernel trace."""
    d = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"])) for r in _rows(trace_csv)
               if _short(r["Kernel_Name"]) == kernel)
    d = d[-n:]
    return (sum(e - b for b, e in d) / len(d) / 1e3 if d else None), len(d)


def stats(csv_path, out_path, command, tails=()):
    rows = _rows(csv_path)
    lines = [f"command: {command}", f"source: {os.path.basename(csv_path)} (rocprofv3 --kernel-trace --stats)",
             f"kernel sources sha1: {source_sha1()}", "",
             f"{'kernel':60s} {'calls':>8s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} {'total_ms':>10s} {'pct':>6s}"]
    for r in rows:
        name = r.get("Name") or r.get("KernelName") or r.get("Kernel_Name")
        calls = int(float(r.get("Calls", 0)))
        avg = float(r.get("AverageNs", 0)) / 1e3
        mn = float(r.get("MinNs", 0)) / 1e3
        mx = float(r.get("MaxNs", 0)) / 1e3
        tot = float(r.get("TotalDurationNs", 0)) / 1e6
        pct = float(r.get("Percentage", 0))
        lines.append(f"{_short(name):60s} {calls:8d} {avg:10.2f} {mn:10.2f} {mx:10.2f} {tot:10.2f} {pct:6.2f}")
    if tails:
        trace = csv_path.replace("kernel_stats", "kernel_trace")
        lines.append("")
        for kernel, n in tails:
            avg, cnt = tail_average(trace, kernel, n)
            lines.append(f"last {cnt} dispatches of {kernel}: avg {avg:.2f} us ({os.path.basename(trace)})")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _counter_by_kernel(path, counter):
    vals = defaultdict(list)
    for r in _rows(path):
        cn = r.get("Counter_Name") or r.get("CounterName")
        if cn != counter:
            continue
        name = r.get("Kernel_Name") or r.get("KernelName") or r.get("Name")
        vals[_short(name)].append(float(r.get("Counter_Value") or r.get("CounterValue")))
    return vals


def pmc(fetch_csv, write_csv, out_path, calib_bytes, command):
    fetch = _counter_by_kernel(fetch_csv, "FETCH_SIZE")
    write = _counter_by_kernel(write_csv, "WRITE_SIZE")
    calib = float(calib_bytes)

    def copy_kernel(d):
        cands = [k for k in d if "copy" in k.lower() or "elementwise" in k.lower()]
        # the calibration copy is the largest-traffic copy kernel
        return max(cands, key=lambda k: max(d[k])) if cands else None

    kf, kw = copy_kernel(fetch), copy_kernel(write)
    f_scale = calib / (max(fetch[kf]) * 1024.0) if kf else None
    w_scale = calib / (max(write[kw]) * 1024.0) if kw else None
    out = {"command": command, "kernel_sources_sha1": source_sha1(),
           "calibration": {"bytes": calib, "fetch_kernel": kf, "write_kernel": kw,
                           "fetch_KiB": max(fetch[kf]) if kf else None,
                           "write_KiB": max(write[kw]) if kw else None,
                           "fetch_scale": f_scale, "write_scale": w_scale},
           "kernels": {}}
    for k in sorted(set(fetch) | set(write)):
        if not k.startswith("void k_") and not k.startswith("k_") and "k_facet" not in k and "k_particle" not in k:
            continue
        fv, wv = fetch.get(k, []), write.get(k, [])
        fa = sum(fv) / len(fv) * 1024.0 if fv else None
        wa = sum(wv) / len(wv) * 1024.0 if wv else None
        out["kernels"][k] = {
            "dispatches": max(len(fv), len(wv)),
            "fetch_bytes_raw": fa, "write_bytes_raw": wa,
            "fetch_bytes": fa * f_scale if (fa is not None and f_scale) else None,
            "write_bytes": wa * w_scale if (wa is not None and w_scale) else None,
        }
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


def counters(csv_path, out_path, command):
    """Per-kernel average of every counter in one --pmc pass, with the
    per-wave figures (instructions and cycles divided by SQ_WAVES)."""
    per = defaultdict(lambda: defaultdict(list))
    for r in _rows(csv_path):
        cn = r.get("Counter_Name") or r.get("CounterName")
        name = _short(r.get("Kernel_Name") or r.get("KernelName") or r.get("Name"))
        per[name][cn].append(float(r.get("Counter_Value") or r.get("CounterValue")))
    lines = [f"command: {command}", f"source: {os.path.basename(csv_path)} (rocprofv3 --pmc)",
             f"kernel sources sha1: {source_sha1()}", ""]
    for k in sorted(per):
        if "k_" not in k:
            continue
        avg = {c: sum(v) / len(v) for c, v in per[k].items()}
        waves = avg.get("SQ_WAVES")
        lines.append(f"{k}  ({max(len(v) for v in per[k].values())} dispatches)")
        for c in sorted(avg):
            extra = f"   {avg[c] / waves:12.1f} per wave" if waves and c != "SQ_WAVES" else ""
            lines.append(f"  {c:24s} {avg[c]:16.1f}{extra}")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    mode = sys.argv[1]
    if mode == "stats":
        rest, tails = sys.argv[4:], []
        while rest and rest[0] == "--tail":
            k, n = rest[1].rsplit("=", 1)
            tails.append((k, int(n)))
            rest = rest[2:]
        stats(sys.argv[2], sys.argv[3], " ".join(rest), tails)
    elif mode == "pmc":
        pmc(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], " ".join(sys.argv[6:]))
    elif mode == "counters":
        counters(sys.argv[2], sys.argv[3], " ".join(sys.argv[4:]))
    else:
        raise SystemExit(__doc__)
