"""Summaries of rocprofv3 output for the force kernel.

Four reports, all plain text:

* ``stats``: the rows of a ``--kernel-trace --stats`` kernel_stats.csv for the
  kernels whose names contain the given filters;
* ``mix``: average per dispatch of every counter of one or more ``--pmc``
  runs (the instruction mix) for one kernel and grid size;
* ``traffic``: HBM bytes per launch of one kernel from two ``--pmc`` runs
  (``FETCH_SIZE``, then ``WRITE_SIZE``, KiB per dispatch), each scaled by what
  the same counter reads for a plain device copy of known size in the same
  run, with the hash of the kernel's sources so that a reader can tell whether
  the figure still applies to the kernel as built;
* ``tail``: from a ``--kernel-trace`` kernel_trace.csv, the last N
  dispatches of every kernel whose name contains one of the filters (the
  timed launches of a run come last, after its autotuner's candidates):
  count, average, minimum and maximum duration, by total time;
* ``rebuild``: from a ``--kernel-trace`` kernel_trace.csv, the average
  duration of every list kernel over the molecular-dynamics steps that
  rebuilt the list and over those that did not (the list kernels of a step
  run from the binning pass to the next force launch; a step rebuilt when its
  list build took longer than a threshold).

    python -m paper_1607_02904_amd.profsum stats STATS_CSV [FILTER ...]
    python -m paper_1607_02904_amd.profsum traffic FETCH_CSV WRITE_CSV \\
        --kernel NAME_PART --grid GRID --copy-bytes BYTES
    python -m paper_1607_02904_amd.profsum mix PMC_CSV [PMC_CSV ...] \\
        --kernel NAME_PART --grid GRID
    python -m paper_1607_02904_amd.profsum rebuild TRACE_CSV [--threshold-us US]
    python -m paper_1607_02904_amd.profsum tail TRACE_CSV [FILTER ...] --last N

The copy kernel is the dispatch whose name contains ``copyBuffer`` and whose
``FETCH_SIZE`` is largest.
"""
import argparse
import csv
import hashlib
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# sources of the wavefront force kernel (the dominant kernel of a step)
KERNEL_SOURCES = ("forward_wave.hip", "ters_math.h", "ters_device.h", "ters_internal.h")


def kernel_hash(sources=KERNEL_SOURCES):
    """SHA-256 over the force kernel's source files, in a fixed order."""
    h = hashlib.sha256()
    for name in sources:
        with open(os.path.join(HERE, "csrc", name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()


def stats(path, filters):
    lines = []
    with open(path) as f:
        for r in csv.DictReader(f):
            if filters and not any(flt in r["Name"] for flt in filters):
                continue
            lines.append("%-90s calls %6s  avg_us %9.2f  min_us %9.2f  max_us %9.2f  total_%% %6s"
                         % (r["Name"][:90], r["Calls"], float(r["AverageNs"]) / 1e3,
                            float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3, r["Percentage"]))
    return lines


def _per_dispatch(path, counter):
    """{dispatch id: (kernel name, grid size, summed counter value)}"""
    out = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            d = int(r["Dispatch_Id"])
            name, grid, v = out.get(d, (r["Kernel_Name"], int(r["Grid_Size"]), 0.0))
            out[d] = (name, grid, v + float(r["Counter_Value"]))
    return out


def traffic(fetch_csv, write_csv, kernel, grid, copy_bytes):
    res = {}
    for key, path, counter in (("fetch", fetch_csv, "FETCH_SIZE"), ("write", write_csv, "WRITE_SIZE")):
        disp = _per_dispatch(path, counter)
        vals = [v for (name, g, v) in disp.values() if kernel in name and g == grid]
        copies = [v for (name, g, v) in disp.values() if "copyBuffer" in name]
        if not vals or not copies:
            raise SystemExit("no %s dispatches of %r (grid %d) or no copy kernel in %s"
                             % (counter, kernel, grid, path))
        copy_kib = max(copies)
        res[key + "_kib_per_launch"] = sum(vals) / len(vals)
        res[key + "_dispatches"] = len(vals)
        res["copy_" + key + "_kib"] = copy_kib
        res[key + "_scale"] = copy_bytes / 1024.0 / copy_kib
    res["traffic_bytes_per_launch"] = 1024.0 * (res["fetch_kib_per_launch"] * res["fetch_scale"]
                                                + res["write_kib_per_launch"] * res["write_scale"])
    return res


def mix(paths, kernel, grid):
    """{counter: average per dispatch} for the dispatches of one kernel and
    grid size in one or more ``--pmc`` counter_collection.csv files."""
    sums, counts = {}, {}
    for path in paths:
        per = {}
        with open(path) as f:
            for r in csv.DictReader(f):
                if kernel not in r["Kernel_Name"] or int(r["Grid_Size"]) != grid:
                    continue
                key = (r["Counter_Name"], int(r["Dispatch_Id"]))
                per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
        for (name, _), v in per.items():
            sums[name] = sums.get(name, 0.0) + v
            counts[name] = counts.get(name, 0) + 1
    if not sums:
        raise SystemExit("no dispatches of %r (grid %d)" % (kernel, grid))
    return {k: sums[k] / counts[k] for k in sums}, counts


def read_summary(path):
    """key: value lines of a summary file (values as strings)."""
    out = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                out[k.strip()] = v.strip()
    return out

def rebuild(path, threshold_us):
    """Average durations (us) of the list kernels of the steps that rebuilt
    the list and of those that did not, in launch order."""
    import re
    rows = []
    with open(path) as f:
        for r in csv.DictReader(f):
            m = re.search(r"(k_\w+|__amd\w+)", r["Kernel_Name"])
            dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
            rows.append((int(r["Start_Timestamp"]), m.group(1) if m else r["Kernel_Name"][:40], dur))
    rows.sort()
    chains = []
    for i, (_, name, _) in enumerate(rows):
        if name != "k_bin":
            continue
        seq = []
        for _, n2, d2 in rows[i:]:
            if n2.startswith("k_force"):
                break
            seq.append((n2, d2))
        chains.append(seq)
    out = {}
    for key, sel in (("rebuild", lambda c: any(n == "k_build" and d > threshold_us for n, d in c)),
                     ("no_rebuild", lambda c: not any(n == "k_build" and d > threshold_us for n, d in c))):
        cs = [c for c in chains if sel(c)]
        per = {}
        for c in cs:
            for n, d in c:
                per.setdefault(n, []).append(d)
        out[key] = (len(cs), {n: sum(v) / len(v) for n, v in per.items()},
                    sum(sum(d for _, d in c) for c in cs) / max(len(cs), 1))
    return out


def tail(path, filters, last):
    """Durations (us) of the last `last` dispatches of each kernel whose
    name contains one of the filters, one line per kernel, by total time."""
    per = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            name = r["Kernel_Name"]
            if filters and not any(flt in name for flt in filters):
                continue
            t0, t1 = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
            per.setdefault(name, []).append((t0, (t1 - t0) / 1e3))
    lines = []
    for name, v in per.items():
        v.sort()
        d = [x for _, x in v[-last:]]
        lines.append((sum(d), "%-90.90s dispatches %4d  avg_us %9.2f  min_us %9.2f  max_us %9.2f"
                      % (name, len(d), sum(d) / len(d), min(d), max(d))))
    return [line for _, line in sorted(lines, reverse=True)]


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("filters", nargs="*")
    t = sub.add_parser("traffic")
    t.add_argument("fetch_csv")
    t.add_argument("write_csv")
    t.add_argument("--kernel", required=True)
    t.add_argument("--grid", type=int, required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    m = sub.add_parser("mix")
    m.add_argument("csv", nargs="+")
    m.add_argument("--kernel", required=True)
    m.add_argument("--grid", type=int, required=True)
    b = sub.add_parser("rebuild")
    b.add_argument("csv")
    b.add_argument("--threshold-us", type=float, default=8.0)
    l = sub.add_parser("tail")
    l.add_argument("csv")
    l.add_argument("filters", nargs="*")
    l.add_argument("--last", type=int, required=True)
    a = ap.parse_args()
    if a.cmd == "stats":
        print("\n".join(stats(a.csv, a.filters)))
    elif a.cmd == "tail":
        print("\n".join(tail(a.csv, a.filters, a.last)))
    elif a.cmd == "rebuild":
        for key, (count, per, total) in rebuild(a.csv, a.threshold_us).items():
            print("%s_steps: %d" % (key, count))
            print("%s_total_us: %.1f" % (key, total))
            for n, d in per.items():
                print("%s_%s_us: %.1f" % (key, n, d))
    elif a.cmd == "mix":
        r, counts = mix(a.csv, a.kernel, a.grid)
        print("kernel: %s" % a.kernel)
        print("grid: %d" % a.grid)
        print("kernel_sources_sha256: %s" % kernel_hash())
        print("dispatches: %d" % max(counts.values()))
        for k in sorted(r):
            print("%s: %.6g" % (k, r[k]))
    else:
        r = traffic(a.fetch_csv, a.write_csv, a.kernel, a.grid, a.copy_bytes)
        print("kernel: %s" % a.kernel)
        print("grid: %d" % a.grid)
        print("kernel_sources_sha256: %s" % kernel_hash())
        for k in sorted(r):
            print("%s: %.6g" % (k, r[k]))


if __name__ == "__main__":
    main()
