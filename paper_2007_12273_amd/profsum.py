"""Summaries of rocprofv3 CSV output for this library's kernels.

    python -m paper_2007_12273_amd.profsum trace  <kernel_trace.csv>
    python -m paper_2007_12273_amd.profsum bytes  <FETCH counter csv> <WRITE counter csv>
    python -m paper_2007_12273_amd.profsum insts  <visits.npz> <call>:<cold|warm> <counter csv> [...]

trace: per-kernel dispatch counts and durations, and per gm_compress call
(a call starts with the k_plan_reset dispatch) the span of its EM phase,
first k_em start to last k_em end (the length buckets run concurrently on
several streams, so the phase span, not a single dispatch, is the unit the
EM roofline is quoted on).

bytes: per gm_compress call the FETCH_SIZE and WRITE_SIZE counter totals
(KiB) over its k_em dispatches, and the same counters for the largest
device copy in the run (a plain copy of known size calibrates them).

insts: instruction counters (any SQ_ counters, one or more csv files of
runs with the same launch sequence) of the k_em dispatches of one
gm_compress call, per wave-update: a component update executed by one
wave of the cell's workgroup.  A dispatch's cells are those of its length
bucket, which under the built-in launch plan holds the cells of up to
64 * per_thread * waves particles (above the next smaller bucket's bound);
visits.npz (bench.py --visits-out) gives the per-cell counts and updates of
the cold and the warm fit.
"""
from __future__ import annotations

import csv
import sys
from collections import OrderedDict


def _rows(path):
    with open(path) as f:
        return list(csv.DictReader(f))


def _calls(rows, key_start):
    """Split dispatches (in dispatch order) into gm_compress calls."""
    rows = sorted(rows, key=lambda r: int(r["Dispatch_Id"]))
    calls, cur, last = [], None, None
    for r in rows:
        name = r["Kernel_Name"]
        # counter files hold one row per (dispatch, counter)
        first = r["Dispatch_Id"] != last
        last = r["Dispatch_Id"]
        if "k_plan_reset" in name and first:
            cur = []
            calls.append(cur)
        if cur is not None and "k_em<" in name:
            cur.append(r)
        if "k_finish<" in name:
            cur = None
    return calls


def trace(path):
    rows = _rows(path)
    agg = OrderedDict()
    for r in rows:
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6
        name = r["Kernel_Name"].split("(")[0][:70]
        a = agg.setdefault(name, [0, 0.0])
        a[0] += 1
        a[1] += d
    print("%-72s %6s %12s %10s" % ("kernel", "calls", "total ms", "avg ms"))
    for name, (n, t) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        print("%-72s %6d %12.3f %10.4f" % (name, n, t, t / n))
    print()
    print("EM phase span per gm_compress call (first k_em start to last k_em end):")
    for i, c in enumerate(_calls(rows, "k_plan_reset")):
        if not c:
            continue
        t0 = min(int(r["Start_Timestamp"]) for r in c)
        t1 = max(int(r["End_Timestamp"]) for r in c)
        busy = sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in c)
        print("  call %2d: %2d k_em dispatches, span %8.3f ms, sum of dispatch durations %8.3f ms"
              % (i, len(c), (t1 - t0) * 1e-6, busy * 1e-6))


def _counter_calls(path):
    rows = _rows(path)
    calls = _calls(rows, "k_plan_reset")
    totals = [sum(float(r["Counter_Value"]) for r in c) for c in calls]
    copies = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]]
    return totals, (max(copies) if copies else 0.0)


def bytes_(fetch_path, write_path):
    f_tot, f_copy = _counter_calls(fetch_path)
    w_tot, w_copy = _counter_calls(write_path)
    print("largest device copy: FETCH_SIZE %.0f KiB, WRITE_SIZE %.0f KiB" % (f_copy, w_copy))
    print("per gm_compress call, k_em dispatches summed (KiB):")
    for i, (f, w) in enumerate(zip(f_tot, w_tot)):
        print("  call %2d: FETCH_SIZE %12.0f  WRITE_SIZE %12.0f" % (i, f, w))


def _dispatch_shape(r):
    """(particles per thread, waves) of a k_em dispatch row."""
    args = r["Kernel_Name"].split("k_em<", 1)[1].split(">", 1)[0].split(",")
    return int(args[2]), int(r["Workgroup_Size"]) // 64


def insts(visits_path, spec, paths):
    import numpy as np
    z = np.load(visits_path)
    n = z["n"]
    call, which = spec.split(":")
    visits = z["visits_" + which]
    tot, wave_updates, updates = OrderedDict(), 0, 0
    for path in paths:
        disp = OrderedDict()
        for r in _calls(_rows(path), "k_plan_reset")[int(call)]:
            d = disp.setdefault(r["Dispatch_Id"], {"row": r, "c": {}})
            d["c"][r["Counter_Name"]] = d["c"].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        shapes = sorted({(64 * P * W, W) for P, W in (_dispatch_shape(d["row"]) for d in disp.values())})
        wu, up, lo = 0, 0, 0
        for hi, W in shapes:
            sel = (n > lo) & (n <= hi)
            up += int(visits[sel].sum())
            wu += int(visits[sel].sum()) * W
            lo = hi
        wave_updates, updates = wu, up
        for d in disp.values():
            for k, v in d["c"].items():
                tot[k] = tot.get(k, 0.0) + v
    print("call %s (%s fit): %d component updates, %d wave-updates" % (call, which, updates, wave_updates))
    for k, v in tot.items():
        print("  %-32s %14.4g total %10.2f per wave-update" % (k, v, v / max(1, wave_updates)))


def main(argv):
    if len(argv) >= 2 and argv[0] == "trace":
        trace(argv[1])
    elif len(argv) >= 3 and argv[0] == "bytes":
        bytes_(argv[1], argv[2])
    elif len(argv) >= 4 and argv[0] == "insts":
        insts(argv[1], argv[2], argv[3:])
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
