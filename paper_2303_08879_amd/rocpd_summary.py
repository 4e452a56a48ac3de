"""Summaries of rocprofv3 output for the profiles/ notes.

    python rocpd_summary.py <results.db>              per-kernel table (kernel trace)
    python rocpd_summary.py --pmc <counter_collection.csv> [name-filter ...]
                                                      mean counter value per dispatch
    python rocpd_summary.py --timeline <results.db> <marker> <k> <n>
                                                      n dispatches in launch order from the
                                                      k-th dispatch whose name contains marker
"""
import csv
import sqlite3
import sys
from collections import defaultdict


def summary(db):
    con = sqlite3.connect(db)
    rows = con.execute("select name, total_calls, total_duration, average, percentage from top_kernels").fetchall()
    # the top_kernels view reports durations in microseconds
    out = ["| kernel | calls | total us | avg us | % |", "|---|---|---|---|---|"]
    for name, calls, tot, avg, pct in rows:
        short = name.split("(")[0].replace("void ", "")
        out.append(f"| `{short}` | {calls} | {tot:.1f} | {avg:.3f} | {pct:.2f} |")
    return "\n".join(out)


def pmc_summary(path, filters=()):
    """Mean and total of every counter per kernel name over its dispatches
    (rocprofv3 --output-format csv counter collection file)."""
    acc = defaultdict(lambda: defaultdict(list))
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            name = row.get("Kernel_Name", "")
            if filters and not any(k in name for k in filters):
                continue
            short = name.split("(")[0].replace("void ", "")
            acc[short][row["Counter_Name"]].append((row.get("Dispatch_Id"), float(row["Counter_Value"])))
    out = ["| kernel | counter | dispatches | mean per dispatch | total |", "|---|---|---|---|---|"]
    for name in sorted(acc):
        for cn in sorted(acc[name]):
            # one value per dispatch (values of one dispatch are summed over their dimensions)
            per = defaultdict(float)
            for d, v in acc[name][cn]:
                per[d] += v
            vals = list(per.values())
            out.append(f"| `{name}` | {cn} | {len(vals)} | {sum(vals) / len(vals):.1f} | {sum(vals):.1f} |")
    return "\n".join(out)


def timeline(db, marker, k, n):
    """Dispatches in start order: kernel, workgroups, start offset and duration
    (us) -- one pass of a sweep, to read per-launch latency against size."""
    con = sqlite3.connect(db)
    rows = con.execute("select name, start, duration, grid_x / workgroup_x from kernels order by start").fetchall()
    hits = [i for i, r in enumerate(rows) if marker in r[0]]
    i0 = hits[k]
    t0 = rows[i0][1]
    out = ["| # | kernel | workgroups | start us | duration us |", "|---|---|---|---|---|"]
    for j, (name, start, dur, wg) in enumerate(rows[i0:i0 + n]):
        short = name.split("(")[0].replace("void ", "")
        out.append(f"| {j} | `{short}` | {wg} | {(start - t0) / 1000:.1f} | {dur / 1000:.1f} |")
    return "\n".join(out)


if __name__ == "__main__":
    if sys.argv[1] == "--pmc":
        print(pmc_summary(sys.argv[2], sys.argv[3:]))
    elif sys.argv[1] == "--timeline":
        print(timeline(sys.argv[2], sys.argv[3], int(sys.argv[4]), int(sys.argv[5])))
    else:
        print(summary(sys.argv[1]))
