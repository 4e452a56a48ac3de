"""Print the per-kernel table of a rocprofv3 SQLite output (kernel trace)."""
import sqlite3
import sys


def summary(db):
    con = sqlite3.connect(db)
    rows = con.execute("select name, total_calls, total_duration, average, percentage from top_kernels").fetchall()
    # the top_kernels view reports durations in microseconds
    out = ["| kernel | calls | total us | avg us | % |", "|---|---|---|---|---|"]
    for name, calls, tot, avg, pct in rows:
        short = name.split("(")[0].replace("void ", "")
        out.append(f"| `{short}` | {calls} | {tot:.1f} | {avg:.3f} | {pct:.2f} |")
    return "\n".join(out)


if __name__ == "__main__":
    print(summary(sys.argv[1]))
