"""Summarise a rocprofv3 rocpd database (kernel trace) as a markdown table:
per kernel name, dispatch count, average / min / max duration (us) and total
time (ms).

    python rocpd_summary.py gpurun_out/prof/bench_results.db
"""
import sqlite3
import sys


def main(path):
    db = sqlite3.connect(path)
    rows = db.execute(
        "select name, count(*), avg(end-start), min(end-start), max(end-start), sum(end-start) "
        "from kernels group by name order by sum(end-start) desc").fetchall()
    print("| kernel | dispatches | avg us | min us | max us | total ms |")
    print("|---|---|---|---|---|---|")
    for n, c, a, lo, hi, s in rows:
        print(f"| `{n}` | {c} | {a / 1e3:.2f} | {lo / 1e3:.2f} | {hi / 1e3:.2f} | {s / 1e6:.3f} |")


if __name__ == "__main__":
    main(sys.argv[1])
