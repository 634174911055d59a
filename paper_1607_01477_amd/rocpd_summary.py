"""Text summary of a rocprofv3 result database (the SQLite `*_results.db`).

    python -m paper_1607_01477_amd.rocpd_summary RESULTS_DB [--by-grid NAME_SUBSTR]

Prints per kernel: calls, total and average duration; for counter-collection
runs, per kernel and counter: dispatches, mean value per dispatch and total.
With --by-grid, durations of the matching kernel grouped by grid size.
"""
from __future__ import annotations

import argparse
import sqlite3
import sys


def short(name: str, width: int = 110) -> str:
    return name if len(name) <= width else name[: width - 3] + "..."


def summarize(db: str, by_grid: str | None = None, out=sys.stdout) -> None:
    con = sqlite3.connect(db)
    views = {r[0] for r in con.execute("select name from sqlite_master where type in ('table','view')")}
    if "kernels" in views:
        rows = con.execute("select name, count(*), sum(duration), avg(duration), min(duration), "
                           "max(duration) from kernels group by name order by sum(duration) desc").fetchall()
        if rows:
            total = sum(r[2] for r in rows)
            print("kernel trace (durations in microseconds)", file=out)
            print("%-110s %7s %12s %10s %10s %10s %6s" % ("kernel", "calls", "total_us", "avg_us",
                                                       "min_us", "max_us", "pct"), file=out)
            for name, n, tot, avg, mn, mx in rows:
                print("%-110s %7d %12.1f %10.2f %10.2f %10.2f %6.2f" % (
                    short(name), n, tot / 1e3, avg / 1e3, mn / 1e3, mx / 1e3, 100.0 * tot / total), file=out)
        if by_grid:
            rows = con.execute("select grid_x, workgroup_x, count(*), avg(duration) from kernels "
                               "where name like ? group by grid_x order by grid_x",
                               ("%" + by_grid + "%",)).fetchall()
            print("\n%s by grid size" % by_grid, file=out)
            print("%10s %8s %8s %10s" % ("workgroups", "wg_size", "calls", "avg_us"), file=out)
            for gx, wx, n, avg in rows:
                print("%10d %8d %8d %10.2f" % (gx // max(1, wx), wx, n, avg / 1e3), file=out)
    if "counters_collection" in views:
        rows = con.execute("select kernel_name, counter_name, count(*), avg(value), sum(value) "
                           "from counters_collection group by kernel_name, counter_name "
                           "order by kernel_name, counter_name").fetchall()
        if rows:
            print("\ncounters (per dispatch mean, total over dispatches)", file=out)
            print("%-110s %-34s %6s %16s %18s" % ("kernel", "counter", "disp", "mean", "total"), file=out)
            for k, c, n, avg, tot in rows:
                print("%-110s %-34s %6d %16.1f %18.1f" % (short(k), c, n, avg, tot), file=out)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("db")
    ap.add_argument("--by-grid", default=None)
    args = ap.parse_args()
    summarize(args.db, args.by_grid)
    return 0


if __name__ == "__main__":
    sys.exit(main())
