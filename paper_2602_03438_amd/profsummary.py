"""Summarise a rocprofv3 kernel-trace database (``*_results.db``) as a short
text table: per kernel symbol (and grid size) the number of dispatches, total
and average duration.

    python -m paper_2602_03438_amd.profsummary gpurun_out/prof/run_results.db [--by-grid] [--top 20]
"""
from __future__ import annotations

import argparse
import sqlite3
import sys


def short(name: str) -> str:
    name = name.replace("negf::(anonymous namespace)::", "").replace("negf::", "")
    name = name.replace("HIP_vector_type<double, 2u>", "double2")
    return name if len(name) < 110 else name[:107] + "..."


def summarize(db: str, by_grid: bool = False, top: int = 25):
    con = sqlite3.connect(db)
    key = "name, grid_x, grid_y, grid_z" if by_grid else "name"
    rows = con.execute(f"select {key}, count(*), sum(duration), avg(duration) from kernels group by {key} "
                       f"order by sum(duration) desc").fetchall()
    total = sum(r[-2] for r in rows)
    out = []
    for r in rows[:top]:
        name = short(r[0])
        grid = f" grid=({r[1]},{r[2]},{r[3]})" if by_grid else ""
        cnt, tot, avg = r[-3], r[-2], r[-1]
        out.append(f"{tot / total * 100:6.2f}%  calls {cnt:6d}  total {tot / 1e6:10.3f} ms  avg {avg / 1e3:9.3f} us  "
                   f"{name}{grid}")
    return f"kernels: {len(rows)} symbols, {sum(r[-3] for r in rows)} dispatches, {total / 1e6:.3f} ms total\n" + \
        "\n".join(out)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("db")
    ap.add_argument("--by-grid", action="store_true")
    ap.add_argument("--top", type=int, default=25)
    a = ap.parse_args()
    print(summarize(a.db, a.by_grid, a.top))
    sys.exit(0)
