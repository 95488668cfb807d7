"""Summaries of rocprofv3 output.

Kernel trace (``*_results.db``): per kernel symbol (and grid size) the number
of dispatches, total and average duration.

    python -m paper_2602_03438_amd.profsummary <output dir>/run_results.db [--by-grid] [--top 20]

Matrix-core activity from one counter run (SQ_INSTS_VALU_MFMA_MOPS_F64,
SQ_VALU_MFMA_BUSY_CYCLES, GRBM_GUI_ACTIVE) of the product kernel:

    python -m paper_2602_03438_amd.profsummary --mfma MFMA_DIR [--kernel REGEX]

HBM traffic from two counter runs (``--pmc FETCH_SIZE`` and ``--pmc
WRITE_SIZE``, csv output) of a program that also ran one streaming kernel of
known size (``bench.py --calibrate-copy MIB``): both counters are scaled by
what they read for that kernel, then averaged per launch of the kernels
matching a pattern.

    python -m paper_2602_03438_amd.profsummary --traffic FETCH_DIR WRITE_DIR --calib-mib 1024 \\
        [--block 512] [--kernel REGEX] [--json out.json]
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
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


def _counter_rows(d: str):
    """(dispatch id, kernel name, counter name, value, grid size, workgroup size) from a csv counter run."""
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no *counter_collection.csv under {d}")
    for f in files:
        with open(f, newline="") as fh:
            for row in csv.DictReader(fh):
                row = {k.lower(): v for k, v in row.items()}
                yield (int(row["dispatch_id"]), row["kernel_name"], row["counter_name"],
                       float(row["counter_value"]), int(row["grid_size"]), int(row["workgroup_size"]))


def per_dispatch(d: str, counter: str):
    """{dispatch id: (kernel name, value summed over the counter's instances, workgroups)}"""
    acc = {}
    for did, name, cname, val, grid, wg in _counter_rows(d):
        if cname != counter:
            continue
        n0, v0, g0 = acc.get(did, (name, 0.0, grid // max(1, wg)))
        acc[did] = (n0, v0 + val, g0)
    return acc


_CFG = re.compile(r"Cfg<(\d+), (\d+), \d, \d>")


def items_of(name: str, wgs: int, block: int) -> float:
    """Batch items (b x b x b complex products) in a dispatch of the product kernel."""
    m = _CFG.search(name)
    bm, bn = int(m.group(1)), int(m.group(2))
    tiles = -(-block // bm) * -(-block // bn)
    return wgs / tiles


def gemm_source_hash(root: str, source: str = "gemm.hip") -> str:
    """First 16 hex digits of the sha256 of a kernel source under csrc/ (the product kernels by default)."""
    h = hashlib.sha256()
    with open(os.path.join(root, "paper_2602_03438_amd", "csrc", source), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def traffic(fetch_dir: str, write_dir: str, calib_mib: int, kernel: str, block: int,
            calib_kernel: str = "elementwise", items: float = 0.0):
    """HBM bytes of the product kernel: per launch and per b x b x b item (so that a
    launch of any batch can be priced as items x bytes_per_item).  With items > 0 every
    launch of the kernel counts that many items (another kernel's unit: elements, say)."""
    fetch = per_dispatch(fetch_dir, "FETCH_SIZE")
    write = per_dispatch(write_dir, "WRITE_SIZE")
    nbytes = calib_mib << 20

    def calib(table):
        cands = [v for (n, v, _) in table.values() if calib_kernel in n]
        if not cands:
            raise RuntimeError(f"no dispatch of a kernel matching '{calib_kernel}'")
        return max(cands) * 1024.0      # the largest one is the calibration copy; counters are in KiB

    f_cal, w_cal = calib(fetch), calib(write)
    f_scale, w_scale = nbytes / f_cal, nbytes / w_cal
    pat = re.compile(kernel)
    count = (lambda n, g: items) if items > 0 else (lambda n, g: items_of(n, g, block))
    fk = [(v * 1024.0 * f_scale, count(n, g)) for (n, v, g) in fetch.values() if pat.search(n)]
    wk = [(v * 1024.0 * w_scale, count(n, g)) for (n, v, g) in write.values() if pat.search(n)]
    if not fk or not wk:
        raise RuntimeError(f"no dispatch matching '{kernel}'")
    f_item = sum(b for b, _ in fk) / sum(i for _, i in fk)
    w_item = sum(b for b, _ in wk) / sum(i for _, i in wk)
    return {"kernel_pattern": kernel, "block": block, "launches_fetch": len(fk), "launches_write": len(wk),
            "fetch_bytes_per_launch": sum(b for b, _ in fk) / len(fk),
            "write_bytes_per_launch": sum(b for b, _ in wk) / len(wk),
            "bytes_per_launch": sum(b for b, _ in fk) / len(fk) + sum(b for b, _ in wk) / len(wk),
            "items_per_launch": sum(i for _, i in fk) / len(fk),
            "fetch_bytes_per_item": f_item, "write_bytes_per_item": w_item, "bytes_per_item": f_item + w_item,
            "calibration": {"bytes": nbytes, "fetch_counter_bytes": f_cal, "write_counter_bytes": w_cal,
                            "fetch_scale": f_scale, "write_scale": w_scale}}


def _gpu_agent(d: str):
    """(SIMD count, XCC count, max engine clock in MHz) of the GPU agent of a counter run."""
    files = glob.glob(os.path.join(d, "**", "*agent_info.csv"), recursive=True)
    for f in files:
        with open(f, newline="") as fh:
            for row in csv.DictReader(fh):
                if row.get("Agent_Type") == "GPU":
                    return int(row["Simd_Count"]), int(row["Num_Xcc"]), float(row["Max_Engine_Clk_Fcompute"])
    return 1024, 8, 2400.0


def mfma(mfma_dir: str, kernel: str, mops_counter: str = "SQ_INSTS_VALU_MFMA_MOPS_F64"):
    """Matrix-core activity of the product kernel from one counter run with
    SQ_INSTS_VALU_MFMA_MOPS_F64, SQ_VALU_MFMA_BUSY_CYCLES and GRBM_GUI_ACTIVE,
    per launch: the FP64 matrix flops the hardware counted (MOPS x 512, the
    derived MfmaFlopsF64 of rocprofv3); the fraction of SIMD cycles the matrix
    cores were busy, busy / (GUI-active cycles of one XCC x SIMDs) (MfmaUtil;
    the csv holds GRBM_GUI_ACTIVE summed over the XCCs, so it is divided by
    their number); and the engine clock the GUI-active cycles imply over the
    launch's duration."""
    mops = per_dispatch(mfma_dir, mops_counter)
    busy = per_dispatch(mfma_dir, "SQ_VALU_MFMA_BUSY_CYCLES")
    simd_num, n_xcc, clk = _gpu_agent(mfma_dir)
    gui, dur = {}, {}
    files = glob.glob(os.path.join(mfma_dir, "**", "*counter_collection.csv"), recursive=True)
    for f in files:
        with open(f, newline="") as fh:
            for row in csv.DictReader(fh):
                did = int(row["Dispatch_Id"])
                dur[did] = (int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) * 1e-9
                if row["Counter_Name"] == "GRBM_GUI_ACTIVE":
                    gui[did] = gui.get(did, 0.0) + float(row["Counter_Value"]) / n_xcc
    pat = re.compile(kernel)
    rows = [did for did, (n, _, _) in mops.items() if pat.search(n)]
    if not rows:
        raise RuntimeError(f"no dispatch matching '{kernel}'")
    fl = [mops[d][1] * 512.0 for d in rows]
    util = [busy[d][1] / (gui[d] * simd_num) for d in rows if d in busy and gui.get(d)]
    mhz = [gui[d] / dur[d] / 1e6 for d in rows if gui.get(d) and dur.get(d)]
    mean = lambda x: sum(x) / len(x) if x else None
    return {"kernel_pattern": kernel, "launches": len(rows), "mops_counter": mops_counter,
            "mfma_flops_per_launch": mean(fl),
            "mfma_busy_frac_mean": mean(util), "mfma_busy_frac_min": min(util) if util else None,
            "mfma_busy_frac_max": max(util) if util else None, "simd_num": simd_num, "xcc": n_xcc,
            "engine_clock_mhz_from_gui_active": mean(mhz), "max_engine_clock_mhz": clk}


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("db", nargs="?")
    ap.add_argument("--by-grid", action="store_true")
    ap.add_argument("--top", type=int, default=25)
    ap.add_argument("--traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--calib-mib", type=int, default=1024)
    ap.add_argument("--kernel", default=r"zgemm_kernel<double, [01], [01], [^>]*Cfg<\d+, \d+, \d, \d>, 0(, (true|false))*>")
    ap.add_argument("--block", type=int, default=512, help="block size b of the products")
    ap.add_argument("--items", type=float, default=0.0, help="items per launch for a kernel other than the "
                    "product (e.g. the elements of an energy convolution)")
    ap.add_argument("--calib-kernel", default="elementwise", help="name fragment of the calibration copy "
                    "(the largest matching dispatch is taken)")
    ap.add_argument("--source", default="gemm.hip", help="csrc/ file whose hash is stored with the summary")
    ap.add_argument("--mfma", metavar="MFMA_DIR", help="counter run with SQ_INSTS_VALU_MFMA_MOPS_F64, "
                    "SQ_VALU_MFMA_BUSY_CYCLES and GRBM_GUI_ACTIVE")
    ap.add_argument("--mops", default="SQ_INSTS_VALU_MFMA_MOPS_F64", help="matrix-op counter of the --mfma run")
    ap.add_argument("--json")
    ap.add_argument("--note", default="", help="what the counter runs measured (stored in the JSON)")
    a = ap.parse_args()
    if a.mfma:
        rec = mfma(a.mfma, a.kernel, a.mops)
        print(json.dumps(rec, indent=1))
        if a.json:
            with open(a.json, "w") as f:
                json.dump(rec, f, indent=1)
    elif a.traffic:
        rec = traffic(a.traffic[0], a.traffic[1], a.calib_mib, a.kernel, a.block, calib_kernel=a.calib_kernel,
                      items=a.items)
        root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
        rec["kernel_sha"] = gemm_source_hash(root, a.source)
        rec["source"] = a.source
        rec["note"] = a.note
        print(json.dumps(rec, indent=1))
        if a.json:
            with open(a.json, "w") as f:
                json.dump(rec, f, indent=1)
    else:
        print(summarize(a.db, a.by_grid, a.top))
    sys.exit(0)
