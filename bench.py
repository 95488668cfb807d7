"""Throughput of the NEGF hot path on one MI355X: energy points per second of
RGF G^R + G^< at Nb = 60 blocks of b = 512 (plain FP64 and the chosen
single-product form with refinement), with the roofline of the dominant kernel
and the CPU oracle timed on the host beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--points P]

A step is one pass of the whole hot path -- both lead decimations, the forward
and backward retarded sweeps and the forward and backward lesser sweeps,
outputs written to HBM -- over a batch of P energy points of the synthetic
nano-ribbon-like device (the Si ribbon Hamiltonian of the paper is not
available; see workloads.slab_device).  Inputs are resident in HBM before the
timed region.  One JSON line is printed on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f64": 78.6e12, "f32": 157.3e12}   # MI355X dense matrix peaks (FLOP/s)
NB, B, SEED = 60, 512, 2
N_GRID = 1024
ETA, MU_L, MU_R, KT = 1e-8, 0.1, -0.1, 0.025


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def energy_batches(P):
    grid = np.linspace(-1.5, 1.5, N_GRID)
    # interleaved batches: batch j takes every (N_GRID/P)-th energy starting at j
    stride = max(1, N_GRID // P)
    return [grid[j::stride][:P] for j in range(stride)]


def kernel_hash():
    h = hashlib.sha256()
    for f in ("gemm.hip",):
        with open(os.path.join(ROOT, "paper_2602_03438_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_record():
    """HBM traffic of the dominant kernel from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", "gemm_f64_traffic.json")
    if not os.path.exists(p):
        return None
    try:
        rec = json.load(open(p))
    except Exception:
        return None
    if rec.get("kernel_sha") != kernel_hash():
        return None
    return rec.get("bytes_per_launch")


def run_steps(nb, probs, batches, prec, steps, warmup, outputs, ws, opts, profile=False):
    import torch
    times = []
    n_done = 0
    for k in range(warmup + steps):
        if k == warmup:
            torch.cuda.synchronize()
            if profile:
                nb.negf_profile_enable(1)
            t0 = time.perf_counter()
        probs[0].energies.copy_(torch.from_numpy(batches[k % len(batches)]).to("cuda"))
        res = nb.rgf_lesser_greater(probs, prec, opts=opts, ws=ws, outputs=outputs, lower=True)
        if k >= warmup:
            n_done += probs[0].n_e
        torch.cuda.synchronize()
        log(f"  prec={prec} step {k + 1}/{warmup + steps} done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stats = None
    if profile:
        stats = nb.negf_profile_read()
        nb.negf_profile_enable(0)
    return dt, n_done, res, stats


def cpu_baseline(dev, energies):
    """The FP64 oracle on one energy point of the same workload."""
    from oracle import rgf as orgf
    try:
        from threadpoolctl import threadpool_info
        info = threadpool_info()
        threads = max([x.get("num_threads", 1) for x in info if x.get("user_api") == "blas"] or [1])
        blas = ",".join(sorted({x.get("internal_api", "?") for x in info if x.get("user_api") == "blas"}))
    except Exception:
        threads, blas = os.cpu_count(), "?"
    E = float(energies[len(energies) // 2])
    t0 = time.perf_counter()
    ref = orgf.solve_point(dev, E, ETA, MU_L, MU_R, KT)
    dt = time.perf_counter() - t0
    return dict(value=1.0 / dt, unit="energy points/s", cores=int(threads), kind="oracle",
                sample=f"1 energy point (E={E:.4f}) of the Nb=60 b=512 slab workload: both lead decimations, "
                       f"G^R and G^< sweeps in NumPy complex128 ({blas} BLAS)", seconds=dt,
                host_cpus=os.cpu_count()), ref, E


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--points", type=int, default=64)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-chosen", action="store_true")
    ap.add_argument("--inv-nb", type=int, default=32)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU's share of the energy grid; --gpus {args.gpus} is not supported "
              f"(energy points are independent and shard across GPUs with no exchange).", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as w
    from paper_2602_03438_amd import binding as nb

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    nb.lib()
    log("generating the Nb=60 b=512 slab device ...")
    dev = w.slab_device(NB, B, SEED)
    batches = energy_batches(args.points)
    gdev = nb.DeviceOnGPU(dev)
    prob = nb.Problem(gdev, batches[0], eta=ETA, mu_l=MU_L, mu_r=MU_R, kT=KT)
    probs = [prob]
    opts = nb.make_options(inv_nb=args.inv_nb)
    ws = nb.Workspace()
    outputs = nb._rgf_outputs(probs, True, False, True)
    torch.cuda.synchronize()

    log("plain FP64 ...")
    dt, n_pts, res, stats = run_steps(nb, probs, batches, nb.PLAIN_FP64, args.steps, args.warmup, outputs, ws, opts,
                                      profile=True)
    info = res["info"].cpu().numpy()
    value = n_pts / dt
    g = stats["gemm_f64"]
    achieved = g["flops"] / (g["total_ms"] * 1e-3) if g["total_ms"] > 0 else 0.0
    launches = max(1, g["launches"])
    traffic = traffic_record()
    # algorithmic flops of the whole step (dense-block count of the method, K_SR measured)
    roof = {"bound": "mfma", "kernel": "zgemm_kernel<double> (batched complex FP64 product)",
            "achieved": achieved / 1e12, "peak": PEAK["f64"] / 1e12, "unit": "TFLOP/s",
            "frac": achieved / PEAK["f64"], "traffic": traffic,
            "launches": int(g["launches"]), "avg_launch_ms": g["total_ms"] / launches,
            "flops_per_launch": g["flops"] / launches}
    kstats = {k: {"launches": int(v["launches"]), "total_ms": round(v["total_ms"], 3),
                  "tflops": (v["flops"] / (v["total_ms"] * 1e-3) / 1e12) if v["total_ms"] > 0 and v["flops"] else None}
              for k, v in stats.items() if v["launches"]}

    chosen = None
    if not args.no_chosen:
        plain_GR = outputs["GR_diag"].clone()
        plain_GL = outputs["GL_diag"].clone()
        last_batch = batches[(args.warmup + args.steps - 1) % len(batches)]
        out = {}
        for prec, name in ((nb.FP32_REFINE, "fp32_refine"), (nb.FP32_NOREFINE, "fp32_norefine")):
            log(f"{name} ...")
            dtc, nc, resc, st = run_steps(nb, probs, batches, prec, args.steps, args.warmup, outputs, ws, opts,
                                          profile=True)
            eR = (torch.linalg.vector_norm(outputs["GR_diag"] - plain_GR) / torch.linalg.vector_norm(plain_GR)).item()
            eL = (torch.linalg.vector_norm(outputs["GL_diag"] - plain_GL) / torch.linalg.vector_norm(plain_GL)).item()
            ideal = st["gemm_f64"]["flops"] / PEAK["f64"] + st["gemm_f32"]["flops"] / PEAK["f32"]
            out[name] = {"value": nc / dtc, "ms_per_step": dtc / args.steps * 1e3,
                         "err_vs_plain_GR_diag": eR, "err_vs_plain_GL_diag": eL,
                         "gemm_f32_tflops": (st["gemm_f32"]["flops"] / (st["gemm_f32"]["total_ms"] * 1e-3) / 1e12)
                         if st["gemm_f32"]["total_ms"] > 0 else None,
                         "mixed_peak_frac_of_products": ideal / ((st["gemm_f64"]["total_ms"] + st["gemm_f32"]["total_ms"]) * 1e-3)
                         if (st["gemm_f64"]["total_ms"] + st["gemm_f32"]["total_ms"]) > 0 else None}
        chosen = out

    cpu = None
    if not args.no_cpu:
        log("CPU oracle on one point ...")
        cpu, _, _ = cpu_baseline(dev, batches[0])

    line = {
        "metric": "energy points/s, RGF G^R+G^< (Nb=60, b=512): plain FP64 vs chosen form",
        "value": value,
        "unit": "energy points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "nano-ribbon-like slab device, Nb=60 blocks of b=512 (52 atoms x 10 orbitals, "
                               "~14% dense blocks, S = I + PSD), Sancho-Rubio leads at eta=1e-8, "
                               "muL=0.1 muR=-0.1 kT=0.025, energies from 1024 in [-1.5,1.5]",
                   "points_per_step": args.points, "nb": NB, "b": B, "precision": "plain FP64",
                   "outputs": "G^R diag/upper/lower + G^< diag/upper in HBM"},
        "info_nonzero": int(np.count_nonzero(info)),
        "roofline": roof,
        "kernels": kstats,
        "chosen_form": chosen,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
