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


def point_flops(nb, b, steps=28):
    """Algorithmic flops of one energy point of G^R + G^< by the dense count (one complex
    product or inversion of b x b blocks = 8 b^3): G^R (8 + 56 (nb - 1)) b^3, G^< (16 + 64 (nb - 1)) b^3,
    both leads 2 (56 steps + 24) b^3 with `steps` decimation steps."""
    return float(b) ** 3 * ((8 + 56 * (nb - 1)) + (16 + 64 * (nb - 1)) + 2 * (56 * steps + 24))


def algorithmic_roofline(flops, seconds, note):
    """The dense algorithmic rate of a whole run against the FP64 matrix peak (the executed work
    differs: three real products per complex one, zero coupling slabs skipped, refinement products)."""
    r = flops / seconds
    return {"bound": "mfma", "achieved": r / 1e12, "peak": PEAK["f64"] / 1e12, "unit": "TFLOP/s",
            "frac": r / PEAK["f64"], "traffic": None, "flop_count": "dense algorithmic: " + note}


def executed_roofline(nb, stats, seconds, cmul, note=""):
    """Roofline of the dominant kernel (the batched FP64 products) from the flops the kernels count as they
    execute and the products' event-timed durations, plus the executed fraction of the whole timed region."""
    g = stats["gemm_f64"]
    real = 3 if cmul == 3 else 4
    ex = g["flops"] / (g["total_ms"] * 1e-3) if g["total_ms"] > 0 else 0.0
    step = sum(v["flops"] for v in stats.values())
    return {"bound": "mfma", "kernel": "zgemm_kernel<double> (batched complex FP64 product)", "achieved": ex / 1e12,
            "peak": PEAK["f64"] / 1e12, "unit": "TFLOP/s", "frac": ex / PEAK["f64"], "traffic": None,
            "launches": int(g["launches"]), "avg_launch_ms": g["total_ms"] / max(1, g["launches"]),
            "flop_count": f"{2 * real} M N K per complex product ({real} real products), counted by the kernels",
            "step_executed_tflops": step / seconds / 1e12, "step_frac": step / seconds / PEAK["f64"], "note": note}


def profiled(nb, fn):
    """fn() with the kernels counting their executed flops and the products timed by events; returns
    (fn's result, wall seconds, per-class stats)."""
    import torch
    torch.cuda.synchronize()
    nb.negf_profile_time_classes(1 << nb.KC_NAMES.index("gemm_f64"))
    nb.negf_profile_enable(1)
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stats = nb.negf_profile_read()
    nb.negf_profile_enable(0)
    nb.negf_profile_time_classes(~0)
    return out, dt, stats


def kernel_hash(source="gemm.hip"):
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2602_03438_amd", "csrc", source), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def econv_traffic_per_element():
    """HBM bytes per element of the energy-convolution kernel from the committed counter
    summary, if it was taken on the current source."""
    p = os.path.join(ROOT, "profiles", "econv_traffic.json")
    if not os.path.exists(p):
        return None
    try:
        rec = json.load(open(p))
    except Exception:
        return None
    if rec.get("kernel_sha") != kernel_hash("econv.hip"):
        return None
    return rec.get("bytes_per_item")


def traffic_per_item():
    """HBM bytes per b x b x b complex product of the dominant kernel, from the
    committed rocprofv3 counter summary, if it was taken on the current kernel
    source at this block size."""
    p = os.path.join(ROOT, "profiles", "gemm_f64_traffic.json")
    if not os.path.exists(p):
        return None
    try:
        rec = json.load(open(p))
    except Exception:
        return None
    if rec.get("kernel_sha") != kernel_hash() or rec.get("block") != B:
        return None
    return rec.get("bytes_per_item")


def make_runner(nb, probs, prec, outputs, ws, opts, streams, points, sr_max_iter=40):
    """One step of the hot path: the plain call (opts carries the decimation
    step count), or a plan that splits the batch over worker streams so that
    one half's latency-bound inversion panels overlap the other half's
    products."""
    import torch
    if streams <= 1:
        def run():
            return nb.rgf_lesser_greater(probs, prec, opts=opts, ws=ws, outputs=outputs, lower=True)["info"]
        return run, None
    per = max(1, points // streams)
    plan = nb.Plan(probs, prec, opts=nb.make_options(sr_max_iter=sr_max_iter, inv_nb=opts.inv_nb, cmul=opts.cmul),
                   tunings=[(B, opts.gemm_tile, opts.gemm_tile_f32, opts.inv_nb, per)], n_streams=streams)
    info = torch.zeros(points, dtype=torch.int32, device="cuda")

    def run():
        plan.execute(outputs, info, use_graph=False)
        return info
    return run, plan


def run_steps(nb, probs, batches, prec, steps, warmup, runner, profile=False, time_mask=~0):
    """warmup + steps steps; the last `steps` timed.  With profile the kernels count their
    executed flops (every class) and the classes in time_mask get a timing event pair per
    launch (each pair costs host time: timing every class of an RGF call slows it ~4 %)."""
    import torch
    n_done = 0
    info = None
    failures = []
    for k in range(warmup + steps):
        if k == warmup:
            torch.cuda.synchronize()
            if profile:
                nb.negf_profile_time_classes(time_mask)
                nb.negf_profile_enable(1)
            t0 = time.perf_counter()
        probs[0].energies.copy_(torch.from_numpy(batches[k % len(batches)]).to("cuda"))
        info = runner()
        if k >= warmup:
            n_done += probs[0].n_e
            bad = info.cpu().numpy()
            for q in np.nonzero(bad)[0]:
                failures.append((float(batches[k % len(batches)][q]), int(bad[q])))
        torch.cuda.synchronize()
        log(f"  prec={prec} step {k + 1}/{warmup + steps} done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stats = None
    if profile:
        stats = nb.negf_profile_read()
        nb.negf_profile_enable(0)
        nb.negf_profile_time_classes(~0)
    return dt, n_done, {"info": info, "failures": failures}, stats


ORACLE_NAMES = ("GR_diag", "GR_upper", "GR_lower", "GL_diag", "GL_upper")


def point_outputs(nb, probs, outputs, batch0, runner):
    """One untimed step on the first energy batch; the host copy of the outputs
    of its middle point (the point the CPU oracle solves)."""
    import torch
    probs[0].energies.copy_(torch.from_numpy(batch0).to("cuda"))
    info = runner()
    torch.cuda.synchronize()
    k0 = len(batch0) // 2
    views = nb._views(outputs, probs)
    return {n: views[n][0][k0].cpu().numpy() for n in ORACLE_NAMES}, int(info[k0].item())


def errors_vs_oracle(pt, ref):
    return {n: float(np.linalg.norm(pt[n] - getattr(ref, n)) / np.linalg.norm(getattr(ref, n))) for n in ORACLE_NAMES}


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
    ap.add_argument("--points", type=int, default=128,
                    help="energy points per step (128 at b=512 takes ~200 GiB of the 288 GB HBM)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-chosen", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="serinv workload: skip the graph-replayed timings")
    ap.add_argument("--gemm-f32", action="store_true", help="gemm workload: the single-precision product kernel")
    ap.add_argument("--inv-nb", type=int, default=0, help="inversion panel width (0: tuned)")
    ap.add_argument("--cmul", type=int, choices=[3, 4], default=3,
                    help="real products per complex double product (3: Gauss's method)")
    ap.add_argument("--workload", choices=["ribbon", "uneven", "learned", "gemm", "serinv", "econv", "scba", "small",
                                           "scattering"],
                    default="ribbon",
                    help="ribbon: the headline Nb=60 b=512 measurement; uneven: six devices of different block "
                         "shapes x 4 k-points in one plan; learned: the MLP-seeded lead decimation; gemm: the "
                         "dominant product kernel alone through negf_zgemm_batched at the headline's block size "
                         "and batch (for hardware counters); serinv: few energies per call, plain RGF against the "
                         "partitioned inversion; econv: the energy convolution of Eq. (3) and the energy/element "
                         "layout change over one GPU's share of the selected entries; scba: the self-consistent "
                         "loop of Fig. 1 at the headline device; small: G^R and T of the small ballistic devices "
                         "(Nb=32, b=8) at every point against the oracle; scattering: G^R, G^<, G^> with "
                         "scattering self-energies at 4 k-points x 512 energies")
    ap.add_argument("--econv-cpu-elements", type=int, default=8192,
                    help="elements the oracle computes for the econv workload's cpu_baseline")
    ap.add_argument("--econv-elements", type=int, default=1 << 21, help="elements (matrix entries) in the econv "
                    "workload")
    ap.add_argument("--gemm-batch", type=int, default=256, help="products per launch in the gemm workload")
    ap.add_argument("--scba-energies", type=int, default=64, help="energies of the scba workload's uniform grid")
    ap.add_argument("--scattering-energies", type=int, default=512, help="energies per k-point of the scattering "
                                                                          "workload")
    ap.add_argument("--scattering-batch", type=int, default=64, help="points per call in the scattering workload")
    ap.add_argument("--scba-freqs", type=int, default=17, help="bath frequencies of the scba workload")
    ap.add_argument("--scba-kpoints", type=int, default=1, help="transverse momenta of the scba workload (k = pi j / 4; "
                                                             "the self-energies are shared, built from their average)")
    ap.add_argument("--scba-strength", type=float, default=0.05, help="bath strength of the scba workload")
    ap.add_argument("--scba-memory", type=int, default=0, help="Anderson memory of the scba workload (0: linear "
                    "mixing at 0.5; 1..4: Anderson mixing at 1.0, with 4 M + 4 more [energies][Nb][b][b] "
                    "arrays of workspace)")
    ap.add_argument("--scba-tol", type=float, default=0.0, help="stopping tolerance of the scba workload's timed "
                    "call (0: exactly --steps iterations)")
    ap.add_argument("--serinv-points", default="1,2,4,8", help="energy points per call in the serinv workload")
    ap.add_argument("--serinv-parts", default="4,8", help="partition counts in the serinv workload")
    ap.add_argument("--uneven-points", type=int, default=8, help="energies per (device, k) in the uneven workload "
                    "(with --uneven-queue: the slots per (device, k) that the task lists stream through)")
    ap.add_argument("--uneven-queue", action="store_true",
                    help="the whole uneven workload: 2048 energies x 4 k = 8192 points (grid energy e on device "
                         "e mod 6) streamed through the plan by the device-side point queue")
    ap.add_argument("--uneven-grid", type=int, default=2048, help="grid energies of --uneven-queue (x 4 k points)")
    ap.add_argument("--uneven-plain", action="store_true",
                    help="uneven workload in plain FP64 instead of the refined single-product form")
    ap.add_argument("--uneven-batch", type=int, default=0,
                    help="points per chunk in the uneven workload (0: all points of a block shape in one chunk)")
    ap.add_argument("--streams", type=int, default=None,
                    help="worker streams the batch is split over (1: the plain call on the current stream); "
                         "default 1 for the ribbon workload, 4 for the uneven one")
    ap.add_argument("--sr-max-iter", type=int, default=40,
                    help="decimation steps enqueued per call (converged points are masked out of later steps)")
    ap.add_argument("--learned-energies", type=int, default=250, help="training energies per lead")
    ap.add_argument("--learned-eval", type=int, default=256, help="evaluation energies per held-out lead")
    ap.add_argument("--learned-b", type=int, default=512)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="before the run, copy one buffer of this many MiB (a plain copy kernel of known size, "
                         "the reference for hardware byte counters)")
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
    if args.calibrate_copy > 0:
        # one streaming elementwise kernel: reads and writes exactly N bytes each
        src = torch.ones(args.calibrate_copy << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        log(f"calibration copy of {args.calibrate_copy} MiB done")
        del src, dst
    if args.workload == "gemm":
        return bench_gemm(args)
    if args.workload == "serinv":
        return bench_serinv(args)
    if args.workload == "econv":
        return bench_econv(args)
    if args.workload == "scba":
        return bench_scba(args)
    if args.workload == "small":
        return bench_small(args)
    if args.workload == "scattering":
        return bench_scattering(args)
    if args.workload == "uneven":
        # four worker streams (the hardware queues HIP gives a process by default); each device
        # shape's points form one chunk (see --uneven-batch)
        args.streams = args.streams or 4
        return bench_uneven(args)
    args.streams = args.streams or 1
    if args.workload == "learned":
        return bench_learned(args)
    log("generating the Nb=60 b=512 slab device ...")
    dev = w.slab_device(NB, B, SEED)
    batches = energy_batches(args.points)
    gdev = nb.DeviceOnGPU(dev)
    prob = nb.Problem(gdev, batches[0], eta=ETA, mu_l=MU_L, mu_r=MU_R, kT=KT)
    probs = [prob]
    from paper_2602_03438_amd import autotune
    tuned = autotune.lookup(B, args.cmul)
    opts = nb.make_options(inv_nb=args.inv_nb or tuned["inv_nb"], cmul=args.cmul, gemm_tile=tuned["gemm_tile"],
                           gemm_tile_f32=tuned["gemm_tile_f32"], sr_max_iter=args.sr_max_iter)
    ws = nb.Workspace()
    outputs = nb._rgf_outputs(probs, True, False, True)
    torch.cuda.synchronize()

    log(f"plain FP64, {args.streams} stream(s) ...")
    runner, plan = make_runner(nb, probs, nb.PLAIN_FP64, outputs, ws, opts, args.streams, args.points,
                               args.sr_max_iter)
    # timed steps: timing events on the dominant kernel class only (the products), flop counters on all
    dt, n_pts, res, stats = run_steps(nb, probs, batches, nb.PLAIN_FP64, args.steps, args.warmup, runner,
                                      profile=True, time_mask=1 << nb.KC_NAMES.index("gemm_f64"))
    # one more (untimed) step with every class timed, for the step's breakdown by kernel class
    _, _, _, class_stats = run_steps(nb, probs, batches, nb.PLAIN_FP64, 1, 0, runner, profile=True)
    value = n_pts / dt
    n_valid = n_pts - len(res["failures"])
    g = stats["gemm_f64"]
    # the library counts the flops the matrix cores execute: a complex product of
    # M x K by K x N takes four real products (8 M N K flop) or, in Gauss's form,
    # three (6 M N K flop; the operand sums are O(MK + KN) and not counted).  The
    # conventional complex count 8 M N K is reported beside it as zgemm_equiv_tflops.
    real_products = 3 if args.cmul == 3 else 4
    executed = g["flops"] / (g["total_ms"] * 1e-3) if g["total_ms"] > 0 else 0.0
    launches = max(1, g["launches"])
    per_item = traffic_per_item()
    items_per_launch = g["flops"] / launches / (2.0 * real_products * B ** 3)
    traffic = per_item * items_per_launch if per_item else None
    # every class's executed flops over the whole timed region (the step, not just the products)
    step_flops = sum(v["flops"] for v in stats.values())
    roof = {"bound": "mfma", "kernel": "zgemm_kernel<double> (batched complex FP64 product)",
            "achieved": executed / 1e12, "peak": PEAK["f64"] / 1e12, "unit": "TFLOP/s",
            "frac": executed / PEAK["f64"], "traffic": traffic,
            "launches": int(g["launches"]), "avg_launch_ms": g["total_ms"] / launches,
            "flops_per_launch": g["flops"] / launches,
            "flop_count": f"{2 * real_products} M N K per complex product ({real_products} real products)",
            "zgemm_equiv_tflops": executed * 4.0 / real_products / 1e12,
            "step_executed_tflops": step_flops / dt / 1e12,
            "step_frac": step_flops / dt / PEAK["f64"],
            "items_per_launch": items_per_launch,
            "traffic_bytes_per_item": per_item,
            "algorithmic_bytes_per_item": 3 * 16 * B * B,
            "note": "average over the launches of both worker streams; launches overlap, so per-launch durations "
                    "include time shared with the other stream" if args.streams > 1 else ""}
    kstats = {k: {"launches": int(v["launches"]), "total_ms": round(v["total_ms"], 3),
                  "tflops": (v["flops"] / (v["total_ms"] * 1e-3) / 1e12) if v["total_ms"] > 0 and v["flops"] else None}
              for k, v in class_stats.items() if v["launches"]}

    # one untimed step on the first energy batch: the middle point's outputs (compared with the
    # oracle below) and 8 points spread over the batch (compared with the other forms)
    at_oracle = {"plain_fp64": point_outputs(nb, probs, outputs, batches[0], runner)}
    # a property of every point of that step: the spectral current is the same at all interfaces
    cur = nb.observables(probs, outputs, dos=False)["current"][0].cpu().numpy()
    scale = float(np.abs(cur).max())
    per_pt = np.abs(cur - cur[:, :1]).max(axis=1) / scale
    conservation = {"points": int(cur.shape[0]), "interfaces": int(cur.shape[1]),
                    "max_spread_rel_to_largest_current": float(per_pt.max()),
                    "median_spread": float(np.median(per_pt)),
                    "note": "negf_observables on the first energy batch's outputs (all points, flagged ones "
                            "included); exact conservation in exact arithmetic"}
    # decimation steps per point and lead on that batch (negf_obc_surface with the step's options): the
    # Sancho-Rubio step histogram and the points whose surface Green's function is flagged
    decim = {}
    for side, name in ((0, "left"), (1, "right")):
        o = nb.obc_surface(probs, side, opts=opts, ws=ws)
        its = o["iters"].cpu().numpy()
        vals, counts = np.unique(its, return_counts=True)
        decim[name] = {"mean": float(its.mean()), "min": int(its.min()), "max": int(its.max()),
                       "histogram": {str(int(v)): int(c) for v, c in zip(vals, counts)},
                       "flagged": int(np.count_nonzero(o["info"].cpu().numpy())),
                       "max_residual": float(o["resid"].max().item())}
        del o
    if plan:
        plan.close()          # its workspace is not needed by the runs below
    chosen = None
    if not args.no_chosen:
        # (a copy of every point's diagonal blocks would not fit next to the refined form's workspace)
        views = nb._views(outputs, probs)
        sample = torch.from_numpy(np.linspace(0, args.points - 1, 8).astype(np.int64)).cuda()
        plain_GR = views["GR_diag"][0].index_select(0, sample)
        plain_GL = views["GL_diag"][0].index_select(0, sample)
        out = {}
        for prec, name in ((nb.FP32_REFINE, "fp32_refine"), (nb.FP32_NOREFINE, "fp32_norefine")):
            log(f"{name} ...")
            runner_c, plan_c = make_runner(nb, probs, prec, outputs, ws, opts, args.streams, args.points,
                                             args.sr_max_iter)
            dtc, nc, resc, st = run_steps(nb, probs, batches, prec, args.steps, args.warmup, runner_c, profile=True,
                                          time_mask=(1 << nb.KC_NAMES.index("gemm_f64")) | (1 << nb.KC_NAMES.index("gemm_f32")))
            at_oracle[name] = point_outputs(nb, probs, outputs, batches[0], runner_c)   # first batch again
            gr = views["GR_diag"][0].index_select(0, sample)
            gl = views["GL_diag"][0].index_select(0, sample)
            if plan_c:
                plan_c.close()
            eR = (torch.linalg.vector_norm(gr - plain_GR) / torch.linalg.vector_norm(plain_GR)).item()
            eL = (torch.linalg.vector_norm(gl - plain_GL) / torch.linalg.vector_norm(plain_GL)).item()
            # matrix-core time at peak of the executed products
            ideal = st["gemm_f64"]["flops"] / PEAK["f64"] + st["gemm_f32"]["flops"] / PEAK["f32"]
            out[name] = {"value": nc / dtc, "ms_per_step": dtc / args.steps * 1e3,
                         "single_precision_products": "backward retarded sweep only, each block followed by one "
                                                      "FP64 residual correction; forward retarded and both lesser "
                                                      "sweeps, inversions and decimation in FP64"
                         if name == "fp32_refine" else "every sweep product (no correction)",
                         "err_vs_plain_GR_diag": eR, "err_vs_plain_GL_diag": eL, "err_sample_points": 8,
                         "gemm_f32_tflops": (st["gemm_f32"]["flops"] / (st["gemm_f32"]["total_ms"] * 1e-3) / 1e12)
                         if st["gemm_f32"]["total_ms"] > 0 else None,
                         "mixed_peak_frac_of_products": ideal / ((st["gemm_f64"]["total_ms"] + st["gemm_f32"]["total_ms"]) * 1e-3)
                         if (st["gemm_f64"]["total_ms"] + st["gemm_f32"]["total_ms"]) > 0 else None}
        chosen = out

    cpu = None
    vs_oracle = None
    if not args.no_cpu:
        log("CPU oracle on one point ...")
        cpu, ref, E0 = cpu_baseline(dev, batches[0])
        # every form's outputs at the same point against the oracle (all output kinds)
        vs_oracle = {"E": E0, "oracle_lead_residuals": [ref.lead_l.residual, ref.lead_r.residual]}
        for name, (pt, inf) in at_oracle.items():
            vs_oracle[name] = {"info": inf, **errors_vs_oracle(pt, ref)}

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
                   "streams": args.streams, "inversion_panel": opts.inv_nb, "gemm_tile": opts.gemm_tile,
                   "sr_max_iter": args.sr_max_iter,
                   "real_products_per_complex_product": args.cmul,
                   "outputs": "G^R diag/upper/lower + G^< diag/upper in HBM"},
        "valid_points_per_s": n_valid / dt,
        "info_nonzero": len(res["failures"]),
        "failures": res["failures"][:8],
        "roofline": roof,
        "current_conservation": conservation,
        "decimation_steps": {**decim, "note": "Sancho-Rubio steps per point of the first energy batch, each lead "
                                              "(negf_obc_surface, untimed)"},
        "kernels": kstats,
        "kernels_note": "one extra untimed step with every kernel class timed (the timed steps time the products only)",
        "chosen_form": chosen,
        "errors_vs_oracle": vs_oracle,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def bench_gemm(args):
    """The dominant kernel alone: batched b x b x b complex FP64 products (Gauss's
    three-product form, the headline's tile) launched through negf_zgemm_batched,
    timed with HIP events on the launching stream.  Used for hardware counters
    of the product kernel (MFMA activity, HBM bytes)."""
    import torch
    from paper_2602_03438_amd import autotune
    from paper_2602_03438_amd import binding as nb
    tuned = autotune.lookup(B, args.cmul)
    batch = args.gemm_batch
    g = torch.Generator(device="cuda").manual_seed(7)
    A = torch.randn(batch, B, B, dtype=torch.complex128, device="cuda", generator=g)
    Bm = torch.randn(batch, B, B, dtype=torch.complex128, device="cuda", generator=g)
    Cm = torch.zeros(batch, B, B, dtype=torch.complex128, device="cuda")
    f32 = args.gemm_f32
    prec = 1 if f32 else (2 if args.cmul == 3 else 0)
    tile = tuned["gemm_tile_f32"] if f32 else tuned["gemm_tile"]
    for _ in range(args.warmup):
        nb.zgemm(A, Bm, Cm, prec=prec, tile=tile)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(s)
        nb.zgemm(A, Bm, Cm, prec=prec, tile=tile)
        ev[k][1].record(s)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = [a.elapsed_time(b) for a, b in ev]
    real_products = 3 if (args.cmul == 3 and not f32) else 4
    flops = 2.0 * real_products * B ** 3 * batch
    a0, b0, c0 = A[0].cpu().numpy(), Bm[0].cpu().numpy(), Cm[0].cpu().numpy()
    ref = a0 @ b0
    err = float(np.linalg.norm(c0 - ref) / np.linalg.norm(ref))
    avg = float(np.mean(ms))
    peak = PEAK["f32"] if f32 else PEAK["f64"]
    line = {"metric": f"batched complex {'FP32' if f32 else 'FP64'} product (b x b x b), executed TFLOP/s",
            "value": flops / (avg * 1e-3) / 1e12,
            "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True, "dtype": "f32" if f32 else "f64",
            "data": "synthetic",
            "config": {"workload": f"{batch} products of {B}x{B} complex128 per launch"
                                   f"{' (operands rounded to single precision at staging)' if f32 else ''}, "
                                   f"tile {tile}, {real_products} real products per complex product"},
            "avg_launch_ms": avg, "min_launch_ms": float(np.min(ms)),
            f"frac_of_{'fp32' if f32 else 'fp64'}_peak": flops / (avg * 1e-3) / peak,
            "algorithmic_bytes_per_launch": 3 * 16 * B * B * batch, "rel_err_vs_torch_item0": err}
    print(json.dumps(line), flush=True)


def bench_econv(args):
    """Energy convolution of Eq. (3) over one GPU's share of the selected entries: n_el
    elements x 1024 energies of G and of a two-sided kernel W (1024 frequencies), by
    zero-padded FFTs of length 2048 per element, read and written energy-major; and the
    energy/element layout change of the same array.  Roofline: HBM (every byte of G, W
    and B moves once)."""
    import torch
    from paper_2602_03438_amd import binding as nb
    n_e, n_w, k0, n_el = N_GRID, N_GRID, N_GRID // 2, args.econv_elements
    g = torch.Generator(device="cuda").manual_seed(11)
    G = torch.randn(n_e, n_el, dtype=torch.complex128, device="cuda", generator=g)
    W = torch.randn(n_w, n_el, dtype=torch.complex128, device="cuda", generator=g)
    B = torch.empty_like(G)
    ws = nb.Workspace()
    s = torch.cuda.current_stream()

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
        for a, b in ev:
            a.record(s)
            fn()
            b.record(s)
        torch.cuda.synchronize()
        return float(np.mean([a.elapsed_time(b) for a, b in ev]))

    ms = timed(lambda: nb.energy_convolution(G, W, k0, 1.0, out=B, ws=ws))
    # a sampled element against the plain sum, computed here on the host
    x = n_el // 3
    Gx, Wx, Bx = G[:, x].cpu().numpy(), W[:, x].cpu().numpy(), B[:, x].cpu().numpy()
    ref = np.convolve(Gx, Wx)[k0:k0 + n_e]
    err = float(np.linalg.norm(Bx - ref) / np.linalg.norm(ref))
    cpu = None
    if not args.no_cpu:
        # the oracle (the sum over k as written) on a contiguous run of elements of the same arrays
        from oracle import econv as oec
        n_s = min(args.econv_cpu_elements, n_el)
        x0 = n_el // 2
        Gs, Ws, Bs = (X[:, x0:x0 + n_s].cpu().numpy() for X in (G, W, B))
        t0 = time.perf_counter()
        ref_s = oec.energy_convolution(Gs, Ws, k0, 1.0)
        dt = time.perf_counter() - t0
        cpu = dict(value=n_s * n_e / dt, unit="element-energies/s", cores=1, kind="oracle",
                   sample=f"{n_s} elements x {n_e} energies (elements {x0}..{x0 + n_s - 1}), the sum over the "
                          f"{n_w} kernel frequencies in NumPy complex128 (single-threaded element-wise)",
                   seconds=dt, host_cpus=os.cpu_count(),
                   rel_err_gpu_vs_oracle=float(np.linalg.norm(Bs - ref_s) / np.linalg.norm(ref_s)))
    del W
    torch.cuda.empty_cache()
    T = torch.empty(n_el, n_e, dtype=torch.complex128, device="cuda")
    ms_t = timed(lambda: nb.transpose(G, out=T))
    ok_t = bool(torch.equal(T[x], G[:, x]))
    bytes_conv = 16.0 * n_el * (2 * n_e + n_w)
    bytes_t = 32.0 * n_el * n_e
    L = 2048
    fft_flops = 3 * 5.0 * L * np.log2(L) * n_el + 6.0 * L * n_el
    line = {"metric": "energy convolution of Eq. (3) by FFT, elements x energies per second",
            "value": n_el * n_e / (ms * 1e-3), "unit": "element-energies/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"{n_el} elements x {n_e} energies, two-sided kernel of {n_w} frequencies "
                                   f"(k0 = {k0}), FFT length {L}, energy-major in and out"},
            "roofline": {"bound": "hbm", "achieved": bytes_conv / (ms * 1e-3) / 1e9, "peak": 8000.0, "unit": "GB/s",
                         "frac": bytes_conv / (ms * 1e-3) / 8e12,
                         "traffic": (per_el * n_el if (per_el := econv_traffic_per_element()) else None),
                         "algorithmic_bytes_per_launch": bytes_conv, "fft_tflops": fft_flops / (ms * 1e-3) / 1e12},
            "rel_err_sampled_element_vs_plain_sum": err,
            "cpu_baseline": cpu,
            "transpose": {"ms": ms_t, "gb_per_s": bytes_t / (ms_t * 1e-3) / 1e9, "frac_of_hbm": bytes_t / (ms_t * 1e-3) / 8e12,
                          "rows": n_e, "cols": n_el, "sampled_column_exact": ok_t}}
    print(json.dumps(line), flush=True)


def bench_small(args):
    """The small ballistic workload: a random device Nb = 32, b = 8 (seed 1), the 1D chain (b = 1,
    Nb = 32), the chain folded into cells of 8 sites and a periodic random wire (b = 8, seed 1), each at
    64 energies in [-3, 3], eta = 1e-6: 256 points per step, G^R (every block) and the transmission per
    point through negf_rgf_retarded and negf_transmission, both leads.  Timed eagerly and as a captured
    graph replayed (each replay checked equal to the eager result); plain FP64 and the refined
    single-product form of the retarded call.  Every point is compared with the oracle (G^R diagonal
    and T), the chains with the closed form (T = 1 inside |E| < 2t, 0 outside) and the wire with
    integers; the oracle over all 256 points is the CPU baseline."""
    import torch
    import workloads as w
    from oracle import leads as oleads
    from oracle import rgf as orgf
    from paper_2602_03438_amd import binding as nb
    eta = 1e-6
    E = np.linspace(-3.0, 3.0, 64)
    devs = {"random": w.random_device(32, 8, 1), "chain": w.chain_device(32),
            "folded_chain": w.folded_chain_device(32, 8), "wire": w.periodic_wire_device(32, 8, 1)}
    probs = [nb.Problem(nb.DeviceOnGPU(d), E, eta=eta, mu_l=MU_L, mu_r=MU_R, kT=KT) for d in devs.values()]
    npts = len(probs) * E.size
    # the decimation steps enqueued per call (the leads here need at most 27 at eta = 1e-6)
    sopts = nb.make_options(sr_max_iter=args.sr_max_iter)
    ws_r, ws_t = nb.Workspace(), nb.Workspace()
    res = {}
    for prec, name in ((nb.PLAIN_FP64, "plain"), (nb.FP32_REFINE, "fp32_refine")):
        outs = nb._rgf_outputs(probs, False, False, True)

        def step():
            r = nb.rgf_retarded(probs, prec, opts=sopts, ws=ws_r, outputs=outs)
            t = nb.transmission(probs, opts=sopts, ws=ws_t)
            return r["info"], t

        for _ in range(max(1, args.warmup)):
            step()
        torch.cuda.synchronize()
        reps = 20 * args.steps
        t0 = time.perf_counter()
        for _ in range(reps):
            info, tr = step()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        gd = nb._views(outs, probs)["GR_diag"]
        eager = {k: v.clone() for k, v in outs.items() if v is not None}
        T_eager = tr["T"].clone()
        # the same step captured once and replayed
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            step()
        torch.cuda.current_stream().wait_stream(side)
        with torch.cuda.graph(g):
            _, tg = step()
        torch.cuda.synchronize()
        same = True
        for _ in range(2):
            for v in outs.values():
                if v is not None:
                    v.zero_()
            g.replay()
            torch.cuda.synchronize()
            same = same and all(torch.equal(outs[k], eager[k]) for k in eager) and torch.equal(tg["T"], T_eager)
        t0 = time.perf_counter()
        for _ in range(reps):
            g.replay()
        torch.cuda.synchronize()
        dtg = (time.perf_counter() - t0) / reps
        del g
        res[name] = {"points_per_s": npts / dt, "ms_per_step": dt * 1e3, "graph_points_per_s": npts / dtg,
                     "graph_ms_per_step": dtg * 1e3, "graph_replays_equal_eager": bool(same),
                     "info_nonzero": int(torch.count_nonzero(info).item()), "gd": [x.cpu().numpy() for x in gd],
                     "T": T_eager.cpu().numpy()}
        log(f"small workload {name}: {npts / dt:.0f} points/s eager, {npts / dtg:.0f} points/s graph-replayed "
            f"(replays equal to eager: {same})")
    # the oracle at every point: G^R diagonal and T; the CPU baseline is its time.  A device without
    # broadening inside (leads at eta = 1e-6 only) is nearly singular at energies of states localised
    # away from the leads, so each point's G^R error is read against the oracle's own spread there
    # (its change when every inversion is Newton-refined)
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests"))
    from helpers import refined_inversions
    t0 = time.perf_counter()
    refs = [[orgf.solve_point(d, float(e), eta, MU_L, MU_R, KT, lesser_greater=False, want_T=True) for e in E]
            for d in devs.values()]
    cpu_s = time.perf_counter() - t0
    with refined_inversions():
        refs2 = [[orgf.solve_point(d, float(e), eta, MU_L, MU_R, KT, lesser_greater=False) for e in E]
                 for d in devs.values()]
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    spread = [[rel(refs2[q][k].GR_diag, refs[q][k].GR_diag) for k in range(E.size)] for q in range(len(devs))]
    errs = {}
    for name, bar in (("plain", 1e-10), ("fp32_refine", 1e-6)):
        e_all, e_stable, n_stable, t_err = [], [], 0, 0.0
        for q, d in enumerate(devs):
            for k in range(E.size):
                err = rel(res[name]["gd"][q][k], refs[q][k].GR_diag)
                e_all.append(err)
                if 4.0 * spread[q][k] <= bar:
                    e_stable.append(err)
                t_err = max(t_err, abs(float(res[name]["T"][q * E.size + k]) - refs[q][k].T))
        errs[name] = {"GR_diag_max_rel_all_points": max(e_all), "GR_diag_median_rel": float(np.median(e_all)),
                      "bar": bar, "points_where_oracle_stable_to_bar": len(e_stable),
                      "GR_diag_max_rel_stable_points": max(e_stable) if e_stable else None,
                      "stable_points_meeting_bar": int(sum(e <= bar for e in e_stable)),
                      "oracle_spread_max": float(np.max(spread)), "T_max_abs": t_err}
    T_plain = res["plain"]["T"].reshape(len(devs), E.size)
    inband = np.abs(E) < 2.0
    dev_int = np.abs(T_plain[3] - np.round(T_plain[3]))
    closed = {"chain_T_vs_step": float(np.abs(T_plain[1] - inband).max()),
              "folded_chain_T_vs_step": float(np.abs(T_plain[2] - inband).max()),
              "wire_T_vs_integer_max": float(dev_int.max()), "wire_T_vs_integer_median": float(np.median(dev_int)),
              "wire_points_within_1e-6_of_an_integer": int(np.count_nonzero(dev_int < 1e-6)),
              "wire_note": "T steps between integers at the wire's subband edges; within ~eta of an edge it is not "
                           "an integer"}
    sr = {}
    for q, d in enumerate(devs):
        it = [oleads.lead_self_energy(devs[d], side, float(e), eta).iters for side in (0, 1) for e in E[::8]]
        sr[d] = {"oracle_mean_steps": float(np.mean(it)), "oracle_max_steps": int(np.max(it))}
    for name in res:
        res[name].pop("gd")
        res[name].pop("T")
    # dense algorithmic flops of one step: per point G^R (8 + 56 (nb - 1)) b^3, the transmission's corner
    # recursion 16 (nb - 1) b^3 and both leads 2 (56 K + 24) b^3 with K = 30 steps
    step_flops = E.size * sum(float(d.b) ** 3 * ((8 + 56 * (d.nb - 1)) + 16 * (d.nb - 1) + 2 * (56 * 30 + 24))
                              for d in devs.values())
    best = res["plain"]["graph_points_per_s"]
    rate = step_flops / (res["plain"]["graph_ms_per_step"] * 1e-3)
    line = {"metric": "energy points/s, G^R + transmission of the small ballistic workload (Nb=32, b=8)",
            "value": best, "unit": "energy points/s", "n_gpus": 1, "steps": 20 * args.steps, "warmup": args.warmup,
            "ms_per_step": res["plain"]["graph_ms_per_step"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "random device Nb=32 b=8 (seed 1), 1D chain Nb=32 b=1, chain folded into cells "
                                   "of 8 (Nb=32), periodic random wire Nb=32 b=8; 64 energies in [-3, 3] each, "
                                   "eta=1e-6; one step = negf_rgf_retarded + negf_transmission over the 256 points, "
                                   "value = graph-replayed plain FP64", "sr_max_iter": args.sr_max_iter},
            "forms": res, "errors_vs_oracle_every_point": errs, "closed_forms": closed, "decimation_steps": sr,
            "roofline": {"bound": "mfma", "achieved": rate / 1e12, "peak": PEAK["f64"] / 1e12, "unit": "TFLOP/s",
                         "frac": rate / PEAK["f64"], "traffic": None,
                         "note": "blocks of 8 x 8 (and 1 x 1): every launch is a few microseconds of latency; the "
                                 "fraction of the matrix peak is tiny by construction"},
            "cpu_baseline": {"value": npts / cpu_s, "unit": "energy points/s", "cores": os.cpu_count(),
                             "kind": "oracle", "sample": f"all {npts} points (G^R sweeps, both leads, T) in NumPy "
                                                         f"complex128", "seconds": cpu_s}}
    print(json.dumps(line), flush=True)


def bench_scattering(args):
    """The scattering workload: the benchmark device (Nb = 60, b = 512) with block-diagonal scattering
    self-energies (norm 0.01, seed 3) at 4 transverse momenta k = 0, pi/4, pi/2, 3 pi/4 (H_ii(k), seed 31)
    x --scattering-energies energies on [-1.5, 1.5]: G^R (diagonal, upper, lower), G^< and G^>
    (diagonal, upper) and both leads per point, in calls of --scattering-batch points (one k each);
    plain FP64 and the refined single-product form, each over the whole grid.  The point in the middle
    of the k = 0 grid is compared with the oracle for every output (with the oracle's own spread under
    refined inversions), and its oracle time is the CPU baseline."""
    import torch
    import workloads as w
    from oracle import rgf as orgf
    from paper_2602_03438_amd import autotune
    from paper_2602_03438_amd import binding as nb
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests"))
    from helpers import oracle_spread
    log("generating the Nb=60 b=512 device with scattering self-energies and its 4 k-points ...")
    base = w.scattering_self_energies(w.slab_device(NB, B, SEED), 3)
    ks = [np.pi * j / 4 for j in range(4)]
    devs = [w.k_device(base, 31, k) for k in ks]
    gdevs = [nb.DeviceOnGPU(d) for d in devs]
    E = np.linspace(-1.5, 1.5, args.scattering_energies)
    nbat = args.scattering_batch
    t = autotune.lookup(B, args.cmul)
    opts = nb.make_options(inv_nb=args.inv_nb or t["inv_nb"], cmul=args.cmul, gemm_tile=t["gemm_tile"],
                           gemm_tile_f32=t["gemm_tile_f32"], sr_max_iter=args.sr_max_iter)
    probs = [nb.Problem(g, E[:nbat], eta=ETA, mu_l=MU_L, mu_r=MU_R, kT=KT) for g in gdevs]
    ws = nb.Workspace()
    outs = nb._rgf_outputs([probs[0]], True, True, True)
    calls = [(q, e0) for q in range(len(devs)) for e0 in range(0, E.size, nbat)]
    k_mid = E.size // 2
    res = {}
    for prec, name in ((nb.PLAIN_FP64, "plain"), (nb.FP32_REFINE, "fp32_refine")):
        def call(q, e0):
            pr = probs[q]
            pr.energies.copy_(torch.from_numpy(np.ascontiguousarray(E[e0:e0 + nbat])).to("cuda"))
            return nb.rgf_lesser_greater([pr], prec, opts=opts, ws=ws, outputs=outs, greater=True)["info"]
        for _ in range(args.warmup):
            call(0, 0)
        torch.cuda.synchronize()

        def sweep_all():
            bad = 0
            for j, (q, e0) in enumerate(calls):
                bad += int(torch.count_nonzero(call(q, e0)).item())
                if j % 8 == 7:
                    log(f"  scattering {name}: {j + 1}/{len(calls)} calls")
            return bad
        if prec == nb.PLAIN_FP64:
            n_bad, dt, stats = profiled(nb, sweep_all)
            roof = executed_roofline(nb, stats, dt, args.cmul)
        else:
            t0 = time.perf_counter()
            n_bad = sweep_all()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        # the sampled point: k = 0, the middle energy (its call recomputed, untimed)
        call(0, (k_mid // nbat) * nbat)
        torch.cuda.synchronize()
        v = nb._views(outs, [probs[0]])
        pt = {n: v[n][0][k_mid % nbat].cpu().numpy()
              for n in ("GR_diag", "GR_upper", "GR_lower", "GL_diag", "GL_upper", "GG_diag", "GG_upper")}
        res[name] = {"points_per_s": len(calls) * nbat / dt, "seconds": dt, "info_nonzero": n_bad, "pt": pt}
        log(f"scattering {name}: {len(calls) * nbat / dt:.2f} points/s, {n_bad} points flagged")
    names = ("GR_diag", "GR_upper", "GR_lower", "GL_diag", "GL_upper", "GG_diag", "GG_upper")
    log(f"oracle at E = {E[k_mid]:+.4f}, k = 0 ...")
    t0 = time.perf_counter()
    ref = orgf.solve_point(devs[0], float(E[k_mid]), ETA, MU_L, MU_R, KT, greater=True)
    cpu_s = time.perf_counter() - t0
    _, spread = oracle_spread(lambda: orgf.solve_point(devs[0], float(E[k_mid]), ETA, MU_L, MU_R, KT, greater=True),
                              names)
    for name in res:
        pt = res[name].pop("pt")
        res[name]["errors_vs_oracle"] = {n: float(np.linalg.norm(pt[n] - getattr(ref, n)) / np.linalg.norm(getattr(ref, n)))
                                         for n in names}
    res_sr = {"oracle_lead_steps": [ref.lead_l.iters, ref.lead_r.iters],
              "oracle_lead_residuals": [ref.lead_l.residual, ref.lead_r.residual]}
    flops = point_flops(NB, B) + float(B) ** 3 * (16 + 64 * (NB - 1))      # + G^>
    value = res["plain"]["points_per_s"]
    line = {"metric": "energy points/s, RGF G^R + G^< + G^> with scattering self-energies at 4 k-points (Nb=60, b=512)",
            "value": value, "unit": "energy points/s", "n_gpus": 1, "steps": len(calls), "warmup": args.warmup,
            "ms_per_step": res["plain"]["seconds"] / len(calls) * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"nano-ribbon-like slab device Nb={NB} b={B} with block-diagonal scattering "
                                   f"self-energies (norm 0.01), 4 k-points x {E.size} energies on [-1.5, 1.5], "
                                   f"eta={ETA}; one step = one call of {nbat} points (one k)",
                       "real_products_per_complex_product": args.cmul, "sr_max_iter": args.sr_max_iter},
            "forms": res, "sampled_point": {"E": float(E[k_mid]), "k": 0.0, "oracle_spread": spread},
            "decimation": res_sr,
            "roofline": roof,
            "algorithmic": algorithmic_roofline(flops, 1.0 / value,
                                                "G^R + G^< + G^> of one energy point (both leads, 28 decimation "
                                                "steps); above 1 because the executed work is smaller (three real "
                                                "products per complex one, zero coupling slabs skipped)"),
            "cpu_baseline": {"value": 1.0 / cpu_s, "unit": "energy points/s", "cores": os.cpu_count(),
                             "kind": "oracle", "sample": f"1 point (E={E[k_mid]:.4f}, k=0): both leads, G^R, G^<, "
                                                         f"G^> sweeps in NumPy complex128", "seconds": cpu_s}}
    print(json.dumps(line), flush=True)


def bench_scba(args):
    """The self-consistent loop of Fig. 1 around Eq. (1)-(3) at the headline device (Nb = 60,
    b = 512): --scba-energies energies, uniform on [-1.5, 1.5], and a boson bath of --scba-freqs
    frequencies (the grid spacing apart).  An iteration solves every energy (G^R, G^<, G^>, both
    leads), convolves the diagonal blocks of G^< and of G^> with the bath (Eq. (3)), reduces the
    residual, reads it on the host and mixes (linearly, or by Anderson's extrapolation with
    --scba-memory).  --steps iterations are timed as one call with tol = --scba-tol (0: no early
    stop), after --warmup iterations in a call of their own; points/s = energies x iterations
    performed / wall time of the call.  The convolutions are also timed alone, on the
    same arrays, for their share of an iteration."""
    import torch
    import workloads as w
    from paper_2602_03438_amd import autotune
    from paper_2602_03438_amd import binding as nb
    n_e, n_w, nk = args.scba_energies, args.scba_freqs, args.scba_kpoints
    memory = args.scba_memory
    mixing = 1.0 if memory > 0 else 0.5
    k0 = (n_w - 1) // 2
    dev = w.slab_device(NB, B, SEED)
    devs = [dev] if nk == 1 else [w.k_device(dev, 31, np.pi * j / 4) for j in range(nk)]
    E = np.linspace(-1.5, 1.5, n_e)
    dE = float(E[1] - E[0])
    Wl, Wg = w.boson_bath(NB, B, n_w, k0, dE, KT, strength=args.scba_strength)
    gWl, gWg = torch.from_numpy(Wl).cuda(), torch.from_numpy(Wg).cuda()
    del Wl, Wg
    t = autotune.lookup(B, args.cmul)
    opts = nb.make_options(inv_nb=args.inv_nb or t["inv_nb"], cmul=args.cmul, gemm_tile=t["gemm_tile"],
                           gemm_tile_f32=t["gemm_tile_f32"], sr_max_iter=args.sr_max_iter)
    probs = [nb.Problem(nb.DeviceOnGPU(d), E, eta=ETA, mu_l=MU_L, mu_r=MU_R, kT=KT) for d in devs]
    prob = probs if nk > 1 else probs[0]
    ws = nb.Workspace()
    outs = nb._rgf_outputs(probs, True, True, True)
    shape = (n_e, NB, B, B)
    sig = {k: torch.zeros(shape, dtype=torch.complex128, device="cuda") for k in ("sig_r", "sig_l", "sig_g")}
    scale = 1j * dE / (2 * np.pi)
    log(f"scba: {nk} k-point(s) x {n_e} energies x Nb={NB} b={B}, {n_w} bath frequencies; warm-up {args.warmup} "
        f"iteration(s)")
    if args.warmup > 0:
        nb.scba(prob, gWl, gWg, k0, scale, mixing=mixing, tol=0.0, max_iter=args.warmup, opts=opts, ws=ws, outputs=outs,
                sigmas=sig, memory=memory)
    for v in sig.values():
        v.zero_()
    torch.cuda.synchronize()
    log(f"scba: {args.steps} timed iteration(s)")
    r, dt, stats = profiled(nb, lambda: nb.scba(prob, gWl, gWg, k0, scale, mixing=mixing, tol=args.scba_tol,
                                                max_iter=args.steps, opts=opts, ws=ws, outputs=outs, sigmas=sig,
                                                memory=memory))
    its = r["n_iter"]
    log(f"scba: {its} iteration(s) in {dt:.2f} s, residuals {['%.2e' % h for h in r['history']]}")
    # the two convolutions of one iteration, alone
    n_el = NB * B * B
    GL = outs["GL_diag"][: n_e * n_el].view(n_e, n_el)
    GG = outs["GG_diag"][: n_e * n_el].view(n_e, n_el)
    Fl = torch.empty_like(GL)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    s = torch.cuda.current_stream()
    nb.energy_convolution(GL, gWl.view(n_w, n_el), k0, scale, out=Fl, ws=ws)
    ev[0].record(s)
    for _ in range(3):
        nb.energy_convolution(GL, gWl.view(n_w, n_el), k0, scale, out=Fl, ws=ws)
        nb.energy_convolution(GG, gWg.view(n_w, n_el), k0, scale, out=Fl, ws=ws)
    ev[1].record(s)
    torch.cuda.synchronize()
    conv_ms = ev[0].elapsed_time(ev[1]) / 3
    it_ms = dt / its * 1e3
    flops = point_flops(NB, B) + float(B) ** 3 * (16 + 64 * (NB - 1))      # + G^>
    line = {"metric": "self-consistent loop (Fig. 1, Eq. (1)-(3)) at Nb=60, b=512: energy points solved and "
                      "convolved per second",
            "value": nk * n_e * its / dt, "unit": "energy points/s", "n_gpus": 1, "steps": its, "warmup": args.warmup,
            "ms_per_step": it_ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": f"nano-ribbon-like slab device Nb={NB} b={B}, {nk} k-point(s) x {n_e} energies on "
                                   f"[-1.5, 1.5], "
                                   f"boson bath of {n_w} frequencies (strength {args.scba_strength}, kT={KT}), "
                                   f"eta={ETA}, "
                                   + (f"Anderson mixing (memory {memory}, mixing 1.0)" if memory else "mixing 0.5")
                                   + f", tol {args.scba_tol}, one iteration per step",
                       "real_products_per_complex_product": args.cmul, "sr_max_iter": args.sr_max_iter},
            "ms_per_iteration": it_ms, "convolutions_ms_per_iteration": conv_ms,
            "convolution_share": conv_ms / it_ms, "residual_history": r["history"], "status": r["status"],
            "info_nonzero": int(torch.count_nonzero(r["info"]).item()),
            "roofline": executed_roofline(nb, stats, dt, args.cmul, "timed iterations, products event-timed"),
            "algorithmic": algorithmic_roofline(flops, it_ms * 1e-3 / (nk * n_e),
                                                "G^R + G^< + G^> of one energy point (both leads, 28 decimation "
                                                "steps) per (iteration time / energies); the convolutions add no "
                                                "flops to the count"),
            "cpu_baseline": None,
            "cpu_baseline_note": "not taken: one oracle iteration at this shape solves every energy point "
                                 "(about 1.4e12 flop each) on the host"}
    print(json.dumps(line), flush=True)


def bench_serinv(args):
    """Few energy points per call at the headline shape (Nb = 60, b = 512): the plain
    RGF call (batch = the points) against the partitioned inversion with P partitions
    (batch = P x the points), G^R + G^<, both leads included; points/s per case."""
    import torch
    import workloads as w
    from paper_2602_03438_amd import autotune
    from paper_2602_03438_amd import binding as nb
    # the interacting device (scattering self-energies of norm 0.01 on every block): the partitioned
    # elimination needs the broadening inside the device that such self-energies give
    dev = w.scattering_self_energies(w.slab_device(NB, B, SEED), 3)
    gdev = nb.DeviceOnGPU(dev)
    t = autotune.lookup(B, args.cmul)
    opts = nb.make_options(inv_nb=args.inv_nb or t["inv_nb"], cmul=args.cmul, gemm_tile=t["gemm_tile"],
                           gemm_tile_f32=t["gemm_tile_f32"], sr_max_iter=args.sr_max_iter)
    grid = np.linspace(-1.5, 1.5, N_GRID)
    res = []
    for npts in [int(x) for x in args.serinv_points.split(",")]:
        E = grid[np.linspace(0, N_GRID - 1, npts + 2).astype(int)[1:-1]]
        prob = nb.Problem(gdev, E, eta=ETA, mu_l=MU_L, mu_r=MU_R, kT=KT)
        ws = nb.Workspace()
        outs = nb._rgf_outputs([prob], True, False, True)
        cases = [("rgf", None)] + [("serinv", int(p)) for p in args.serinv_parts.split(",")]
        first = None
        for name, parts in cases:
            def run():
                if parts is None:
                    return nb.rgf_lesser_greater([prob], opts=opts, ws=ws, outputs=outs)["info"]
                return nb.serinv_lesser_greater(prob, parts, opts=opts, ws=ws, outputs=outs)["info"]
            for _ in range(args.warmup):
                run()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                info = run()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / args.steps
            # every output of the first point next to the plain RGF call's
            pt = {k: outs[k][:(NB if k.endswith("diag") else NB - 1) * B * B].clone()
                  for k in ("GR_diag", "GR_upper", "GL_diag", "GL_upper")}
            if first is None:
                first = pt
            diff = max((torch.linalg.vector_norm(pt[k] - first[k]) / torch.linalg.vector_norm(first[k])).item()
                       for k in pt)
            # the same call captured once as a hipGraph and replayed: at a few points per call the
            # kernels are short and the gaps between launches weigh
            graph_ms, graph_same = None, None
            if not args.no_graph:
                gr = torch.cuda.CUDAGraph()
                side = torch.cuda.Stream()
                side.wait_stream(torch.cuda.current_stream())
                with torch.cuda.stream(side):
                    run()
                torch.cuda.current_stream().wait_stream(side)
                with torch.cuda.graph(gr):
                    run()
                torch.cuda.synchronize()
                graph_same = True
                for _ in range(2):          # replays separated by eager work, each checked
                    for v in outs.values():
                        if v is not None:
                            v.zero_()
                    gr.replay()
                    torch.cuda.synchronize()
                    graph_same = graph_same and all(torch.equal(outs[k][:pt[k].numel()], pt[k]) for k in pt)
                t0 = time.perf_counter()
                for _ in range(args.steps):
                    gr.replay()
                torch.cuda.synchronize()
                graph_ms = (time.perf_counter() - t0) / args.steps * 1e3
                del gr
            res.append({"points": npts, "solver": name, "partitions": parts, "ms_per_call": dt * 1e3,
                        "points_per_s": npts / dt, "info_nonzero": int(torch.count_nonzero(info).item()),
                        "rel_diff_vs_rgf_first_point": diff, "graph_ms_per_call": graph_ms,
                        "graph_points_per_s": npts / (graph_ms * 1e-3) if graph_ms else None,
                        "graph_replays_equal_eager": graph_same})
            log(f"  {npts} point(s), {name}{'' if parts is None else f' P={parts}'}: {dt * 1e3:.1f} ms "
                f"({npts / dt:.2f} points/s)" + (f", graph replay {graph_ms:.1f} ms (equal to eager: {graph_same})"
                                                  if graph_ms else ""))
        del outs, ws
        torch.cuda.empty_cache()
    best = {}
    for r in res:
        if r["solver"] == "serinv":
            best[r["points"]] = max(best.get(r["points"], 0.0), r["points_per_s"], r["graph_points_per_s"] or 0.0)
    line = {"metric": "energy points/s at few points per call, RGF G^R+G^< (Nb=60, b=512): partitioned vs plain",
            "value": best.get(1), "unit": "energy points/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "higher_is_better": True, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "nano-ribbon-like slab device Nb=60 b=512 with scattering self-energies (norm 0.01), "
                                   "eta=1e-8, 1..8 energies per call",
                       "real_products_per_complex_product": args.cmul, "sr_max_iter": args.sr_max_iter},
            "cases": res,
            "roofline": algorithmic_roofline(point_flops(NB, B), 1.0 / best.get(1),
                                             "G^R + G^< of one energy point per call (both leads, 28 decimation steps), "
                                             "best partitioned case")}
    print(json.dumps(line), flush=True)


def bench_uneven(args):
    """Six slab devices (b, Nb) in {(128,20),(256,40),(384,60),(512,80),(640,20),(768,40)} x 4 k-points,
    refined single-product form, one plan (shape-grouped chunks over worker streams) captured as one
    hipGraph and replayed; points/s and per-device p50/p99 completion times from GPU timestamps."""
    import torch
    import workloads as w
    from paper_2602_03438_amd import autotune
    from paper_2602_03438_amd import binding as nb
    if args.uneven_queue:
        return bench_uneven_queue(args)
    ks = [np.pi * j / 4 for j in range(4)]
    grid = np.linspace(-1.5, 1.5, 2048)
    probs, dev_of = [], []
    n_e = args.uneven_points
    for d, (b, nbk) in enumerate(w.DEVICE_MIX):
        log(f"device {d}: b={b} Nb={nbk}")
        base = w.slab_device(nbk, b, 40 + d)
        S_d = nb.to_gpu(base.S_diag)
        S_u = nb.to_gpu(base.S_upper)
        for ki, k in enumerate(ks):
            dk = w.k_device(base, 1000 + d, k)
            g = nb.DeviceOnGPU.__new__(nb.DeviceOnGPU)
            g.nb, g.b = dk.nb, dk.b
            g.H_diag, g.H_upper = nb.to_gpu(dk.H_diag), nb.to_gpu(dk.H_upper)
            g.S_diag, g.S_upper = S_d, S_u
            g.sig_r = g.sig_l = g.sig_g = None
            # energy index e of the grid belongs to device e mod 6 (at every k): this device's share, n_e per k
            share = grid[d::len(w.DEVICE_MIX)]
            E = share[np.linspace(0, share.size - 1, n_e).astype(int)]
            probs.append(nb.Problem(g, E, eta=ETA, mu_l=MU_L, mu_r=MU_R, kT=KT))
            dev_of.append(d)
    tunings = []
    for b, _ in w.DEVICE_MIX:
        t = autotune.lookup(b, args.cmul)
        tunings.append((b, t["gemm_tile"], t["gemm_tile_f32"], t["inv_nb"], args.uneven_batch))
    plan = nb.Plan(probs, nb.FP32_REFINE, opts=nb.make_options(sr_max_iter=40, cmul=args.cmul), tunings=tunings,
                   n_streams=args.streams)
    chunks = plan.chunks()
    outs = plan.outputs()
    npts = sum(p.n_e for p in probs)
    info = torch.zeros(npts, dtype=torch.int32, device="cuda")
    stamps = torch.zeros(len(chunks) + 1, dtype=torch.int64, device="cuda")
    log(f"{len(probs)} problems, {npts} points, {len(chunks)} chunks on {args.streams} streams; capturing ...")
    plan.execute(outs, info, use_graph=True, stamps=stamps)
    torch.cuda.synchronize()
    log("captured; replaying")
    for _ in range(args.warmup):
        plan.execute(outs, info, use_graph=True, stamps=stamps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        plan.execute(outs, info, use_graph=True, stamps=stamps)
        torch.cuda.synchronize()
        log(f"  replay {k + 1}/{args.steps} done")
    dt = time.perf_counter() - t0
    hz = nb.Plan.clock_hz()
    st = stamps.cpu().numpy().astype(np.float64)
    t_chunk = (st[1:] - st[0]) / hz
    # per-point completion = completion of its chunk
    first = np.array([c[0] for c in chunks])
    count = np.array([c[1] for c in chunks])
    pt_done = np.zeros(npts)
    for c in range(len(chunks)):
        pt_done[first[c]:first[c] + count[c]] = t_chunk[c]
    dev_pt = np.concatenate([[dev_of[q]] * p.n_e for q, p in enumerate(probs)])
    per_dev = {}
    for d, (b, nbk) in enumerate(w.DEVICE_MIX):
        x = pt_done[dev_pt == d]
        per_dev[f"b{b}_nb{nbk}"] = {"points": int(x.size), "p50_s": float(np.percentile(x, 50)),
                                    "p99_s": float(np.percentile(x, 99)), "last_s": float(x.max())}
    # eager (no graph) for comparison, timed like the replays (one untimed run first)
    plan.execute(outs, info, use_graph=False, stamps=stamps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for k in range(args.steps):
        plan.execute(outs, info, use_graph=False, stamps=stamps)
        torch.cuda.synchronize()
        log(f"  eager {k + 1}/{args.steps} done")
    dt_eager = (time.perf_counter() - t1) / args.steps
    line = {"metric": "energy points/s, batched uneven workload (6 devices x 4 k, refined single-product form)",
            "value": npts * args.steps / dt, "unit": "energy points/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True,
            "dtype": "f32 products + f64 refinement", "data": "synthetic",
            "config": {"workload": "uneven: six slab devices (b, Nb) in " + str(w.DEVICE_MIX) +
                       f" x 4 k-points, {n_e} energies per (device, k)", "points_per_step": npts,
                       "real_products_per_complex_product": args.cmul,
                       "chunks": len(chunks), "streams": args.streams, "tunings": tunings},
            "eager_points_per_s": npts / dt_eager,
            "info_nonzero": int(torch.count_nonzero(info).item()),
            "per_device_completion": per_dev}
    print(json.dumps(line), flush=True)
    plan.close()


def uneven_devices(nb, w):
    """The six slab devices of the uneven workload at the 4 k-points: [(device index, k, BTDevice,
    device-side copy)], the overlap shared by the k copies of a device."""
    ks = [np.pi * j / 4 for j in range(4)]
    out = []
    for d, (b, nbk) in enumerate(w.DEVICE_MIX):
        log(f"device {d}: b={b} Nb={nbk}")
        base = w.slab_device(nbk, b, 40 + d)
        S_d, S_u = nb.to_gpu(base.S_diag), nb.to_gpu(base.S_upper)
        for ki, k in enumerate(ks):
            dk = w.k_device(base, 1000 + d, k)
            g = nb.DeviceOnGPU.__new__(nb.DeviceOnGPU)
            g.nb, g.b = dk.nb, dk.b
            g.H_diag, g.H_upper = nb.to_gpu(dk.H_diag), nb.to_gpu(dk.H_upper)
            g.S_diag, g.S_upper = S_d, S_u
            g.sig_r = g.sig_l = g.sig_g = None
            out.append((d, ki, dk, g))
    return out


def bench_uneven_queue(args):
    """The whole uneven workload (2048 energies x 4 k = 8192 points; grid energy e belongs to device
    e mod 6) streamed through one plan by the device-side point queue: every (device, k) problem has
    --uneven-points slots, each worker stream replays its captured round until its task lists are
    done, and every task gets its density of states, info and a GPU completion stamp.  Points/s over
    the whole run; per-device p50/p99/last completion from the stamps; the oracle on one task per
    block shape (the cpu_baseline leg) against the task's density of states."""
    import torch
    import workloads as w
    from paper_2602_03438_amd import autotune
    from paper_2602_03438_amd import binding as nb
    grid = np.linspace(-1.5, 1.5, args.uneven_grid)
    ndev = len(w.DEVICE_MIX)
    devs = uneven_devices(nb, w)
    slots = args.uneven_points
    probs, tasks, dev_of = [], [], []
    for d, ki, dk, g in devs:
        probs.append(nb.Problem(g, np.zeros(slots), eta=ETA, mu_l=MU_L, mu_r=MU_R, kT=KT))
        tasks.append(grid[d::ndev].copy())
        dev_of.append(d)
    tunings = []
    for b, _ in w.DEVICE_MIX:
        t = autotune.lookup(b, args.cmul)
        tunings.append((b, t["gemm_tile"], t["gemm_tile_f32"], t["inv_nb"], args.uneven_batch))
    prec = nb.PLAIN_FP64 if args.uneven_plain else nb.FP32_REFINE
    plan = nb.Plan(probs, prec, opts=nb.make_options(sr_max_iter=40, cmul=args.cmul), tunings=tunings,
                   n_streams=args.streams)
    chunks = plan.chunks()
    outs = plan.outputs()
    info = torch.zeros(sum(p.n_e for p in probs), dtype=torch.int32, device="cuda")
    tE = [torch.from_numpy(t).cuda() for t in tasks]
    n_tasks = int(sum(t.size for t in tasks))
    rounds = max(-(-t.size // slots) for t in tasks)
    log(f"{len(probs)} problems x {slots} slots, {n_tasks} tasks, {len(chunks)} chunks on {args.streams} streams, "
        f"{rounds} rounds")
    # the task lists go through the queue in parts of at most 10 rounds (one run_queue call each,
    # enqueued back to back): the host call returns once the GPU has taken most of its part (the HIP
    # runtime bounds the launches in flight), which gives a progress line every ~40 s
    part_rounds = 10
    parts = -(-rounds // part_rounds)
    results = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in range(parts):
        lo = j * part_rounds * slots
        sl = [t[lo:lo + part_rounds * slots] for t in tE]
        results.append(plan.run_queue(sl, outs, info, use_graph=True))
        log(f"  part {j + 1}/{parts} ({sum(x.numel() for x in sl)} tasks) enqueued after {time.perf_counter() - t0:.1f} s")
    t_enq = time.perf_counter() - t0
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    hz = nb.Plan.clock_hz()
    # per-part results back in task order (problem-major, each problem's tasks in list order)
    st, tinfo, dos = [], [], []
    for q in range(len(tasks)):
        for j, r in enumerate(results):
            lo = j * part_rounds * slots
            n_j = max(0, min(tasks[q].size - lo, part_rounds * slots))
            off = sum(max(0, min(tasks[p].size - lo, part_rounds * slots)) for p in range(q))
            st.append(r["stamps"][off:off + n_j].cpu().numpy())
            tinfo.append(r["info"][off:off + n_j].cpu().numpy())
            dos.append(r["dos"][off:off + n_j].cpu().numpy())
    st, tinfo, dos = np.concatenate(st).astype(np.float64), np.concatenate(tinfo), np.concatenate(dos)
    t_done = (st - float(results[0]["start"].item())) / hz
    dev_task = np.concatenate([[dev_of[q]] * t.size for q, t in enumerate(tasks)])
    per_dev = {}
    for d, (b, nbk) in enumerate(w.DEVICE_MIX):
        x = t_done[dev_task == d]
        per_dev[f"b{b}_nb{nbk}"] = {"points": int(x.size), "p50_s": float(np.percentile(x, 50)),
                                    "p99_s": float(np.percentile(x, 99)), "last_s": float(x.max()),
                                    "info_nonzero": int(np.count_nonzero(tinfo[dev_task == d]))}
    cpu = None
    if not args.no_cpu:
        # the oracle on one task per block shape (k = 0, the middle task of its list)
        from oracle import rgf as orgf
        checks, secs = [], 0.0
        off = np.cumsum([0] + [t.size for t in tasks])
        for q, (d, ki, dk, g) in enumerate(devs):
            if ki != 0:
                continue
            i = tasks[q].size // 2
            E = float(tasks[q][i])
            t1 = time.perf_counter()
            o = orgf.solve_point(dk, E, ETA, MU_L, MU_R, KT, lesser_greater=False)
            secs += time.perf_counter() - t1
            dos_o = -np.imag(sum(np.trace(x) for x in o.GR_diag)) / np.pi
            checks.append({"b": dk.b, "nb": dk.nb, "E": E, "dos_gpu": float(dos[off[q] + i]), "dos_oracle": float(dos_o),
                           "rel_err": float(abs(dos[off[q] + i] - dos_o) / abs(dos_o)), "info": int(tinfo[off[q] + i]),
                           "oracle_lead_residuals": [o.lead_l.residual, o.lead_r.residual]})
            log(f"  oracle b={dk.b} Nb={dk.nb} E={E:+.4f}: rel. DOS error {checks[-1]['rel_err']:.2e}")
        cpu = {"value": len(checks) / secs, "unit": "energy points/s", "cores": os.cpu_count(), "kind": "oracle",
               "sample": "one task per block shape (k = 0), G^R only, NumPy complex128", "seconds": secs,
               "checks": checks}
    form = "plain FP64" if args.uneven_plain else "refined single-product form"
    line = {"metric": "energy points/s, batched uneven workload streamed by the point queue (6 devices x 4 k, "
                      f"2048 energies, {form})",
            "value": n_tasks / dt, "unit": "energy points/s", "n_gpus": 1, "steps": 1, "warmup": 0,
            "ms_per_step": dt * 1e3, "higher_is_better": True,
            "dtype": "f64" if args.uneven_plain else "f32 products + f64 refinement",
            "data": "synthetic",
            "config": {"workload": "uneven: six slab devices (b, Nb) in " + str(w.DEVICE_MIX) +
                       f" x 4 k-points x {args.uneven_grid} energies (grid energy e on device e mod 6): "
                       f"{n_tasks} points",
                       "slots_per_device_k": slots, "rounds": rounds, "queue_calls": parts, "chunks": len(chunks),
                       "streams": args.streams, "tunings": tunings,
                       "real_products_per_complex_product": args.cmul},
            "roofline": algorithmic_roofline(sum(point_flops(nbk, b) * tasks[q].size
                                                 for q, (d, ki, dk, g) in enumerate(devs)
                                                 for (b, nbk) in [w.DEVICE_MIX[d]]), dt,
                                             "G^R + G^< of every task at its device's (Nb, b), 28 decimation steps; "
                                             "single-precision products of the refined form counted like double"),
            "gpu_seconds_start_to_last": float(t_done.max()), "host_enqueue_s": t_enq,
            "stamped_tasks": int(np.count_nonzero(st)),
            "info_nonzero": int(np.count_nonzero(tinfo)),
            "per_device_completion": per_dev,
            "cpu_baseline": cpu}
    print(json.dumps(line), flush=True)
    plan.close()


def bench_learned(args):
    """MLP-seeded lead decimation: train on decimation-converged samples of 8 leads, evaluate on held-out
    leads; report iterations to convergence, acceptance of the seed and points/s with and without it."""
    import torch
    import workloads as w
    from paper_2602_03438_amd import binding as nb
    from paper_2602_03438_amd import learned as Lm
    b = args.learned_b
    # points in flight per decimation call (bounds the workspace: ~54 MiB per point at b = 512)
    lopts = nb.make_options(batch=1024)
    rng = np.random.Generator(np.random.PCG64(599))
    t_start = time.perf_counter()
    X_all, T_all = [], []
    sr_iters_train = []
    for seed in range(500, 508):
        lead = w.slab_lead(b, seed)
        basis = Lm.lead_basis(lead, 0)
        gb = Lm.GPUBasis(basis)
        E = rng.uniform(-1.5, 1.5, args.learned_energies)
        prob = nb.Problem(nb.DeviceOnGPU(lead), E, eta=ETA)
        out = nb.obc_surface([prob], 0, opts=lopts)
        g = out["g_surf"][0][:, 0].contiguous()
        T_all.append(gb.targets(g))
        X_all.append(torch.from_numpy(Lm.features(basis, E)).cuda())
        sr_iters_train.append(out["iters"].cpu().numpy())
        log(f"lead {seed}: {E.size} samples, mean decimation steps {sr_iters_train[-1].mean():.1f}")
    X = torch.cat(X_all)
    T = torch.cat(T_all)
    gen_s = time.perf_counter() - t_start
    # targets span decades near band edges: train on a signed-log compression, invert at inference
    Tc = Lm.signed_log(T)
    net = Lm.MLP(seed=0)
    t0 = time.perf_counter()
    losses = net.train(X, Tc, epochs=4, batch=65536, lr=1e-3, log=log)
    train_s = time.perf_counter() - t0
    res = {"plain": {"iters": [], "s": 0.0}, "seeded": {"iters": [], "s": 0.0, "accepted": 0, "closed": 0},
           "zero": {"iters": []}}
    n_eval = 0
    for seed in range(600, 604):
        lead = w.slab_lead(b, seed)
        basis = Lm.lead_basis(lead, 0)
        gb = Lm.GPUBasis(basis)
        E = np.linspace(-1.5, 1.5, args.learned_eval)
        prob = nb.Problem(nb.DeviceOnGPU(lead), E, eta=ETA)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        plain = nb.obc_surface([prob], 0, opts=lopts)
        torch.cuda.synchronize()
        res["plain"]["s"] += time.perf_counter() - t1
        t1 = time.perf_counter()
        Xh = torch.from_numpy(Lm.features(basis, E)).cuda()
        Yc = net.infer_bf16(Xh)
        Y = Lm.signed_log(Yc, inverse=True)
        seeds = gb.seeds(Y)
        seeded = nb.obc_surface([prob], 0, opts=lopts, seed=seeds)
        torch.cuda.synchronize()
        res["seeded"]["s"] += time.perf_counter() - t1
        # the seeded closure alone (a zero seed: no learned information) for comparison
        zero = nb.obc_surface([prob], 0, opts=lopts, seed=torch.zeros_like(seeds))
        ip = plain["iters"].cpu().numpy()
        res["plain"]["iters"] += ip.tolist()
        it = seeded["iters"].cpu().numpy()
        res["seeded"]["iters"] += it.tolist()
        res["seeded"]["accepted"] += int(np.count_nonzero(it == 0))
        res["seeded"]["closed"] += int(np.count_nonzero((it > 0) & (it < ip)))
        res["zero"]["iters"] += zero["iters"].cpu().tolist()
        d = (seeded["g_surf"][0] - plain["g_surf"][0]).abs().max().item()
        log(f"held-out lead {seed}: plain {np.mean(ip):.2f} steps, seeded {np.mean(it):.2f} steps "
            f"(zero seed {np.mean(zero['iters'].cpu().numpy()):.2f}), candidate accepted {np.count_nonzero(it == 0)}"
            f"/{E.size}, closed early {np.count_nonzero((it > 0) & (it < ip))}/{E.size}, max |dg| {d:.2e}")
        n_eval += E.size
    line = {"metric": "learned lead initialiser: decimation steps and energy points/s with vs without the seed",
            "unit": "energy points/s", "value": n_eval / res["seeded"]["s"], "higher_is_better": True,
            "plain_value": n_eval / res["plain"]["s"],
            "mean_steps_plain": float(np.mean(res["plain"]["iters"])),
            "mean_steps_seeded": float(np.mean(res["seeded"]["iters"])),
            "mean_steps_zero_seed_closure": float(np.mean(res["zero"]["iters"])),
            "seed_acceptance": res["seeded"]["accepted"] / n_eval,
            "closure_rate": res["seeded"]["closed"] / n_eval,
            "fallback_rate": 1.0 - (res["seeded"]["accepted"] + res["seeded"]["closed"]) / n_eval,
            "train_samples": int(X.shape[0] // b), "train_rows": int(X.shape[0]), "final_mse": losses[-1],
            "data_generation_s": gen_s, "train_s": train_s, "b": b, "eval_points": n_eval,
            "dtype": "f32 training, bf16 inference, f64 decimation", "data": "synthetic"}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
