"""Tile and schedule tuner for the NEGF kernels on the local GPU.

For a block size b it times, on the GPU, every candidate of
  * the complex product kernel: output tile 64x64 (4 or 8 waves) / 128x64 (8 or 16) / 128x128, for the
    double (four and three real products per complex one) and the
    single-precision products, at the batch the sweeps use;
  * the block inversion: panel width 16 / 32;
and keeps the fastest (for the products: a 64x64 tile within 2 % of the fastest,
because only those tiles skip the zero slabs of a coupling-block operand).  Results are cached as JSON keyed by
"<arch>/b=<b>/<dtype>/<op>" (dtype f64, f64g = three-product double, f32) (``tune_cache.json`` next to this file, or the
path in $NEGF_TUNE_CACHE); a block size with no entry gets the deterministic
default (64x64 tiles, panel 16).

With --step it then times the whole hot path (both lead decimations and the
G^R and G^< sweeps of one batched call) for the product tiles within 10 % of the
fastest and both panel widths, on a random block-tridiagonal device of that
block size, and keeps the fastest combination under op "step"; lookup() prefers
that entry, so kernel timings in isolation only decide where no step was timed.

    python -m paper_2602_03438_amd.autotune [--step] 128 256 384 512 640 768
"""
from __future__ import annotations

import json
import os
import sys
import time

from . import binding as nb

HERE = os.path.dirname(os.path.abspath(__file__))
ARCH = "gfx950"
TILES = {1: "64x64", 2: "128x64", 3: "128x128", 4: "64x64/8w", 5: "128x64/16w", 6: "32x32"}
DEFAULT = {"gemm_tile": 1, "gemm_tile_f32": 1, "inv_nb": 16}


def cache_path() -> str:
    return os.environ.get("NEGF_TUNE_CACHE", os.path.join(HERE, "tune_cache.json"))


def load_cache() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def key(b: int, dtype: str, op: str) -> str:
    return f"{ARCH}/b={b}/{dtype}/{op}"


def lookup(b: int, cmul: int = 4) -> dict:
    """Tuned choices for block size b (defaults where the cache has none).
    cmul = 3 takes the tile timed for the three-product double kernel."""
    c = load_cache()
    out = dict(DEFAULT)
    g64 = c.get(key(b, "f64g" if cmul == 3 else "f64", "zgemm")) or c.get(key(b, "f64", "zgemm"))
    g32 = c.get(key(b, "f32", "zgemm"))
    inv = c.get(key(b, "f64", "zinv"))
    if g64:
        out["gemm_tile"] = int(g64["best"])
    if g32:
        out["gemm_tile_f32"] = int(g32["best"])
    if inv:
        out["inv_nb"] = int(inv["best"])
    step = c.get(key(b, "f64g" if cmul == 3 else "f64", "step"))
    if step:
        out["gemm_tile"] = int(step["best"]["gemm_tile"])
        out["inv_nb"] = int(step["best"]["inv_nb"])
    return out


# Only the 64 x 64 tiles skip the zero slabs of a coupling-block operand (about a
# third of the sweep products), so they win any near tie of the dense timings.
SLAB_TILES = (1, 4)
TIE = 0.02


def pick(times: dict) -> int:
    """Fastest tile; a 64 x 64 tile within TIE of it is preferred."""
    best = min(times, key=times.get)
    near = [t for t in SLAB_TILES if t in times and times[t] <= times[best] * (1.0 + TIE)]
    return min(near, key=times.get) if near else best


def _time(fn, reps=5):
    import torch
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def tune_block(b: int, batch: int = 64, log=print) -> dict:
    import torch
    res = {}
    A = torch.randn(batch, b, b, dtype=torch.complex128, device="cuda")
    B = torch.randn(batch, b, b, dtype=torch.complex128, device="cuda")
    C = torch.empty_like(A)
    for prec, dtype in ((0, "f64"), (2, "f64g"), (1, "f32")):
        times = {}
        for tile in TILES:
            t = _time(lambda: nb.zgemm(A, B, C, prec=prec, tile=tile))
            times[tile] = t
            log(f"b={b} {dtype} zgemm tile {TILES[tile]}: {t * 1e3:.3f} ms "
                f"({8.0 * batch * b ** 3 / t / 1e12:.1f} TFLOP/s)")
        res[key(b, dtype, "zgemm")] = {"best": pick(times), "ms": {TILES[k]: v * 1e3 for k, v in times.items()},
                                       "batch": batch}
    M = A + 2.0 * b ** 0.5 * torch.eye(b, dtype=torch.complex128, device="cuda")
    times = {}
    for panel in (16, 32):
        t = _time(lambda: nb.zinv(M, panel), reps=3)
        times[panel] = t
        log(f"b={b} zinv panel {panel}: {t * 1e3:.3f} ms ({8.0 * batch * b ** 3 / t / 1e12:.1f} TFLOP/s)")
    best = min(times, key=times.get)
    res[key(b, "f64", "zinv")] = {"best": best, "ms": {str(k): v * 1e3 for k, v in times.items()}, "batch": batch}
    return res


def pick_step(times: dict):
    """Fastest (tile, panel) of a step timing; as for the products, a 64 x 64 tile within TIE of it
    is preferred (the tuner's device has dense couplings, where the other tiles lose nothing to
    slab skipping)."""
    best = min(times, key=times.get)
    near = [k for k in times if k[0] in SLAB_TILES and times[k] <= times[best] * (1.0 + TIE)]
    return min(near, key=times.get) if near else best


def _step_device(b: int, nblocks: int, seed: int):
    """A random block-tridiagonal device of block size b on the GPU: Hermitian on-site blocks,
    couplings of norm about one, S = I (the tuner's own input, not a physical model)."""
    import torch
    g = torch.Generator(device="cuda").manual_seed(seed)
    X = torch.randn(nblocks, b, b, dtype=torch.complex128, device="cuda", generator=g)
    Hd = (X + X.conj().transpose(-1, -2)) * (0.5 / b ** 0.5)
    Hu = torch.randn(nblocks - 1, b, b, dtype=torch.complex128, device="cuda", generator=g) * (0.3 / b ** 0.5)
    dev = nb.DeviceOnGPU.__new__(nb.DeviceOnGPU)
    dev.nb, dev.b = nblocks, b
    dev.H_diag, dev.H_upper = Hd.contiguous(), Hu.contiguous()
    dev.S_diag = dev.S_upper = None
    dev.sig_r = dev.sig_l = dev.sig_g = None
    return dev


def tune_step(b: int, cmul: int = 3, points: int = 32, nblocks: int = 8, log=print) -> dict:
    """Time one batched G^R + G^< call (decimation of both leads included) for every
    combination of the product tiles within 10 % of the fastest (from the kernel timings
    in the cache) and the two panel widths."""
    import numpy as np
    import torch
    c = load_cache()
    dtype = "f64g" if cmul == 3 else "f64"
    g = c.get(key(b, dtype, "zgemm"))
    tiles = [1]
    if g:
        ms = {k: v for k, v in g["ms"].items()}
        fastest = min(ms.values())
        tiles = [t for t, name in TILES.items() if name in ms and ms[name] <= 1.10 * fastest]
    dev = _step_device(b, nblocks, 7 + b)
    prob = nb.Problem(dev, np.linspace(-0.9, 0.9, points), eta=1e-6)
    ws = nb.Workspace()
    times = {}
    for tile in tiles:
        for panel in (16, 32):
            opts = nb.make_options(cmul=cmul, gemm_tile=tile, inv_nb=panel, sr_max_iter=40)
            t = _time(lambda: nb.rgf_lesser_greater([prob], nb.PLAIN_FP64, opts=opts, ws=ws), reps=3)
            times[(tile, panel)] = t
            log(f"b={b} step ({nblocks} blocks, {points} points) tile {TILES[tile]} panel {panel}: "
                f"{t * 1e3:.1f} ms ({points / t:.1f} points/s)")
    best = pick_step(times)
    return {key(b, dtype, "step"): {"best": {"gemm_tile": best[0], "inv_nb": best[1]},
                                    "ms": {f"{TILES[k[0]]}/panel{k[1]}": v * 1e3 for k, v in times.items()},
                                    "points": points, "blocks": nblocks}}


def tune(blocks, batch=64, log=print, save=True, step=False) -> dict:
    cache = load_cache()
    for b in blocks:
        cache.update(tune_block(int(b), batch, log))
        if step:
            if save:
                with open(cache_path(), "w") as f:
                    json.dump(cache, f, indent=1, sort_keys=True)
            cache.update(tune_step(int(b), log=log))
    if save:
        with open(cache_path(), "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return cache


if __name__ == "__main__":
    import torch
    assert torch.cuda.is_available(), "the tuner runs on the GPU"
    bs = [int(x) for x in sys.argv[1:] if not x.startswith("--")] or [512]
    tune(bs, log=lambda m: print(m, flush=True), step="--step" in sys.argv)
    print("wrote", cache_path())
