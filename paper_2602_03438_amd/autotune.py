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

    python -m paper_2602_03438_amd.autotune 128 256 384 512 640 768
"""
from __future__ import annotations

import json
import os
import sys
import time

from . import binding as nb

HERE = os.path.dirname(os.path.abspath(__file__))
ARCH = "gfx950"
TILES = {1: "64x64", 2: "128x64", 3: "128x128", 4: "64x64/8w", 5: "128x64/16w"}
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


def tune(blocks, batch=64, log=print, save=True) -> dict:
    cache = load_cache()
    for b in blocks:
        cache.update(tune_block(int(b), batch, log))
    if save:
        with open(cache_path(), "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return cache


if __name__ == "__main__":
    import torch
    assert torch.cuda.is_available(), "the tuner runs on the GPU"
    bs = [int(x) for x in sys.argv[1:]] or [512]
    tune(bs, log=lambda m: print(m, flush=True))
    print("wrote", cache_path())
