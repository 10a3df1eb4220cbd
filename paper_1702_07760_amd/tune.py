"""Autotuner for the launch shape of the neighbour passes.

Times short graph-replayed runs of a scene over the launch options and keeps the
fastest.  It searches only options that leave every result bit-identical, since
each particle's arithmetic, and its order, do not depend on them:
  block        threads per block of the neighbour passes (64, 128, 192, 256);
  xcd_remap    tile order: dispatch order (0), consecutive tiles per XCD (1), and K
               consecutive tiles per CU as well (K = 4, 16), or chunks of C tiles
               dealt round-robin to the XCDs (-C: C = 4, 16).
Lanes per particle split a particle's sums differently, and the neighbour skin sets
the cell size and so the sorted order: both change results at the rounding level,
so they keep the library's defaults.  The search is coordinate descent from the
library's defaults (one option at a time, repeated until nothing improves).
Results are cached per (GPU arch, dimension, precision, particle-count bucket) in
``tune_cache.json`` beside this module; ``binding.Sim`` applies the cached entry of
its scene when one exists.
"""
from __future__ import annotations

import json
import math
import os
import time

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")
BLOCKS = (64, 128, 192, 256)
REMAPS = (0, 1, 4, 16, -4, -16)
KEYS = ("block", "xcd_remap")


def cache_key(dim, n, precision, arch="gfx950"):
    bucket = 2 ** int(round(math.log2(max(n, 1))))
    return f"{arch}/d{dim}/p{precision}/n{bucket}"


def load_cache() -> dict:
    if os.path.exists(CACHE):
        with open(CACHE) as fh:
            return json.load(fh)
    return {}


def best_for(dim, n, precision):
    """Cached launch options (block, xcd_remap) for a scene of this kind, or None."""
    entry = load_cache().get(cache_key(dim, n, precision))
    return {k: int(entry["best"][k]) for k in KEYS} if entry else None


def _time(scene, precision, opts, steps, warmup, repeats):
    from . import binding
    sim = binding.Sim(scene, precision=precision, tuned=False)
    try:
        if opts:
            sim.set_launch(**opts)
        sim.step(warmup)
        sim.sync()
        best = math.inf
        for _ in range(repeats):
            t0 = time.perf_counter()
            sim.step(steps)
            sim.sync()
            best = min(best, (time.perf_counter() - t0) / steps)
        return best
    finally:
        sim.close()


def tune(scene, precision, steps=20, warmup=3, repeats=3, blocks=BLOCKS, remaps=REMAPS,
         save=True, log=print) -> dict:
    """Coordinate descent over block and tile order; returns (and caches) the fastest."""
    from . import binding
    probe = binding.Sim(scene, precision=precision, tuned=False)
    best = {k: probe.launch_options()[k] for k in KEYS}
    probe.close()
    grid = {"block": blocks, "xcd_remap": remaps}
    results = []
    best_ms = 1e3 * _time(scene, precision, best, steps, warmup, repeats)
    results.append(dict(best, ms_per_step=best_ms, default=True))
    improved = True
    while improved:
        improved = False
        for key, values in grid.items():
            for v in values:
                if v == best[key]:
                    continue
                trial = dict(best, **{key: v})
                if any(all(r[k] == trial[k] for k in KEYS) for r in results):
                    continue
                ms = 1e3 * _time(scene, precision, trial, steps, warmup, repeats)
                results.append(dict(trial, ms_per_step=ms))
                if log:
                    log(f"tune {scene.name} p{precision} {trial}: {ms:.4f} ms/step")
                if ms < best_ms:
                    best, best_ms, improved = trial, ms, True
    best = dict(best, ms_per_step=best_ms)
    if save:
        cache = load_cache()
        cache[cache_key(scene.dim, scene.n, precision)] = dict(scene=scene.name, n=scene.n, best=best,
                                                               all=results)
        with open(CACHE, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
    return best


SCENES = {
    "drop3d": lambda i: i.drop3d(),
    "paper_sphere": lambda i: i.paper_drop("sphere"),
    "lab_flume_5mm": lambda i: i.lab_flume(3, dx=5e-3, width=0.05),
    "lab_flume_1mm": lambda i: i.lab_flume(3, dx=1e-3, width=0.015),
    "flume2d": lambda i: i.flume2d(),
    "flume3d": lambda i: i.flume3d(),
    "tanks256": lambda i: i.batched_drops(),
    "drop2d": lambda i: i.drop2d(),
}


def main(argv=None):
    """Tune named scenes and merge the results into the cache (or another JSON file):
    python -m paper_1702_07760_amd.tune drop3d:1 drop3d:0 flume3d:1 [--out FILE]
    (scene:precision, 0 = FP64, 1 = FP32 cell-relative)."""
    import argparse
    from . import inputs
    ap = argparse.ArgumentParser()
    ap.add_argument("cases", nargs="+")
    ap.add_argument("--out", default=None, help="JSON file to merge into (default: the cache)")
    ap.add_argument("--steps", type=int, default=20)
    args = ap.parse_args(argv)
    if args.out:
        globals()["CACHE"] = args.out
    for case in args.cases:
        name, prec = case.split(":")
        scene = SCENES[name](inputs)
        best = tune(scene, int(prec), steps=args.steps)
        print(f"best {name} p{prec} n={scene.n}: {best}", flush=True)


if __name__ == "__main__":
    main()
