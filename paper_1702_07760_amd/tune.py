"""Autotuner for the launch shape of the neighbour passes.

Times short graph-replayed runs of a scene over a grid of options and keeps the
fastest.  The options:
  block        threads per block of the neighbour passes (64, 128, 256);
  xcd_remap    tile order: dispatch order (0), consecutive tiles per XCD (1), and K
               consecutive tiles per CU as well (K = 4, 16);
  lanes        lanes per particle in the renormalisation pass (1, 2, 4);
  force_lanes  lanes per particle in the force pass (1, 2, 4);
  skin         neighbour skin in units of h, which sets the cell size and list radius
               (2 + skin) h; a larger skin means longer lists, a smaller one more
               frequent rebuilds (a particle may move skin h / 4 between them).
The skin changes which extra pairs sit in the lists (they are filtered out), not
the physics, except through the time-step limit dt <= skin h / (2 max|u|).  The grid
is searched one option at a time (coordinate descent from the defaults), not as a
full product.
Results are cached per (GPU arch, dimension, precision, particle-count bucket) in
a JSON file beside this module.
"""
from __future__ import annotations

import json
import math
import os
import time

from . import binding

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")
BLOCKS = (64, 128, 256)
REMAPS = (0, 1, 4, 16)
LANES = (1, 2, 4)
SKINS = (0.05, 0.1, 0.2)
DEFAULTS = {"skin": 0.1, "block": 64, "xcd_remap": None, "lanes": 4, "force_lanes": None}


def cache_key(scene, precision, arch="gfx950"):
    bucket = 2 ** int(round(math.log2(max(scene.n, 1))))
    return f"{arch}/d{scene.dim}/p{precision}/n{bucket}"


def load_cache() -> dict:
    if os.path.exists(CACHE):
        with open(CACHE) as fh:
            return json.load(fh)
    return {}


def _time(scene, precision, opts, steps, warmup):
    sim = binding.Sim(scene.with_params(skin_coef=opts["skin"]), precision=precision)
    try:
        sim.set_option(binding.OPT_BLOCK, opts["block"])
        sim.set_option(binding.OPT_XCD_REMAP, opts["xcd_remap"])
        sim.set_option(binding.OPT_LANES, opts["lanes"])
        if opts["force_lanes"] is not None:
            sim.set_option(binding.OPT_FORCE_LANES, opts["force_lanes"])
        sim.step(warmup)
        sim.sync()
        t0 = time.perf_counter()
        sim.step(steps)
        sim.sync()
        return (time.perf_counter() - t0) / steps
    finally:
        sim.close()


def tune(scene, precision=binding.FP32_CELLREL, steps=20, warmup=3, skins=SKINS,
         blocks=BLOCKS, remaps=REMAPS, lanes=LANES, save=True, log=print) -> dict:
    """Coordinate descent over the options; returns (and caches) the fastest set."""
    grid = {"skin": skins, "block": blocks, "xcd_remap": remaps, "lanes": lanes, "force_lanes": lanes}
    # start from the library's own defaults for this precision, dimension and size
    best = dict(DEFAULTS)
    fp32 = precision == binding.FP32_CELLREL
    best["force_lanes"] = 2 if scene.dim == 3 else 1
    d3 = scene.dim == 3
    best["xcd_remap"] = 0 if d3 else (4 if fp32 else 1)
    best["block"] = (256 if scene.n >= 1 << 19 else 128) if d3 else 64
    if not d3 and scene.n >= 1 << 16 and (fp32 or scene.n < 1 << 20):
        best["block"], best["xcd_remap"] = 128, 16
    best["lanes"] = 1 if scene.dim == 2 and scene.n >= 1 << 20 else 4
    results = []
    best_ms = 1e3 * _time(scene, precision, best, steps, warmup)
    results.append(dict(best, ms_per_step=best_ms))
    for key, values in grid.items():
        for v in values:
            if v == best[key]:
                continue
            trial = dict(best, **{key: v})
            ms = 1e3 * _time(scene, precision, trial, steps, warmup)
            results.append(dict(trial, ms_per_step=ms))
            if log:
                log(f"tune {trial}: {ms:.4f} ms/step")
            if ms < best_ms:
                best, best_ms = trial, ms
    best = dict(best, ms_per_step=best_ms)
    if save:
        cache = load_cache()
        cache[cache_key(scene, precision)] = dict(best=best, all=results)
        with open(CACHE, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
    return best


def best_for(scene, precision):
    """Cached best options for a scene, or None."""
    entry = load_cache().get(cache_key(scene, precision))
    return entry["best"] if entry else None


def apply(sim, best):
    """Apply cached launch options to a Sim (the skin must be set on the scene)."""
    if best:
        sim.set_option(binding.OPT_BLOCK, int(best["block"]))
        sim.set_option(binding.OPT_XCD_REMAP, int(best["xcd_remap"]))
        sim.set_option(binding.OPT_LANES, int(best["lanes"]))
        if best.get("force_lanes") is not None:
            sim.set_option(binding.OPT_FORCE_LANES, int(best["force_lanes"]))
