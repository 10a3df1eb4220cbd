"""Autotuner for the launch shape of the neighbour passes.

Times short graph-replayed runs of a scene over a grid of options and keeps the
fastest.  The options:
  block      threads per block of the neighbour passes (64, 128, 256);
  xcd_remap  consecutive tiles on one XCD, or the default round-robin;
  skin       neighbour skin in units of h, which sets the cell size (2 + skin) h and
             the list radius (2 + skin/2) h; larger cells mean more candidates per
             list build, a larger skin means longer lists.
The skin changes which extra pairs sit in the lists (they are filtered out), not
the physics, except through the time-step limit dt <= skin h / (2 max|u|).
Results are cached per (GPU arch, dimension, precision, particle-count bucket) in
a JSON file beside this module.
"""
from __future__ import annotations

import itertools
import json
import math
import os
import time

from . import binding

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")
BLOCKS = (64, 128, 256)
REMAPS = (0, 1)
SKINS = (0.05, 0.1, 0.2)


def cache_key(scene, precision, arch="gfx950"):
    bucket = 2 ** int(round(math.log2(max(scene.n, 1))))
    return f"{arch}/d{scene.dim}/p{precision}/n{bucket}"


def load_cache() -> dict:
    if os.path.exists(CACHE):
        with open(CACHE) as fh:
            return json.load(fh)
    return {}


def _time(scene, precision, block, remap, steps, warmup):
    sim = binding.Sim(scene, precision=precision)
    try:
        sim.set_option(binding.OPT_BLOCK, block)
        sim.set_option(binding.OPT_XCD_REMAP, remap)
        sim.step(warmup)
        sim.sync()
        t0 = time.perf_counter()
        sim.step(steps)
        sim.sync()
        return (time.perf_counter() - t0) / steps
    finally:
        sim.close()


def tune(scene, precision=binding.FP32_CELLREL, steps=20, warmup=3, skins=SKINS,
         blocks=BLOCKS, remaps=REMAPS, save=True, log=print) -> dict:
    """Time every option combination and return (and cache) the fastest."""
    results = []
    for skin in skins:
        sc = scene.with_params(skin_coef=skin)
        for block, remap in itertools.product(blocks, remaps):
            ms = 1e3 * _time(sc, precision, block, remap, steps, warmup)
            results.append(dict(skin=skin, block=block, xcd_remap=remap, ms_per_step=ms))
            if log:
                log(f"tune skin={skin} block={block} remap={remap}: {ms:.4f} ms/step")
    best = min(results, key=lambda r: r["ms_per_step"])
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
