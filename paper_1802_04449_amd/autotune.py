"""Tile-shape autotuner: times every workgroup tile shape of the stencil kernels on
a given grid through the C ABI and keeps the fastest.

The library's default (fewest padded thread slots, coalescing-aware) is a
reasonable start; the best shape depends on the grid's extents, the vacuum
fraction and the mode, so it is measured.  Results are cached per
(nx, ny, ne, viscous, cartesian) in a JSON file next to this module.
"""
from __future__ import annotations

import json
import os
import time

from . import (KtmiError, ktmi_get_tile, ktmi_set_tile, ktmi_tile_count, ktmi_tile_shape)

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json")


def _key(hydro) -> str:
    d = hydro.desc
    return f"{d.nx}x{d.ny}x{d.ne}:v{d.viscous}:c{d.cartesian}:p{d.precision}"


def tune(hydro, steps: int = 3, repeats: int = 2, use_cache: bool = True, verbose=False):
    """Time `steps` steps per tile shape (best of `repeats`) on hydro's current state
    and select the fastest.  The state advances during tuning, so call it before the
    run of interest (or on a throwaway copy).  Returns (tile, {tile: ms_per_step})."""
    torch = hydro.torch
    key = _key(hydro)
    cache = {}
    if use_cache and os.path.exists(CACHE):
        try:
            cache = json.load(open(CACHE))
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        t = int(cache[key]["tile"])
        ktmi_set_tile(hydro.h, t)
        return t, cache[key]["ms"]
    times = {}
    for t in range(ktmi_tile_count()):
        try:
            ktmi_set_tile(hydro.h, t)
        except KtmiError:
            continue
        best = float("inf")
        hydro.step(1)  # first launch of this shape
        for _ in range(repeats):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            hydro.step(steps)
            torch.cuda.synchronize()
            best = min(best, (time.perf_counter() - t0) / steps * 1e3)
        times[t] = best
        if verbose:
            print(f"tile {t} {ktmi_tile_shape(t)}: {best:.3f} ms/step", flush=True)
    t = min(times, key=times.get)
    ktmi_set_tile(hydro.h, t)
    if use_cache:
        cache[key] = {"tile": t, "shape": list(ktmi_tile_shape(t)),
                      "ms": {str(k): v for k, v in times.items()}}
        try:
            json.dump(cache, open(CACHE, "w"), indent=1)
        except OSError:
            pass
    return t, times


def current_shape(hydro):
    return ktmi_tile_shape(ktmi_get_tile(hydro.h))
