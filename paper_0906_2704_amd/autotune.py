"""Schedule autotuner for ragged batches.

For every FFT size class of a batch it times ht_batch_restore restricted to that class
(HIP events, median of a few launches) over the kernel variants (8 or 16 points per
thread where both exist) and persistent-grid sizes (fractions and multiples of the
occupancy-derived default), keeps the fastest, and records the choice in a JSON cache
keyed by device and class sizes so later runs reuse it.  Results never depend on the
schedule, only the time does.
"""

import json
import os

import torch

from . import ht

CACHE = os.environ.get("HT_AUTOTUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "ht_autotune.json"))
GRID_FACTORS = (0.5, 1.0, 2.0, 4.0)


def _key(batch):
    name = torch.cuda.get_device_name()
    counts = [batch.class_count(c) for c in range(ht.NCLASS)]
    return "%s|%s" % (name, ",".join(str(c) for c in counts))


def _time(fn, reps):
    fn()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
    times.sort()
    return times[len(times) // 2]


def load_cache(path=CACHE):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def apply(batch, choice):
    for c, (grid, variant) in choice.items():
        batch.schedule(int(c), int(grid), int(variant))


def tune(batch, run, reps=3, use_cache=True, path=CACHE, log=None):
    """Tune `batch`; `run()` launches ht_batch_restore with the caller's arrays.
    Returns {class: (workgroups, variant)} and the per-class timings (ms)."""
    key = _key(batch)
    cache = load_cache(path) if use_cache else {}
    if key in cache:
        choice = {int(c): tuple(v) for c, v in cache[key]["choice"].items()}
        apply(batch, choice)
        return choice, cache[key].get("ms", {})
    choice, timing = {}, {}
    for c in range(ht.NCLASS):
        if batch.class_count(c) == 0:
            continue
        batch.class_mask(1 << c)
        base_grid, base_var = batch.schedule(c)
        variants = (0, 1) if c >= 3 else (0,)
        best = None
        for var in variants:
            batch.schedule(c, 0, var)
            # occupancy-derived default of this variant: query after resetting the grid
            for fac in GRID_FACTORS:
                grid = max(1, int(round(base_grid * fac)))
                grid, _ = batch.schedule(c, grid, var)
                ms = _time(run, reps)
                if log:
                    log("class %d variant %d grid %d: %.3f ms" % (c, var, grid, ms))
                if best is None or ms < best[0]:
                    best = (ms, grid, var)
        choice[c] = (best[1], best[2])
        timing[c] = best[0]
        batch.schedule(c, best[1], best[2])
    batch.class_mask((1 << ht.NCLASS) - 1)
    if use_cache:
        cache = load_cache(path)
        cache[key] = {"choice": {str(c): list(v) for c, v in choice.items()}, "ms": {str(c): t for c, t in timing.items()}}
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path, "w") as fh:
                json.dump(cache, fh, indent=1, sort_keys=True)
        except OSError:
            pass
    return choice, timing
