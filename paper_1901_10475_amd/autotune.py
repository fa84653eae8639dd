"""Autotuner for the traversal's launch shapes and the tree's time slabs.

``tune`` searches the fields of ``cd_tuning`` (node-pair workgroups per level
and lanes per workgroup, per-leaf-walk lanes, traversal mode) on a built
tree, timing the query alone; ``tune_slab`` searches the width of the time
field of the tree key (``slab_ticks`` of cd_build_tree) for boxes without a
slab structure (per-object steps), timing tree build and query together.
Timings are medians of ``reps`` runs after one warm-up, from device events on
the current stream.  The best choice is cached in a JSON file keyed by (GPU
architecture, tree precision, box-count bucket, step mode, what was tuned).
Every candidate yields the same record list -- only time differs -- and the
tuner checks that before it accepts a timing.
"""
import json
import math
import os

import numpy as np
import torch

from . import cd_get_tuning, cd_set_tuning

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_1901_10475_amd",
                             "tuning.json")


def candidates():
    out = []
    for blocks in (512, 1024, 2048, 4096, 8192):
        for threads in (128, 256, 512):
            out.append({"mode": 0, "expand_blocks": blocks, "expand_threads": threads,
                        "walk_threads": 256})
    for walk in (64, 128, 256):
        out.append({"mode": 1, "walk_threads": walk})
    return out


def cache_key(precision, boxes, dt_mode, arch=None, what="launch"):
    if arch is None:
        arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    bucket = int(round(math.log2(max(int(boxes), 1))))
    prec = "fp64" if precision == 0 else "fp32"
    key = f"{arch}|{prec}|2^{bucket}|{dt_mode}"
    return key if what == "launch" else key + "|" + what


def load_cache(path=None):
    path = path or os.environ.get("CD4D_TUNE_CACHE", DEFAULT_CACHE)
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache, path=None):
    path = path or os.environ.get("CD4D_TUNE_CACHE", DEFAULT_CACHE)
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time_query(query, reps):
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    out = query()   # warm-up, and the record list to compare
    for a, b in ev:
        a.record()
        query()
        b.record()
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in ev])), out


def tune(query, reps=3, cands=None, log=None):
    """query(): runs one query on a built tree and returns its record list.
    Returns (best tuning dict, [(tuning, ms)])."""
    saved = cd_get_tuning()
    results = []
    ref = None
    try:
        for c in (cands or candidates()):
            cd_set_tuning(c)
            ms, out = _time_query(query, reps)
            if ref is None:
                ref = out.cpu()
            elif not torch.equal(out.cpu(), ref):
                raise RuntimeError(f"tuning {c} changed the record list")
            results.append((c, ms))
            if log:
                log(f"[tune] {c} {ms:.3f} ms")
    finally:
        cd_set_tuning(saved)
    best = min(results, key=lambda r: r[1])[0]
    return best, results


def tuned(query, precision, boxes, dt_mode, path=None, reps=3, log=None):
    """Cached best tuning for this key, searched (and stored) on a miss."""
    key = cache_key(precision, boxes, dt_mode)
    cache = load_cache(path)
    if key in cache:
        return cache[key]["tuning"], True
    best, results = tune(query, reps=reps, log=log)
    cache[key] = {"tuning": best,
                  "ms": {json.dumps(c, sort_keys=True): ms for c, ms in results}}
    save_cache(cache, path)
    return best, False


def slab_candidates(horizon_ticks):
    """Time-slab widths from 1/1024 of the horizon to a quarter of it."""
    T = max(int(horizon_ticks), 1)
    return sorted({max(1, T // d) for d in (1024, 256, 64, 16, 4)})


def tune_slab(run, horizon_ticks, reps=3, log=None):
    """run(slab_ticks): builds the tree with that slab width and queries it,
    returning the record list.  Returns (best slab_ticks, [(slab, ms)])."""
    results = []
    ref = None
    for w in slab_candidates(horizon_ticks):
        ms, out = _time_query(lambda: run(w), reps)
        if ref is None:
            ref = out.cpu()
        elif not torch.equal(out.cpu(), ref):
            raise RuntimeError(f"slab width {w} changed the record list")
        results.append((w, ms))
        if log:
            log(f"[tune] slab {w} ticks {ms:.3f} ms")
    return min(results, key=lambda r: r[1])[0], results


def tuned_slab(run, horizon_ticks, precision, boxes, dt_mode, path=None, reps=3, log=None):
    key = cache_key(precision, boxes, dt_mode, what="slab")
    cache = load_cache(path)
    if key in cache:
        return cache[key]["slab_ticks"], True
    best, results = tune_slab(run, horizon_ticks, reps=reps, log=log)
    cache[key] = {"slab_ticks": best, "ms": {str(w): ms for w, ms in results}}
    save_cache(cache, path)
    return best, False
