"""Launch-shape autotuner for the traversal.

Searches the fields of ``cd_tuning`` (node-pair workgroups per level and lanes
per workgroup, per-leaf-walk lanes, traversal mode) on a built tree, timing
the query alone (median of ``reps`` runs after one warm-up, device events on
the query's stream), and caches the best shape in a JSON file keyed by
(GPU architecture, tree precision, box-count bucket, step mode).  Every
candidate yields the same record list -- only time differs -- and ``tune``
checks that before it accepts a timing.
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
        for threads in (128, 256):
            out.append({"mode": 0, "expand_blocks": blocks, "expand_threads": threads,
                        "walk_threads": 256})
    for walk in (64, 128, 256):
        out.append({"mode": 1, "walk_threads": walk})
    return out


def cache_key(precision, boxes, dt_mode, arch=None):
    if arch is None:
        arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    bucket = int(round(math.log2(max(int(boxes), 1))))
    prec = "fp64" if precision == 0 else "fp32"
    return f"{arch}|{prec}|2^{bucket}|{dt_mode}"


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
