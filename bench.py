#!/usr/bin/env python3
"""Benchmark: one n-to-n broad-phase query on the 16 848-object tracked catalog.

A step is the whole hot path over one catalog resident in HBM: 4D boxes
(Kepler propagation + bounds), tree (keys, slab LDS sort, Karras hierarchy,
atomic refit), self-traversal and the canonical sorted, deduplicated pair
list, ending with the pair count on the host.

Prints one JSON line.  value = brute-force-equivalent box-pair tests per second
(different-object box pairs whose time tags overlap, K * C(n, 2) for a uniform
step, divided by the query time).  roofline: the stage with the largest device
time, its algorithmic bytes per launch over its mean duration, from HIP events
recorded on the library's stream during the timed steps.  cpu_baseline: the
CPU oracle (literal all-pairs) on a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps 10] [--warmup 3] [--precision fp64|fp32]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ms per n-to-n query and box-pair tests/s at n=16848, 1h horizon; HBM GB/s vs peak"
HBM_PEAK_GBS = 8000.0

# Measured HBM traffic per launch (rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE, KiB
# per dispatch, one counter per pass), scaled by what the same counters read for
# a 1 GiB device copy (FETCH 524308.56 KiB, WRITE 1048576 KiB).  Valid only for
# the kernel source it was taken on: reported as null once that file changes.
# Summary and commands: profiles/tracked16848_1h_fp64.md
COPY_FETCH_KIB, COPY_WRITE_KIB = 524308.5625, 1048576.0
TRAFFIC = {
    ("sort", "fp64", "fixed"): {"fetch_kib": 3621587.0, "write_kib": 5090350.0,
                       "source": "paper_1901_10475_amd/csrc/k_sort.hip",
                       "sha1": "6ca6284c7b18e59d6201e0b9a212d8c1bba54631"},
    ("refit", "fp64", "fixed"): {"fetch_kib": 2704670.0 + 300841.0 * 4, "write_kib": 3774597.0 + 93490 * 4,
                        "source": "paper_1901_10475_amd/csrc/k_tree.hip",
                        "sha1": "924db231a0b1ebdbfbb178721fe55c525f2abf65"},
}


def measured_traffic(stage, precision, dt_mode):
    import hashlib
    t = TRAFFIC.get((stage, precision, dt_mode))
    if not t:
        return None
    try:
        sha = hashlib.sha1(open(os.path.join(ROOT, t["source"]), "rb").read()).hexdigest()
    except OSError:
        return None
    if sha != t["sha1"]:
        return None
    return int(t["fetch_kib"] * 1024 * (1048576.0 / COPY_FETCH_KIB)
               + t["write_kib"] * 1024 * (1048576.0 / COPY_WRITE_KIB))


def algorithmic_bytes(stage, N, n, P, tree_prec, box_prec, seeds=0):
    """Compulsory HBM bytes of one launch of a stage: every input read once,
    every output written once (intermediate LDS traffic excluded)."""
    fb = 8 if box_prec == 0 else 4          # box float bytes
    box = 6 * fb + 12                         # lo/hi + t0, t1, obj
    node = 64 if tree_prec == 0 else 40       # tree record (box + links)
    nodes = 2 * N - 1
    table = {
        "boxes": N * box,                                    # boxes written
        "keys": 0,                                           # sampled frame only
        "sort": N * box + N * 8 + N * node,                  # slab build: boxes in; sorted
                                                             # keys and leaf records out
        "karras": N * 8 + (N - 1) * (8 + 1) + nodes * (8 + 4),  # keys in; kids, level,
                                                             # links, parents out
        "refit": N * node + nodes * 4 + (N - 1) * (8 + 8) + (N - 1) * node,
                                                             # leaf records, parents, kids
                                                             # and links in; inner records out
        "traverse": seeds * (8 + 2 * node) + P * 16,         # seed pairs and their nodes,
                                                             # records out
        "canon": P * 16 * 3,
    }
    return table.get(stage)


def time_overlap_pairs(dt, T):
    """Brute-force-equivalent test count for per-object steps: pairs of boxes of
    different objects whose half-open tags overlap.  Each object's tags tile
    [0, T + 1), so for objects i, j the overlapping box pairs are the pieces of
    the merged tiling: K_i + K_j - 1 - (interior boundaries they share), and
    the shared boundaries are the multiples of lcm(dt_i, dt_j) in [1, T - 1]."""
    import numpy as np
    n = len(dt)
    d = dt.astype(np.int64)
    K = np.ones(n, np.int64) if T == 0 else -(-T // d)
    total = (n - 1) * int(K.sum()) - n * (n - 1) // 2
    vals, cnt = np.unique(d, return_counts=True)
    for a in range(len(vals)):
        for b in range(a, len(vals)):
            m = (T - 1) // int(np.lcm(vals[a], vals[b])) if T > 0 else 0
            pairs = cnt[a] * (cnt[a] - 1) // 2 if a == b else cnt[a] * cnt[b]
            total -= int(pairs) * int(m)
    return total


def cpu_baseline(sc, seconds):
    """The CPU oracle on the first two steps of the hour (every object, t in
    [0, 2 s)): FP64 boxes, then literal all-pairs over those 2n boxes; repeated
    until `seconds` of wall time have passed."""
    import oracle
    n = sc.n
    T = 2 * sc.dt_ticks - 1          # intervals [0, dt) and [dt, 2 dt), as in the hour
    reps, t_start = 0, time.perf_counter()
    while True:
        b = oracle.boxes(sc.elements, sc.dt_ticks, T, sc.tick_s, sc.threshold_km)
        oracle.pairs(b)
        reps += 1
        el_t = time.perf_counter() - t_start
        if el_t >= seconds:
            break
    tests = reps * 2 * (n * (n - 1) // 2)
    return {"value": tests / el_t, "unit": "box-pair tests/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"first 2 s of the hour ({2 * n} boxes: {n} objects x 2 steps), oracle "
                      f"FP64 boxes + literal all-pairs, {reps} repetitions in {el_t:.1f} s; "
                      f"counted as 2 * C(n, 2) brute-force-equivalent tests per repetition"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64",
                    help="tree precision (boxes stay FP64 unless --boxes fp32)")
    ap.add_argument("--boxes", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--dt", choices=["fixed", "heuristic"], default="fixed",
                    help="fixed 1 s steps, or per-object steps bounding each box's motion "
                         "to 5 km (computed inside the timed step)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (a known-size "
                         "kernel for calibrating HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU only; --gpus must be 1 "
                                   "(multi-GPU sharding is a design note, not a run)"}))
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1901_10475_amd as cd
    from paper_1901_10475_amd import catalog

    torch.cuda.set_device(0)
    if args.copy_mib:
        src = torch.ones(args.copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    sc = catalog.tracked_hour()
    prec = cd.CD_FP64 if args.precision == "fp64" else cd.CD_FP32
    box_prec = cd.CD_FP64 if args.boxes == "fp64" else cd.CD_FP32
    el = cd.soa(sc.elements)
    p = cd.params_struct(sc.tick_s, sc.mu, sc.threshold_km, sc.horizon_ticks, sc.dt_ticks)
    heur = 5.0 if args.dt == "heuristic" else None
    workload = sc.name if heur is None else sc.name.replace("dt1s", "dt_heuristic5km")
    print(f"[bench] workload {workload}: n={sc.n} T={sc.horizon_ticks} ticks",
          file=sys.stderr, flush=True)
    bp = cd.BroadPhase(sc.n, p, None, box_prec, prec, dt_heuristic_km=heur, el_soa=el)
    N = bp.count
    for w in range(args.warmup):
        pairs = bp.run(el)
        print(f"[bench] warmup {w}: {len(pairs)} pairs", file=sys.stderr, flush=True)
    torch.cuda.synchronize()

    cd.cd_profile_read(reset=True)
    cd.cd_profile_enable(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        pairs = bp.run(el)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    cd.cd_profile_enable(False)
    stages = cd.cd_profile_read(reset=True)
    P = int(len(pairs))
    ms_step = wall * 1000.0 / args.steps
    if args.dt == "fixed":
        K = N // sc.n
        tests = K * sc.n * (sc.n - 1) // 2
    else:
        tests = time_overlap_pairs(bp.dt.cpu().numpy().view(np.uint32), sc.horizon_ticks)
    value = tests / (ms_step / 1000.0)
    print(f"[bench] {args.steps} steps: {ms_step:.3f} ms/query, {P} pairs, stages "
          + ", ".join(f"{k}={v[0] / v[1]:.3f}ms" for k, v in stages.items()),
          file=sys.stderr, flush=True)

    dom = max(stages, key=lambda k: stages[k][0])
    mean_ms = stages[dom][0] / stages[dom][1]
    nbytes = algorithmic_bytes(dom, N, sc.n, P, prec, box_prec)
    achieved = nbytes / (mean_ms / 1000.0) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(dom, args.precision, args.dt), "bytes_per_launch": int(nbytes),
                "mean_ms": round(mean_ms, 4)}

    out = {"metric": METRIC, "value": value, "unit": "box-pair tests/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if prec == cd.CD_FP64 else "f64 boxes, f32 tree",
           "data": "synthetic (seeded tracked-population catalog; the paper's TLE catalog is "
                   "not available)",
           "config": {"workload": workload,
                      "n": sc.n, "horizon_s": sc.horizon_ticks * sc.tick_s,
                      "dt_s": sc.dt_ticks * sc.tick_s if args.dt == "fixed" else "per-object",
                      "boxes": N, "threshold_km": sc.threshold_km,
                      "box_precision": args.boxes, "tree_precision": args.precision,
                      "brute_force_tests": tests},
           "pairs": P,
           "stages_ms": {k: round(v[0] / v[1], 4) for k, v in stages.items()},
           "roofline": roofline}
    if not args.no_cpu_baseline and args.dt == "fixed":
        print("[bench] CPU oracle baseline ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(sc, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
