#!/usr/bin/env python3
"""Benchmark: one n-to-n broad-phase query on the 16 848-object tracked catalog.

A step is the whole hot path over one catalog resident in HBM: 4D boxes
(Kepler propagation + bounds), tree (keys, slab LDS sort, Karras hierarchy,
atomic refit), self-traversal and the canonical sorted, deduplicated pair
list, ending with the pair count on the host.

Prints one JSON line.  value = brute-force-equivalent box-pair tests per second
(different-object box pairs whose time tags overlap, K * C(n, 2) for a uniform
step, divided by the query time).  roofline: the stage with the largest device
time (HIP events recorded by the library on its own stream during the timed
steps), its compulsory HBM bytes per launch (the hot-path scope's per-box
figures) over its mean duration, against the 8 TB/s specification and the
measured streaming-copy bandwidth; the same for every stage and for the whole
query.  learned_steps: the learned per-object step with FP32 boxes (eccentric-
anomaly and speed boxes) against this FP64 1 s line.  cpu_baseline: the CPU
oracle (FP64 boxes, bucketed all-pairs within each slab, canonical sort) on the
hour's first 60 slabs, on all host threads and on one.

    python bench.py [--gpus 1] [--steps 10] [--warmup 3] [--precision fp64|fp32]
                    [--boxes fp64|fp32] [--dt fixed|heuristic|mlp] [--workload tracked|batch]

Other workloads (not the default line): --dt heuristic (per-object steps
bounding each box's motion to 5 km), --dt mlp (per-object steps from the step
network, trained beforehand on step sweeps of two other catalogs of the same
recipe; the inference runs inside the timed step), --workload batch (64
independent scenarios of 2 000-50 000 objects, 30-minute horizons, 1 s steps,
replayed as one graph launch per step).
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

# Measured HBM traffic of one query's stage (rocprofv3 --pmc FETCH_SIZE, then
# WRITE_SIZE, KiB summed over the stage's dispatches of one query), scaled by
# what the same counters read for a 1 GiB device copy (FETCH 524308.4 KiB,
# WRITE 1048576 KiB).  Valid only for the kernel sources it was taken on:
# reported as null once one of them changes.  Summary and commands:
# profiles/tracked16848_1h_fp64.md
COPY_FETCH_KIB, COPY_WRITE_KIB = 524308.4375, 1048576.0
# box rule of cd_params (CD_BOX_SPEED, CD_BOX_INTERVAL_NU, CD_BOX_INTERVAL_E)
BOX_RULES = {"speed": 0, "nu": 1, "ecc": 2}
BOX_SUFFIX = {"speed": "", "nu": "_box_interval_nu", "ecc": "_box_interval_ecc"}

TRAFFIC = {
    # k_agglo_leaves + 8 item passes with their scans and compactions
    ("hierarchy", "fp64", "fixed"): {"fetch_kib": 2014019.7 + 57452.5 + 10084.2 + 154.1,
                                     "write_kib": 4469510.2 + 75683.7 + 13266.6 + 234.9,
                                     "sources": {"paper_1901_10475_amd/csrc/k_agglo.hip":
                                                 "5cd4ac788798fc9103eb37ffd7c0fbe8be30b23c"}},
    # k_block_codes + k_block_sort + k_boxes_uniform (records)
    ("boxes", "fp64", "fixed"): {"fetch_kib": 3205.6 + 38913.2 + 43762.8,
                                 "write_kib": 29615.6 + 109775.7 + 4114047.9,
                                 "sources": {"paper_1901_10475_amd/csrc/k_boxes.hip":
                                             "bf37f93ed5022344fdde388ad03e5b9b7779cc91",
                                             "paper_1901_10475_amd/csrc/k_sort.hip":
                                             "fb1eebe7f8229aa0d8e2160512a508b55f851817"}},
}


def measured_traffic(stage, precision, dt_mode):
    import hashlib
    t = TRAFFIC.get((stage, precision, dt_mode))
    if not t:
        return None
    for src, want in t["sources"].items():
        try:
            sha = hashlib.sha1(open(os.path.join(ROOT, src), "rb").read()).hexdigest()
        except OSError:
            return None
        if sha != want:
            return None
    return int(t["fetch_kib"] * 1024 * (1048576.0 / COPY_FETCH_KIB)
               + t["write_kib"] * 1024 * (1048576.0 / COPY_WRITE_KIB))


def compulsory_bytes(stage, N, P, tree_prec, box_prec, per_object_dt=False,
                     sorted_layout=False):
    """Compulsory HBM bytes of one launch of a stage, per box as the hot-path
    scope's measurement section counts them (FP64: boxes 56 + keys 12, per-slab
    sort 24, hierarchy 16, refit 112, traversal 120 plus 16 per record; 340 B
    per box in all), scaled to the FP32 layouts (32-byte leaf boxes, 40-byte
    nodes).  The box stage writes the keys with the boxes, so it is credited
    with both; with the sorted layout it also puts every slab in Morton order
    (no sort stage runs), so it is credited with the sort's bytes too."""
    fb = 8 if box_prec == 0 else 4
    box = 6 * fb + 8 + (4 if per_object_dt else 0)   # bounds, tags (+ object id)
    node = 64 if tree_prec == 0 else 40
    leaf = 56 if tree_prec == 0 else 32
    table = {
        "boxes": N * (box + 12 + (24 if sorted_layout else 0)),   # boxes and keys written
                                               # (and the slab order formed)
        "keys": 0,                             # folded into the box stage
        "sort": N * 24,                        # keys and indices read and written once
        "karras": N * 16,                      # children and parents written
        "refit": N * 2 * leaf,                 # one sibling box read, one node box written
        "hierarchy": N * (16 + 2 * leaf),      # hierarchy and refit in one pass
        "traverse": (N - 1) * node + N * leaf + P * 16,   # every node once, records out
        "canon": P * 32,                       # records read and written once
    }
    return table.get(stage)


def design_bytes(stage, N, n, P, tree_prec, box_prec, sorted_layout=False):
    """What this implementation's kernels are built to move per launch (every
    input it reads once, every output it writes once, LDS traffic excluded):
    the slab build, for one, materialises 64-byte sorted leaf records, which
    the scope's per-slab sort of keys and indices does not."""
    fb = 8 if box_prec == 0 else 4          # box float bytes
    box = 6 * fb + 12                         # lo/hi + t0, t1, obj
    node = 64 if tree_prec == 0 else 40       # tree record (box + links)
    nodes = 2 * N - 1
    table = {
        "boxes": N * (box + 4),                              # boxes and codes written
        "keys": 0,                                           # sampled frame only
        "sort": N * (4 + 4) + N * box + N * 4 + N * node,    # slab build: codes and tags,
                                                             # then boxes in; sorted codes
                                                             # and leaf records out
        "karras": N * (8 if sorted_layout else 4) + (N - 1) * (8 + 1) + nodes * (8 + 4),
                                                             # codes (and tags) in; kids,
                                                             # level, links, parents out
        "refit": (N * (box + node) if sorted_layout else N * node)
                 + nodes * 4 + (N - 1) * (8 + 4) + (N - 1) * node,
                                                             # leaf records (sorted layout:
                                                             # boxes in, leaf records out),
                                                             # parents, kids and escapes in;
                                                             # inner records out
        "hierarchy": N * (node + 4) + (N - 1) * (node + 8) + N * 4,
                                                             # bottom-up pass: leaf records
                                                             # and codes in; inner records,
                                                             # children, leaf skip links out
        "traverse": nodes * node + P * 16,                   # every node read once,
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


def host_cpu():
    """(logical CPUs usable by this process, CPU model name)."""
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return usable, model


def cpu_baseline(sc, slabs=60):
    """The CPU oracle end to end on the first `slabs` steps of the hour (every
    object, t in [0, slabs dt)): FP64 boxes, the bucketed driver (all pairs
    within each slab) and the canonical sort, once on all threads and once on
    one thread.  slabs * C(n, 2) brute-force-equivalent tests per run."""
    import oracle
    n = sc.n
    T = slabs * sc.dt_ticks - 1      # intervals [k dt, (k + 1) dt), k < slabs, as in the hour
    tests = slabs * (n * (n - 1) // 2)
    threads_all = oracle.num_threads()
    runs = {}
    for nt in (threads_all, 1):
        oracle.set_num_threads(nt)
        t_start = time.perf_counter()
        b = oracle.boxes(sc.elements, sc.dt_ticks, T, sc.tick_s, sc.threshold_km)
        rec = oracle.pairs_bucketed(b)
        el_t = time.perf_counter() - t_start
        runs[nt] = (el_t, len(rec))
    oracle.set_num_threads(threads_all)
    usable, model = host_cpu()
    t_all, P = runs[threads_all]
    t_one, _ = runs[1]
    return {"value": tests / t_all, "unit": "box-pair tests/s", "cores": threads_all,
            "kind": "oracle",
            "sample": f"first {slabs} s of the hour ({slabs * n} boxes: {n} objects x {slabs} "
                      f"steps, {P} records): oracle FP64 boxes + bucketed pairs (all pairs "
                      f"within each slab) + canonical sort, end to end, {t_all:.2f} s on "
                      f"{threads_all} threads; {slabs} * C(n, 2) brute-force-equivalent tests",
            "single_thread": {"value": tests / t_one, "seconds": round(t_one, 3)},
            "host": {"usable_cpus": usable, "cpu_model": model},
            "ms_per_query_extrapolated": round(t_all * 1000.0 * (sc.horizon_ticks // sc.dt_ticks)
                                               / slabs, 1)}


def _setup(args):
    import torch
    torch.cuda.set_device(0)
    args.copy = None if args.no_copy else copy_bandwidth()
    if args.copy_mib:
        src = torch.ones(args.copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst


def copy_bandwidth(nbytes=4 << 30, reps=10):
    """The library's streaming copy (cd_stream_copy) over nbytes: read + write
    bytes over the median time, GB/s: the achievable HBM bandwidth."""
    import torch
    import paper_1901_10475_amd as cd
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    cd.cd_stream_copy(dst, src)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for a, b in ev:
        a.record()
        cd.cd_stream_copy(dst, src)
        b.record()
    torch.cuda.synchronize()
    ms = sorted(a.elapsed_time(b) for a, b in ev)[reps // 2]
    ok = bool(torch.equal(dst[:: 1 << 20], src[:: 1 << 20]))
    del src, dst
    torch.cuda.empty_cache()
    gbs = 2 * nbytes / (ms / 1000.0) / 1e9
    return {"kernel": "cd_stream_copy", "bytes": 2 * nbytes, "ms": round(ms, 4),
            "achieved": round(gbs, 1), "unit": "GB/s", "frac_of_spec": round(gbs / HBM_PEAK_GBS, 4),
            "copied_correctly": ok}


def _roofline(stages, N, n, P, prec, box_prec, precision_name, dt_mode, ms_step, copy=None,
              sorted_layout=False):
    """Roofline of the dominant stage (largest device time) with the scope's
    compulsory bytes, plus every stage and the whole query the same way."""
    per_obj = dt_mode != "fixed"
    dom = max(stages, key=lambda k: stages[k][0])
    mean_ms = stages[dom][0] / stages[dom][1]
    nbytes = compulsory_bytes(dom, N, P, prec, box_prec, per_obj, sorted_layout)
    achieved = nbytes / (mean_ms / 1000.0) / 1e9
    out = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
           "traffic": measured_traffic(dom, precision_name, dt_mode),
           "bytes_per_launch": int(nbytes), "mean_ms": round(mean_ms, 4),
           "bytes_rule": "compulsory bytes per box of the scope's measurement section"}
    per_stage = {}
    total = 0
    for k, (ms_tot, launches) in stages.items():
        b = compulsory_bytes(k, N, P, prec, box_prec, per_obj, sorted_layout) or 0
        ms = ms_tot / launches
        total += b
        per_stage[k] = {"mean_ms": round(ms, 4), "bytes": int(b),
                        "frac": round(b / (ms / 1000.0) / 1e9 / HBM_PEAK_GBS, 4) if ms > 0 else None,
                        "traffic": measured_traffic(k, precision_name, dt_mode)}
    out["stages"] = per_stage
    wq = total / (ms_step / 1000.0) / 1e9
    out["whole_query"] = {"bytes": int(total), "ms": round(ms_step, 4), "achieved": round(wq, 1),
                          "frac": round(wq / HBM_PEAK_GBS, 4),
                          "floor_ms": round(total / (HBM_PEAK_GBS * 1e9) * 1000.0, 4)}
    db = design_bytes(dom, N, n, P, prec, box_prec, sorted_layout)
    out["design_bytes"] = {"bytes_per_launch": int(db),
                           "achieved": round(db / (mean_ms / 1000.0) / 1e9, 1),
                           "note": "bytes this implementation's kernel is built to move "
                                   "(it materialises sorted leaf records); not the roofline"}
    if copy:
        out["copy_peak"] = copy["achieved"]
        out["frac_of_copy_peak"] = round(achieved / copy["achieved"], 4)
        out["whole_query"]["frac_of_copy_peak"] = round(wq / copy["achieved"], 4)
    return out


def _train_step_net(sc_recipe, seeds, cd, ld, catalog, log, box_rule=0):
    """Step network trained on step sweeps of catalogs drawn from the same
    recipe with other seeds (outside the timed region), with the box rule of
    the query it will serve."""
    import torch
    xs, ts = [], []
    for seed in seeds:
        sc = sc_recipe(seed)
        p = cd.params_struct(sc.tick_s, sc.mu, sc.threshold_km, sc.horizon_ticks, 0,
                             box_rule=box_rule)
        x, t, summary = ld.sweep_targets(cd.soa(sc.elements), p)
        log(f"[bench] sweep seed {seed}: " + ", ".join(
            f"x{r['scale']:g}: {r['boxes']} boxes {r['records']} rec" for r in summary))
        xs.append(x)
        ts.append(t)
    X, Y = torch.cat(xs), torch.cat(ts)
    net = ld.StepNet(seed=0)
    net.set_output_bias(float(Y.mean().item()))
    losses = net.train(X, Y, steps=1000, lr=3e-3, lr_end=1e-4)
    log(f"[bench] step network: loss {losses[0]:.4f} -> {losses[-1]:.4f} "
        f"(target variance {float(Y.var().item()):.4f})")
    return net


def run_tracked(args, log):
    import numpy as np
    import torch
    import paper_1901_10475_amd as cd
    from paper_1901_10475_amd import catalog
    from paper_1901_10475_amd import learned_dt as ld

    sc = catalog.tracked_hour()
    prec = cd.CD_FP64 if args.precision == "fp64" else cd.CD_FP32
    box_prec = cd.CD_FP64 if args.boxes == "fp64" else cd.CD_FP32
    el = cd.soa(sc.elements)
    p = cd.params_struct(sc.tick_s, sc.mu, sc.threshold_km, sc.horizon_ticks,
                         sc.dt_ticks if args.dt == "fixed" else 0, box_rule=BOX_RULES[args.box])
    workload = {"fixed": sc.name,
                "heuristic": sc.name.replace("dt1s", f"dt_heuristic{args.heur_km:g}km"),
                "mlp": sc.name.replace("dt1s", "dt_mlp")}[args.dt] + BOX_SUFFIX[args.box]
    log(f"[bench] workload {workload}: n={sc.n} T={sc.horizon_ticks} ticks")
    kw = {}
    if args.dt == "heuristic":
        kw = {"dt_heuristic_km": args.heur_km, "el_soa": el}
    elif args.dt == "mlp":
        net = _train_step_net(lambda seed: catalog.tracked_hour(seed=seed, planted=0),
                              (2002, 2003), cd, ld, catalog, log, BOX_RULES[args.box])
        kw = {"dt_mlp": (net.w_bf16, 5.0), "el_soa": el}
    bp = cd.BroadPhase(sc.n, p, None, box_prec, prec, **kw)
    N = bp.count
    for w in range(args.warmup):
        pairs = bp.run(el)
        log(f"[bench] warmup {w}: {len(pairs)} pairs")
    torch.cuda.synchronize()

    cd.cd_profile_read(reset=True)
    cd.cd_profile_enable(True)
    # events on the caller's stream around every step, for the median
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e0, e1 in evs:
        e0.record()
        pairs = bp.run(el)
        e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    cd.cd_profile_enable(False)
    stages = cd.cd_profile_read(reset=True)
    P = int(len(pairs))
    ms_step = wall * 1000.0 / args.steps
    ms_events = sorted(e0.elapsed_time(e1) for e0, e1 in evs)
    ms_median = ms_events[len(ms_events) // 2] if len(ms_events) % 2 else \
        0.5 * (ms_events[len(ms_events) // 2 - 1] + ms_events[len(ms_events) // 2])
    # transfers outside the timed region: the catalog in, the pair list out
    torch.cuda.synchronize()
    t_h = time.perf_counter()
    el_copy = cd.soa(sc.elements)
    torch.cuda.synchronize()
    h2d_ms = (time.perf_counter() - t_h) * 1000.0
    t_h = time.perf_counter()
    pairs_host = pairs.cpu()
    d2h_ms = (time.perf_counter() - t_h) * 1000.0
    del el_copy, pairs_host
    if args.dt == "fixed":
        K = N // sc.n
        tests = K * sc.n * (sc.n - 1) // 2
    else:
        tests = time_overlap_pairs(bp.dt.cpu().numpy().view(np.uint32), sc.horizon_ticks)
    value = tests / (ms_step / 1000.0)
    log(f"[bench] {args.steps} steps: {ms_step:.3f} ms/query, {P} pairs, stages "
        + ", ".join(f"{k}={v[0] / v[1]:.3f}ms" for k, v in stages.items()))
    recall = planted_recall(sc, pairs)
    out = {"metric": METRIC, "value": value, "unit": "box-pair tests/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if prec == cd.CD_FP64 and box_prec == cd.CD_FP64 else
                    ("f64 boxes, f32 tree" if box_prec == cd.CD_FP64 else "f32 boxes, f32 tree"),
           "data": "synthetic (seeded tracked-population catalog; the paper's TLE catalog is "
                   "not available)",
           "config": {"workload": workload,
                      "n": sc.n, "horizon_s": sc.horizon_ticks * sc.tick_s,
                      "dt_s": sc.dt_ticks * sc.tick_s if args.dt == "fixed" else "per-object",
                      "boxes": N, "threshold_km": sc.threshold_km,
                      "box_precision": args.boxes, "tree_precision": args.precision,
                      "box_rule": args.box, "brute_force_tests": tests},
           "pairs": P, "planted_recall": recall,
           "ms_per_step_median_events": round(ms_median, 4),
           "transfers_ms": {"catalog_h2d": round(h2d_ms, 3), "pairs_d2h": round(d2h_ms, 3),
                            "note": "outside the timed region; pageable host memory"},
           "stages_ms": {k: round(v[0] / v[1], 4) for k, v in stages.items()},
           "roofline": _roofline(stages, N, sc.n, P, prec, box_prec, args.precision, args.dt,
                                 ms_step, args.copy,
                                 bp.boxes.desc.layout == cd.CD_LAYOUT_SORTED)}
    out["config"]["box_layout"] = ("sorted" if bp.boxes.desc.layout == cd.CD_LAYOUT_SORTED
                                   else "object")
    if args.copy:
        out["hbm_copy"] = args.copy
    out["executed_tests"] = executed_tests(cd, bp, N, tests, ms_step, log)
    out["narrow_phase"] = narrow_phase(cd, el, p, pairs, log)
    default_line = (args.dt == "fixed" and prec == cd.CD_FP64 and box_prec == cd.CD_FP64
                    and args.box == "speed")
    if default_line and not args.no_learned_steps:
        out["learned_steps"] = learned_step_forms(args, log, sc, el, {
            "ms_per_query": round(ms_step, 4), "boxes": N, "records": P,
            "planted_recall": recall,
            "colliding_object_pairs": out["narrow_phase"]["colliding_object_pairs"]})
    if not args.no_cpu_baseline and args.dt == "fixed":
        log("[bench] CPU oracle baseline ...")
        out["cpu_baseline"] = cpu_baseline(sc, args.cpu_slabs)
    return out


def executed_tests(cd, bp, N, brute_force, ms_step, log):
    """4D box-box tests the tree actually executes for one query (the
    counters build, libcd4d_counters.so, one query outside the timed region):
    the traversal's tests plus the build's one sibling test per inner node,
    per second at the timed query rate."""
    with cd.counters_build():
        cd.cd_counters_reset(None)
        bp.query()
        c = cd.cd_counters_read()
    total = c["tests"] + max(N - 1, 0)
    rate = total / (ms_step / 1000.0)
    log(f"[bench] executed tests: {c['tests']} in the traversal + {max(N - 1, 0)} sibling "
        f"tests = {total} ({rate:.3e}/s at the timed rate; brute force {brute_force})")
    return {"per_query": total, "traversal": c, "build_sibling_tests": max(N - 1, 0),
            "per_s": rate, "brute_force_per_executed": round(brute_force / max(total, 1), 1),
            "from": "CD_COUNTERS build, one query outside the timed region"}


def planted_recall(sc, pairs):
    """Share of the planted conjunctions (i, j, t) covered by a record."""
    import numpy as np
    if not sc.planted:
        return None
    pr = pairs.cpu().numpy().view(np.uint32)
    hit = sum(bool(((pr[:, 0] == i) & (pr[:, 1] == j) & (pr[:, 2] <= t)
                    & (t < pr[:, 3])).any()) for i, j, t in sc.planted)
    return hit / len(sc.planted)


def colliding_object_pairs(cd, el, p, pairs, delta=1):
    """Distinct object pairs with a collision instant on the delta grid (the
    narrow phase over the records): the true collisions every conservative
    form must keep."""
    import torch
    if pairs.shape[0] == 0:
        return 0
    wit, _ = cd.cd_first_witness(el, p, delta, pairs)
    hp = pairs[wit != -1][:, :2].long()
    return int(torch.unique(hp[:, 0] * (1 << 32) + hp[:, 1]).numel()) if hp.shape[0] else 0


def learned_step_forms(args, log, sc, el, base):
    """The learned per-object step with FP32 outward-rounded boxes and tree,
    with the eccentric-anomaly interval box and with the speed box, against the
    plain FP64 form at 1 s (the default line): ms per query over the same
    number of timed steps, planted recall and colliding object pairs.  Each
    network is trained first (step sweeps of two other catalogs of the same
    recipe, outside the timed region); its BF16 inference runs inside every
    timed step.  The traversal's launch shapes for each form come from the
    autotuner (the 256-lane default suits the FP64 line; the FP32 per-object
    trees run faster with 512), searched outside the timed region."""
    import torch
    import paper_1901_10475_amd as cd
    from paper_1901_10475_amd import autotune, catalog
    from paper_1901_10475_amd import learned_dt as ld
    out = {"fp64_dt1s_speed_box": base}
    for rule_name in ("ecc", "speed"):
        rule = BOX_RULES[rule_name]
        t_train = time.perf_counter()
        net = _train_step_net(lambda seed: catalog.tracked_hour(seed=seed, planted=0),
                              (2002, 2003), cd, ld, catalog, log, rule)
        t_train = time.perf_counter() - t_train
        p = cd.params_struct(sc.tick_s, sc.mu, sc.threshold_km, sc.horizon_ticks, 0,
                             box_rule=rule)
        bp = cd.BroadPhase(sc.n, p, None, cd.CD_FP32, cd.CD_FP32, dt_mlp=(net.w_bf16, 5.0),
                           el_soa=el)
        bp.run(el)
        # the traversal's launch shapes from the autotuner (cached per GPU
        # architecture and box-count bucket; outside the timed region)
        shapes, cached = autotune.tuned(bp.query, cd.CD_FP32, bp.count, f"mlp_{rule_name}")
        cd.cd_set_tuning(shapes)
        try:
            for _ in range(args.warmup):
                pairs = bp.run(el)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                pairs = bp.run(el)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1000.0 / args.steps
        finally:
            cd.cd_set_tuning(None)
        form = {"ms_per_query": round(ms, 4), "boxes": int(bp.count),
                "records": int(pairs.shape[0]), "planted_recall": planted_recall(sc, pairs),
                "colliding_object_pairs": colliding_object_pairs(cd, el, p, pairs),
                "speedup_vs_fp64_dt1s": round(base["ms_per_query"] / ms, 3),
                "training_s": round(t_train, 1), "launch_shapes": shapes}
        log(f"[bench] learned steps, FP32, {rule_name} box: {ms:.3f} ms/query, "
            f"{form['boxes']} boxes, {form['records']} records, recall "
            f"{form['planted_recall']}, {form['colliding_object_pairs']} colliding pairs")
        out[f"learned_fp32_{rule_name}_box"] = form
        del bp, pairs, net
        torch.cuda.empty_cache()
    return out


def narrow_phase(cd, el, p, pairs, log, delta=1, reps=5):
    """The first collision instant of every record at every tick (delta = 1),
    timed after the broad-phase steps (it is not part of a step)."""
    import torch
    wit, first = cd.cd_first_witness(el, p, delta, pairs)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for a, b in ev:
        a.record()
        wit, first = cd.cd_first_witness(el, p, delta, pairs)
        b.record()
    torch.cuda.synchronize()
    ms = sorted(a.elapsed_time(b) for a, b in ev)[reps // 2]
    fc = cd.first_collision(pairs, first)
    hit = wit != -1
    hits = int(hit.sum().item())
    # distinct object pairs with a collision in the horizon: the same set for
    # every step and box rule, since every rule's boxes are conservative
    hp = pairs[hit][:, :2].long()
    colliding = int(torch.unique(hp[:, 0] * (1 << 32) + hp[:, 1]).numel()) if hits else 0
    log(f"[bench] narrow phase (delta {delta} tick): {ms:.3f} ms, {hits} records with a "
        f"collision, first {fc}")
    # bulk interval refinement of the same records down to single instants:
    # every collision instant (the speed box gives exactly those; the interval
    # boxes add instants within their 1e-10 rad widening)
    leaves = cd.cd_refine_records(el, p, delta, pairs)
    ev2 = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    for a, b in ev2:
        a.record()
        leaves = cd.cd_refine_records(el, p, delta, pairs)
        b.record()
    torch.cuda.synchronize()
    rms = sorted(a.elapsed_time(b) for a, b in ev2)[reps // 2]
    lp = leaves[:, :2].long()
    lpairs = int(torch.unique(lp[:, 0] * (1 << 32) + lp[:, 1]).numel()) if len(leaves) else 0
    log(f"[bench] refinement to single instants: {rms:.3f} ms, {len(leaves)} collision "
        f"instants, {lpairs} object pairs")
    return {"delta_ticks": delta, "ms": round(ms, 4), "records": int(pairs.shape[0]),
            "refine": {"ms": round(rms, 4), "min_steps": 1, "leaves": int(len(leaves)),
                       "colliding_object_pairs": lpairs},
            "records_with_collision": hits, "colliding_object_pairs": colliding,
            "first_collision": None if fc is None else {"t_ticks": fc[0], "i": fc[1],
                                                        "j": fc[2]}}


def run_batch(args, log):
    """64 uneven scenarios, one graph launch per step."""
    import torch
    import paper_1901_10475_amd as cd
    from paper_1901_10475_amd import catalog
    from paper_1901_10475_amd.batch import BatchRunner

    prec = cd.CD_FP64 if args.precision == "fp64" else cd.CD_FP32
    box_prec = cd.CD_FP64 if args.boxes == "fp64" else cd.CD_FP32
    sizes = catalog.batch_sizes()
    scs = [catalog.batch_member(s, n) for s, n in enumerate(sizes)]
    br = BatchRunner(scs, box_prec, prec)
    log(f"[bench] batch: {len(scs)} scenarios, n {min(sizes)}..{max(sizes)}, "
        f"{br.boxes_total()} boxes")
    # eager pass with stage timing: capacities, and the per-kernel breakdown
    cd.cd_profile_read(reset=True)
    cd.cd_profile_enable(True)
    br.calibrate()
    cd.cd_profile_enable(False)
    stages = cd.cd_profile_read(reset=True)
    def timed_replays(label):
        br.capture()
        log(f"[bench] batch captured ({label} launch shapes)")
        for w in range(args.warmup):
            br.replay()
            res = br.results()
            log(f"[bench] warmup {w}: {sum(int(r.shape[0]) for r in res)} pairs")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            br.replay()
        br.stream.synchronize()
        wall = time.perf_counter() - t0
        res = br.results()
        return wall * 1000.0 / args.steps, res

    ms_default, res_default = timed_replays("default")
    # launch shapes from the autotuner, one search per box-count bucket
    # (cached per GPU architecture; outside the timed region)
    chosen = br.autotune(log=None)
    log("[bench] tuned buckets: " + ", ".join(
        f"{k.split('|')[2]}: {v[0]}{' (cached)' if v[1] else ''}" for k, v in chosen.items()))
    ms_step, res = timed_replays("tuned")
    P = sum(int(r.shape[0]) for r in res)
    assert P == sum(int(r.shape[0]) for r in res_default)
    tests = br.brute_force_tests()
    log(f"[bench] {args.steps} replays: {ms_step:.3f} ms/batch tuned, {ms_default:.3f} ms/batch "
        f"default, {P} pairs; eager stages "
        + ", ".join(f"{k}={v[0]:.1f}ms/{v[1]}" for k, v in stages.items()))
    # roofline of the dominant stage over the eager pass (all scenarios)
    dom = max(stages, key=lambda k: stages[k][0])
    nbytes = sum(compulsory_bytes(dom, N, 0, prec, box_prec)
                 for s, N in zip(scs, br.counts))
    achieved = nbytes / (stages[dom][0] / 1000.0) / 1e9
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None, "bytes_per_launch": int(nbytes / len(scs)),
            "mean_ms": round(stages[dom][0] / stages[dom][1], 4),
            "from": "eager pass over the batch (stage timing is off inside graphs)"}
    return {"metric": METRIC, "value": tests / (ms_step / 1000.0), "unit": "box-pair tests/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None,
            "dtype": "f64" if prec == cd.CD_FP64 and box_prec == cd.CD_FP64 else "f32 tree",
            "data": "synthetic (seeded LEO scenarios)",
            "config": {"workload": f"batch64_leo_30min_dt1s", "scenarios": len(scs),
                       "branches": len(br.branch_streams),
                       "n_min": min(sizes), "n_max": max(sizes), "boxes": br.boxes_total(),
                       "brute_force_tests": tests, "graph": "one launch per step",
                       "in_tree_scenarios": int(sum(br.in_tree)),
                       "launch_shapes": "autotuned per box-count bucket"},
            "ms_per_step_default_shapes": round(ms_default, 4),
            "pairs": P, "stages_ms_eager_total": {k: round(v[0], 3) for k, v in stages.items()},
            "roofline": roof}


def run_debris(args, log):
    """100 000-object projected-debris catalog over 6 h in consecutive
    windows (each the same problem over its own time interval), FP32 boxes,
    per-object steps from the speed bound or from the step network."""
    import numpy as np
    import torch
    import paper_1901_10475_amd as cd
    from paper_1901_10475_amd import catalog
    from paper_1901_10475_amd import learned_dt as ld

    sc = catalog.projected_debris()
    T = sc.horizon_ticks
    W = int(args.window_s * 1000)
    nwin = -(-T // W)
    if T % W:
        raise SystemExit("the window must divide the horizon")
    prec = cd.CD_FP64 if args.precision == "fp64" else cd.CD_FP32
    box_prec = cd.CD_FP64 if args.boxes == "fp64" else cd.CD_FP32
    el = cd.soa(sc.elements)
    p = cd.params_struct(sc.tick_s, sc.mu, sc.threshold_km, W, 0, box_rule=BOX_RULES[args.box])
    if args.dt == "mlp":
        net = _train_step_net(
            lambda seed: catalog.projected_debris(seed=seed, horizon_ticks=300_000, planted=0),
            (5002, 5003), cd, ld, catalog, log, BOX_RULES[args.box])
        kw = {"dt_mlp": (net.w_bf16, 5.0), "el_soa": el}
    elif args.dt == "heuristic":
        kw = {"dt_heuristic_km": args.heur_km, "el_soa": el}
    else:
        raise SystemExit("the debris catalog takes per-object steps (--dt heuristic|mlp)")
    workload = (f"{sc.name}_dt_{'mlp' if args.dt == 'mlp' else f'heuristic{args.heur_km:g}km'}"
                + BOX_SUFFIX[args.box])
    bp = cd.BroadPhase(sc.n, p, None, box_prec, prec, **kw)
    log(f"[bench] workload {workload}: n={sc.n}, {nwin} windows of {W} ticks, "
        f"{bp.count} boxes per window")

    def query():
        # record counts per window (each window's list is overwritten by the next)
        recs = []
        for w in range(nwin):
            bp.params.start_ticks = w * W
            recs.append(bp.run(el))
        return recs

    for k in range(args.warmup):
        recs = query()
        log(f"[bench] warmup {k}: {sum(int(r.shape[0]) for r in recs)} records")
    torch.cuda.synchronize()
    cd.cd_profile_read(reset=True)
    cd.cd_profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        recs = query()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    cd.cd_profile_enable(False)
    stages = cd.cd_profile_read(reset=True)
    ms_step = wall * 1000.0 / args.steps
    P = sum(int(r.shape[0]) for r in recs)
    dt = bp.dt.cpu().numpy().view(np.uint32)
    tests = nwin * time_overlap_pairs(dt, W)
    # recall: every window again, each checked before the next overwrites the
    # shared output buffer
    hit = 0
    for w in range(nwin):
        bp.params.start_ticks = w * W
        pr = bp.run(el).cpu().numpy().view(np.uint32)
        for i, j, t in sc.planted:
            if min(t // W, nwin - 1) != w:
                continue
            tl = t - w * W
            hit += bool(((pr[:, 0] == i) & (pr[:, 1] == j) & (pr[:, 2] <= tl)
                         & (tl < pr[:, 3])).any())
    log(f"[bench] {args.steps} steps: {ms_step:.3f} ms per 6 h query, {P} records, "
        f"recall {hit}/{len(sc.planted)}, stages "
        + ", ".join(f"{k}={v[0] / v[1]:.3f}ms" for k, v in stages.items()))
    return {"metric": METRIC, "value": tests / (ms_step / 1000.0), "unit": "box-pair tests/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None,
            "dtype": "f32 boxes, f32 tree" if box_prec == cd.CD_FP32 else "f64",
            "data": "synthetic (seeded projected-debris catalog with fragment clouds)",
            "config": {"workload": workload, "n": sc.n, "horizon_s": T * sc.tick_s,
                       "windows": nwin, "boxes": bp.count * nwin,
                       "threshold_km": sc.threshold_km, "brute_force_tests": tests,
                       "dt_median_s": float(np.median(dt)) * sc.tick_s},
            "pairs": P, "planted_recall": hit / max(len(sc.planted), 1),
            "stages_ms": {k: round(v[0] / v[1], 4) for k, v in stages.items()},
            "roofline": _roofline(stages, bp.count, sc.n, P // nwin, prec, box_prec,
                                  args.precision, args.dt, ms_step / nwin, args.copy)}


def run_bands(args, log):
    """The tracked hour as altitude-band sub-problems (the potential-collision
    graph's edge partition), run one after another on the one GPU."""
    import numpy as np
    import torch
    import paper_1901_10475_amd as cd
    from paper_1901_10475_amd import catalog
    from paper_1901_10475_amd.bands import BandRunner

    sc = catalog.tracked_hour()
    prec = cd.CD_FP64 if args.precision == "fp64" else cd.CD_FP32
    box_prec = cd.CD_FP64 if args.boxes == "fp64" else cd.CD_FP32
    el = cd.soa(sc.elements)
    p = cd.params_struct(sc.tick_s, sc.mu, sc.threshold_km, sc.horizon_ticks, sc.dt_ticks,
                         box_rule=BOX_RULES[args.box])
    runner = BandRunner(el, p, args.bands, box_precision=box_prec, tree_precision=prec)
    sizes = runner.sizes()
    log(f"[bench] bands: {args.bands} bands, objects per band {[s_[0] for s_ in sizes]}")
    for w in range(args.warmup):
        pairs = runner.run(el)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        pairs = runner.run(el)
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1000.0 / args.steps
    band_ms = []
    runner.run(el, band_ms=band_ms)
    # outside the timed region: the whole catalog's records, band-filtered
    full_bp = cd.BroadPhase(sc.n, p, None, box_prec, prec)
    full = cd.cd_band_filter(el, p, full_bp.run(el).clone())
    same = bool(torch.equal(full.cpu(), pairs.cpu()))
    del full_bp
    K = sc.horizon_ticks // sc.dt_ticks
    tests = K * sc.n * (sc.n - 1) // 2
    dup = sum(s_[0] for s_ in sizes) / sc.n
    log(f"[bench] bands: {ms_step:.3f} ms for all bands in turn, slowest band "
        f"{max(band_ms):.3f} ms, duplication {dup:.3f}, {len(pairs)} records, equal to the "
        f"filtered whole catalog: {same}")
    return {"metric": METRIC, "value": tests / (ms_step / 1000.0), "unit": "box-pair tests/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64" if prec == cd.CD_FP64 else "f32 tree",
            "data": "synthetic (seeded tracked-population catalog)",
            "config": {"workload": f"{sc.name}_bands{args.bands}" + BOX_SUFFIX[args.box],
                       "n": sc.n, "bands": args.bands, "box_rule": args.box},
            "bands": {"objects": [s_[0] for s_ in sizes], "boxes": [s_[1] for s_ in sizes],
                      "ms": [round(x, 4) for x in band_ms], "slowest_ms": round(max(band_ms), 4),
                      "duplication": round(dup, 4), "records": int(len(pairs)),
                      "equals_filtered_catalog": same}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64",
                    help="tree precision (boxes stay FP64 unless --boxes fp32)")
    ap.add_argument("--boxes", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--box", choices=list(BOX_RULES), default="speed",
                    help="occ-int of a box: speed bound, or interval evaluation over the "
                         "true (nu) or eccentric (ecc) anomaly")
    ap.add_argument("--dt", choices=["fixed", "heuristic", "mlp"], default="fixed",
                    help="fixed 1 s steps; per-object steps bounding each box's motion to "
                         "5 km; or per-object steps from the trained step network")
    ap.add_argument("--heur-km", type=float, default=5.0,
                    help="largest displacement per interval of the speed-bound step")
    ap.add_argument("--workload", choices=["tracked", "batch", "debris", "bands"],
                    default="tracked")
    ap.add_argument("--bands", type=int, default=8,
                    help="bands workload: altitude bands of the edge partition")
    ap.add_argument("--window-s", type=float, default=1800.0,
                    help="debris workload: window length in seconds (divides 6 h)")
    ap.add_argument("--cpu-slabs", type=int, default=60,
                    help="CPU baseline: the oracle over the hour's first this many 1 s slabs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned-steps", action="store_true",
                    help="default line: skip the learned-step FP32 forms")
    ap.add_argument("--no-copy", action="store_true",
                    help="skip the streaming-copy bandwidth measurement")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (a known-size "
                         "kernel for calibrating HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "only one GPU is measured; --gpus must be 1 (how the path "
                                   "would shard over several GPUs is described, not run)"}))
        sys.exit(2)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    _setup(args)
    run = {"tracked": run_tracked, "batch": run_batch, "debris": run_debris,
           "bands": run_bands}[args.workload]
    out = run(args, log)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
