"""Full-size parity against the bucketed oracle (Alg. Brute Force's pair test
over every pair of boxes whose time tags overlap), on the GPU's own boxes.

* The benchmark workload (16 848 objects, 1 h, 1 s steps, 60.65 M boxes,
  FP64): every record, slab by slab, plus a check that each record's two boxes
  overlap in 4D.
* Per-object steps (each box's motion bounded by 5 km, 79.7 M boxes), FP64 and
  FP32 outward-rounded boxes: four 45-second windows (5 % of the hour).
* Scenarios of the uneven 64-scenario batch (30-minute horizons), replayed
  from one captured graph: the smallest in full, two large ones on windows.
* The 100 000-object projected-debris catalog (6 h in 30-minute windows,
  FP32 boxes, per-object steps): sub-windows of two windows.

A window [ta, tb) is compared exactly: the oracle runs on the boxes whose tags
meet it, whose records are exactly those of the whole set that meet it.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1901_10475_amd import catalog
from tests.gpu_util import (arrays_of, device_boxes_to_oracle, need_gpu, say,
                            slab_positions, window_index)

pytestmark = pytest.mark.gpu


def _check_window(arrays, records, ta, tb, label):
    ob = device_boxes_to_oracle(arrays, idx=window_index(arrays, ta, tb))
    want = oracle.pairs_bucketed(ob)
    got = oracle.records_in_window(records, ta, tb)
    say(f"  {label} [{ta}, {tb}): {len(ob)} boxes, {len(want)} oracle records")
    assert np.array_equal(got, want), (label, ta, tb, len(got), len(want))
    return len(want)


@pytest.mark.timeout(1200)
def test_tracked_hour_every_record():
    """16 848 objects, 1 h, dt = 1 s, FP64: the GPU's whole record list equals
    the bucketed oracle's (all pairs within each of the 3 600 slabs) on the
    GPU's boxes; every record names two boxes that overlap."""
    need_gpu()
    import paper_1901_10475_amd as cd
    sc = catalog.tracked_hour()
    n, dt, T = sc.n, sc.dt_ticks, sc.horizon_ticks
    say("tracked16848 1h every record")
    el = cd.soa(sc.elements)
    p = cd.params_struct(sc.tick_s, sc.mu, sc.threshold_km, T, dt)
    bp = cd.BroadPhase(sc.n, p)
    pairs = bp.run(el).cpu().numpy().view(np.uint32).copy()
    K = T // dt
    assert bp.count == n * K and len(pairs) > 0
    arr = arrays_of(bp.boxes)
    # every record: the boxes of i and j in slab t_lo / dt overlap, and the
    # record's interval is that slab's tag
    k = pairs[:, 2].astype(np.int64) // dt
    assert np.all(pairs[:, 2].astype(np.int64) == k * dt)
    assert np.all(pairs[:, 3] == np.where(k == K - 1, T + 1, (k + 1) * dt))
    pos = slab_positions(arr[4], n)    # object i's box in slab k, any slab order
    ia = pos[torch.from_numpy(k * n + pairs[:, 0].astype(np.int64)).cuda()]
    ib = pos[torch.from_numpy(k * n + pairs[:, 1].astype(np.int64)).cuda()]
    lo, hi = arr[0], arr[1]
    ok = torch.ones(len(pairs), dtype=torch.bool, device="cuda")
    for d in range(3):
        ok &= (lo[d][ia] <= hi[d][ib]) & (lo[d][ib] <= hi[d][ia])
    assert bool(ok.all())
    # the whole list, 300 slabs at a time (slabs never share a record)
    step = 300
    total = 0
    for s0 in range(0, K, step):
        s1 = min(K, s0 + step)
        ob = device_boxes_to_oracle(arr, lo_hi=(s0 * n, s1 * n))
        want = oracle.pairs_bucketed(ob)
        got = pairs[(pairs[:, 2] >= s0 * dt) & (pairs[:, 2] < s1 * dt)]
        assert np.array_equal(got, want), (s0, s1, len(got), len(want))
        total += len(want)
        say(f"  slabs [{s0}, {s1}): {len(want)} records equal")
    assert total == len(pairs)


@pytest.mark.timeout(900)
def test_tracked_hour_heuristic_steps_windows():
    """Per-object steps (5 km per interval), object-major boxes, device-wide
    sort: exact parity on four 45 s windows (5 % of the hour) with FP64 boxes
    and tree, and with FP32 outward-rounded boxes and tree; the FP64 list is
    contained in the FP32 one (extras counted)."""
    need_gpu()
    import paper_1901_10475_amd as cd
    sc = catalog.tracked_hour()
    T = sc.horizon_ticks
    el = cd.soa(sc.elements)
    p = cd.params_struct(sc.tick_s, sc.mu, sc.threshold_km, T, 0)
    wins = [(0, 45_000), (900_000, 945_000), (2_000_000, 2_045_000), (T - 45_000, T + 1)]
    lists = {}
    for prec in (cd.CD_FP64, cd.CD_FP32):
        say("tracked16848 1h heuristic steps, precision", prec)
        bp = cd.BroadPhase(sc.n, p, None, prec, prec, dt_heuristic_km=5.0, el_soa=el)
        pairs = bp.run(el).cpu().numpy().view(np.uint32).copy()
        assert bp.count > 79_000_000
        arr = arrays_of(bp.boxes)
        for ta, tb in wins:
            _check_window(arr, pairs, ta, tb, f"prec {prec}")
        lists[prec] = pairs
        del bp, arr
        torch.cuda.empty_cache()
    s64 = {tuple(x) for x in lists[cd.CD_FP64].tolist()}
    s32 = {tuple(x) for x in lists[cd.CD_FP32].tolist()}
    assert s64 <= s32
    say(f"  {len(s64)} FP64 records, {len(s32) - len(s64)} extra with FP32 boxes")


@pytest.mark.timeout(900)
def test_batch_scenarios_from_the_graph_replay():
    """Three scenarios of the 64-scenario batch (the smallest, a middle and the
    largest n; 30 min, dt = 1 s), captured into one graph and replayed twice:
    the replayed lists against the bucketed oracle on each scenario's boxes,
    the smallest in full, the others on three 5-slab windows."""
    need_gpu()
    from paper_1901_10475_amd.batch import BatchRunner
    sizes = catalog.batch_sizes()
    order = np.argsort(sizes)
    pick = [int(order[0]), int(order[len(order) // 2]), int(order[-1])]
    scs = [catalog.batch_member(s, sizes[s]) for s in pick]
    say("batch members", pick, [s.n for s in scs])
    br = BatchRunner(scs, shared_buffers=False)
    br.calibrate()
    br.capture()
    for rep in range(2):
        br.replay()
        res = [r.cpu().numpy().view(np.uint32).copy() for r in br.results()]
        for k, sc in enumerate(scs):
            arr = br.box_arrays(k)
            if k == 0:
                ob = device_boxes_to_oracle(arr)
                want = oracle.pairs_bucketed(ob)
                say(f"  replay {rep} scenario n={sc.n}: {len(want)} records, whole list")
                assert np.array_equal(res[k], want)
                continue
            for s in (0, 911, 1795):
                _check_window(arr, res[k], s * sc.dt_ticks, (s + 5) * sc.dt_ticks,
                              f"replay {rep} n={sc.n}")
    br.close()


@pytest.mark.timeout(900)
def test_debris_windows():
    """100 000 objects (fragment clouds included), 6 h as 30-minute windows,
    FP32 boxes and tree, speed-bound per-object steps: two windows, each
    checked on two 1-second sub-windows (one at the window's start, where the
    previous window's last instant is repeated, one inside)."""
    need_gpu()
    import paper_1901_10475_amd as cd
    sc = catalog.projected_debris()
    W = 1_800_000
    el = cd.soa(sc.elements)
    p = cd.params_struct(sc.tick_s, sc.mu, sc.threshold_km, W, 0)
    bp = cd.BroadPhase(sc.n, p, None, cd.CD_FP32, cd.CD_FP32, dt_heuristic_km=5.0, el_soa=el)
    for w in (0, 7):
        bp.params.start_ticks = w * W
        say("debris100000 window", w)
        pairs = bp.run(el).cpu().numpy().view(np.uint32).copy()
        assert len(pairs) > 0
        arr = arrays_of(bp.boxes)
        for ta in (0, 1_234_000):
            _check_window(arr, pairs, ta, ta + 1_000, f"window {w}")
