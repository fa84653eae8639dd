"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Boxes: within 1e-9 relative of the oracle's FP64 boxes; tags, object ids and
counts exact.  Pairs: the canonical record list equals, record for record, the
oracle's literal all-pairs result on the same (GPU-built) boxes.
"""
import numpy as np
import pytest

import oracle
from paper_1901_10475_amd import catalog
from tests.gpu_util import (assert_boxes_close, gpu_to_object_major, need_gpu,
                            records_of_boxes, run_catalog, say, slab_positions)

pytestmark = pytest.mark.gpu


def _oracle_boxes(sc, dt=None):
    return oracle.boxes(sc.elements, sc.dt_ticks if dt is None else dt, sc.horizon_ticks,
                        sc.tick_s, sc.threshold_km)


@pytest.mark.parametrize("n,T,dt", [(200, 60_000, 10_000), (257, 25_000, 10_000),
                                    (64, 0, 1_000), (65, 7_000, 9_000), (1, 50_000, 1_000)])
def test_boxes_uniform_step(n, T, dt):
    need_gpu()
    say("boxes uniform", n, T, dt)
    sc = catalog.scaled(catalog.tracked_hour(seed=11, planted=0), n=n, horizon_ticks=T,
                        dt_ticks=dt)
    bp, _ = run_catalog(sc)
    lo, hi, t0, t1, obj = bp.boxes.to_host()
    ob = _oracle_boxes(sc)
    K = oracle.intervals(dt, T)
    assert bp.count == len(ob) == n * K
    g = gpu_to_object_major(obj, n, K)
    assert np.array_equal(t0[g], ob.t0) and np.array_equal(t1[g], ob.t1)
    assert np.array_equal(obj[g], ob.obj)
    assert_boxes_close(lo[g], hi[g], ob.lo, ob.hi, sc.elements[ob.obj, 0])


def test_boxes_per_object_step():
    need_gpu()
    say("boxes per-object dt")
    sc = catalog.scaled(catalog.tracked_hour(seed=12, planted=0), n=300, horizon_ticks=40_000)
    dt = oracle.dt_heuristic(sc.elements, sc.tick_s, 5.0, sc.horizon_ticks)
    bp, _ = run_catalog(sc, dt_array=dt)
    lo, hi, t0, t1, obj = bp.boxes.to_host()
    ob = _oracle_boxes(sc, dt)
    assert bp.count == len(ob)
    assert np.array_equal(t0, ob.t0) and np.array_equal(t1, ob.t1)
    assert np.array_equal(obj, ob.obj)
    assert_boxes_close(lo, hi, ob.lo, ob.hi, sc.elements[ob.obj, 0])


def test_dt_heuristic_bit_exact():
    need_gpu()
    say("dt heuristic")
    import torch
    import paper_1901_10475_amd as cd
    sc = catalog.tracked_hour(seed=13, planted=0)
    el = cd.soa(sc.elements)
    out = torch.zeros(sc.n, dtype=torch.int32, device="cuda")
    p = cd.params_struct(sc.tick_s, sc.mu, sc.threshold_km, sc.horizon_ticks, 0)
    cd.cd_dt_heuristic(el, p, 5.0, out)
    got = out.cpu().numpy().view(np.uint32)
    want = oracle.dt_heuristic(sc.elements, sc.tick_s, 5.0, sc.horizon_ticks)
    assert np.array_equal(got, want)


def test_pairs_small_leo_full_parity():
    """1000 LEO objects, 10 min, dt = 10 s (60 000 boxes): literal oracle."""
    need_gpu()
    say("pairs leo1000 600s dt10s fp64")
    sc = catalog.small_leo()
    bp, pairs = run_catalog(sc)
    lo, hi, t0, t1, obj = bp.boxes.to_host()
    ref = oracle.pairs(oracle.Boxes(lo, hi, t0, t1, obj))
    assert len(ref) > 0
    assert np.array_equal(pairs, ref)
    # planted conjunctions are among the records, at their planted times
    for i, j, tc in sc.planted:
        hit = pairs[(pairs[:, 0] == i) & (pairs[:, 1] == j)]
        assert np.any((hit[:, 2] <= tc) & (tc < hit[:, 3])), (i, j, tc)


def test_pairs_fp32_tree_superset():
    """FP32 outward-rounded tree: exact parity with the oracle on the rounded
    boxes, and every FP64 record is still reported."""
    need_gpu()
    say("pairs leo1000 fp32 tree")
    sc = catalog.small_leo()
    bp64, p64 = run_catalog(sc)
    bp32, p32 = run_catalog(sc, box_precision=0, tree_precision=1)
    lo, hi, t0, t1, obj = bp32.boxes.to_host()
    r = oracle.outward_f32(oracle.Boxes(lo, hi, t0, t1, obj))
    ref = oracle.pairs(r)
    assert np.array_equal(p32, ref)
    s64 = {tuple(x) for x in p64.tolist()}
    s32 = {tuple(x) for x in p32.tolist()}
    assert s64 <= s32


def test_fp32_boxes_are_outward_rounded():
    need_gpu()
    say("fp32 boxes")
    sc = catalog.scaled(catalog.small_leo(), n=300, horizon_ticks=100_000)
    bp64, p64 = run_catalog(sc)
    bp32, p32 = run_catalog(sc, box_precision=1, tree_precision=1)
    lo, hi, t0, t1, obj = bp64.boxes.to_host()
    l32, h32, u0, u1, uo = bp32.boxes.to_host()
    r = oracle.outward_f32(oracle.Boxes(lo, hi, t0, t1, obj))
    assert np.array_equal(l32, r.lo) and np.array_equal(h32, r.hi)
    assert np.all(l32 <= lo) and np.all(h32 >= hi)
    assert np.array_equal(p32, oracle.pairs(r))
    assert {tuple(x) for x in p64.tolist()} <= {tuple(x) for x in p32.tolist()}


@pytest.mark.parametrize("kind", ["uniform", "identical", "disjoint", "line", "huge"])
@pytest.mark.parametrize("N", [0, 1, 2, 3, 63, 64, 65, 1000, 1024, 1025, 2048, 4095, 4097,
                               20000])
def test_box_soups_general_path(kind, N):
    """Caller-built boxes (device-wide sort path), ragged sizes (the bottom-up
    pass's 1 024-leaf chunks: one exactly full, one leaf over, two full),
    degenerate geometry; FP64 and FP32 trees.  Identical boxes overlap in space
    everywhere (20 000 of them: 6-7 M records, only the time tags separate
    them), so the node-pair queue overflows into the per-leaf walk and the
    records into the radix canonical path."""
    need_gpu()
    say("soup", kind, N)
    import paper_1901_10475_amd as cd
    lo, hi, t0, t1, obj = catalog.random_boxes(N + 101, N, max(2, N // 4), extent=200, size=6,
                                               T=400, max_len=12, kind=kind)
    ob = oracle.Boxes(lo, hi, t0, t1, obj)
    ref = oracle.pairs(ob)
    for tp in (cd.CD_FP64, cd.CD_FP32):
        b = cd.Boxes.from_arrays(lo, hi, t0, t1, obj, cd.CD_FP64, horizon_ticks=400,
                                 obj_count=max(2, N // 4))
        got = cd.query_boxes(b, tp, slab_ticks=16, capacity=64).cpu().numpy().view(np.uint32)
        want = ref if tp == cd.CD_FP64 else oracle.pairs(oracle.outward_f32(ob))
        assert np.array_equal(got, want), (kind, N, tp)


@pytest.mark.parametrize("kind", ["uniform", "identical", "line"])
@pytest.mark.parametrize("N", [65, 4097])
def test_box_soups_wide_keys(kind, N):
    """Wide keys: time tags scaled by 2^20 (half-open overlaps, hence records
    up to the same scale, are unchanged) over one-tick slabs need 29 slab
    bits, so slab, 30-bit code and box index no longer fit one 64-bit word:
    65 boxes keep the code's top 28 bits in 8-byte items, 4 097 boxes would
    keep fewer than 24 and sort 16-byte (key, index) items.  FP64 and FP32
    trees against the oracle."""
    need_gpu()
    say("soup wide keys", kind, N)
    import paper_1901_10475_amd as cd
    lo, hi, t0, t1, obj = catalog.random_boxes(N + 7, N, max(2, N // 4), extent=200, size=6,
                                               T=400, max_len=12, kind=kind)
    scale = 1 << 20
    t0, t1 = t0.astype(np.int64) * scale, t1.astype(np.int64) * scale
    assert t1.max() < 2 ** 32 - 1
    t0, t1 = t0.astype(np.uint32), t1.astype(np.uint32)
    H = 400 * scale
    assert (H // 1).bit_length() + 30 + (N - 1).bit_length() > 64
    ob = oracle.Boxes(lo, hi, t0, t1, obj)
    for tp in (cd.CD_FP64, cd.CD_FP32):
        b = cd.Boxes.from_arrays(lo, hi, t0, t1, obj, cd.CD_FP64, horizon_ticks=H,
                                 obj_count=max(2, N // 4))
        got = cd.query_boxes(b, tp, slab_ticks=1, capacity=64).cpu().numpy().view(np.uint32)
        want = oracle.pairs(ob if tp == cd.CD_FP64 else oracle.outward_f32(ob))
        assert np.array_equal(got, want), (kind, N, tp)


def test_early_canonical_list_across_path_changes():
    """A synchronising query forms the canonical list before the host reads
    the count when the calling thread's previous query took the same path
    (one workgroup up to 4 096 records, tiles and merges above); the guess is
    checked on the device.  Queries alternating between the two paths, each
    twice in a row (first with the other path's guess, then with its own):
    every list equals the oracle's."""
    need_gpu()
    import paper_1901_10475_amd as cd
    cases = {}
    for N in (450, 800):   # identical boxes: records set by the time tags alone
        lo, hi, t0, t1, obj = catalog.random_boxes(N + 3, N, N // 4, extent=200, size=6, T=400,
                                                   max_len=12, kind="identical")
        want = oracle.pairs(oracle.Boxes(lo, hi, t0, t1, obj))
        b = cd.Boxes.from_arrays(lo, hi, t0, t1, obj, cd.CD_FP64, horizon_ticks=400,
                                 obj_count=N // 4)
        cases[N] = (b, want)
    assert len(cases[450][1]) <= 4096 < len(cases[800][1]) <= 1 << 18
    for N in (450, 800, 450, 800, 800, 450):
        b, want = cases[N]
        for rep in range(2):
            got = cd.query_boxes(b, cd.CD_FP64, slab_ticks=16,
                                 capacity=2 * len(want)).cpu().numpy().view(np.uint32)
            assert np.array_equal(got, want), (N, rep)


def test_capacity_retry_gives_identical_set():
    need_gpu()
    say("capacity retry")
    import paper_1901_10475_amd as cd
    lo, hi, t0, t1, obj = catalog.random_boxes(5, 3000, 300, extent=60, size=8, T=50)
    b = cd.Boxes.from_arrays(lo, hi, t0, t1, obj, cd.CD_FP64, horizon_ticks=60, obj_count=300)
    tree = cd.Tree(b.count, cd.CD_FP64)
    ws = cd._bytes(cd.lib().cd_build_tree_ws(b.count), "cuda")
    cd.cd_build_tree(b, cd.CD_FP64, tree, ws, 4)
    import torch
    out = torch.empty((8, 4), dtype=torch.int32, device="cuda")
    wsq = cd._bytes(cd.lib().cd_query_pairs_ws(b.count, 8), "cuda")
    rc, need = cd.cd_query_pairs(tree, out, 8, wsq)
    assert rc == cd.CD_E_CAPACITY and need > 8
    out = torch.empty((need, 4), dtype=torch.int32, device="cuda")
    wsq = cd._bytes(cd.lib().cd_query_pairs_ws(b.count, need), "cuda")
    rc, cnt = cd.cd_query_pairs(tree, out, need, wsq)
    assert rc == cd.CD_OK
    ref = oracle.pairs(oracle.Boxes(lo, hi, t0, t1, obj))
    assert np.array_equal(out[:cnt].cpu().numpy().view(np.uint32), ref)


def test_hand_cases_on_gpu():
    """Identical elements (every interval, last closed at T); n = 0, 1; T = 0."""
    need_gpu()
    say("hand cases")
    el = np.array([[6800.0, 0.001, 0.9, 0.2, 0.3, 0.4]] * 2)
    sc = catalog.Scenario("dup", el, 10_000, 25_000, 1.0)
    _, pairs = run_catalog(sc)
    assert pairs.tolist() == [[0, 1, 0, 10000], [0, 1, 10000, 20000], [0, 1, 20000, 25001]]
    sc = catalog.Scenario("one", el[:1], 1_000, 10_000, 1.0)
    _, pairs = run_catalog(sc)
    assert len(pairs) == 0
    sc = catalog.Scenario("instant", el, 1_000, 0, 1.0)
    _, pairs = run_catalog(sc)
    assert pairs.tolist() == [[0, 1, 0, 1]]


def test_invalid_elements_reported():
    need_gpu()
    say("invalid elements")
    import paper_1901_10475_amd as cd
    el = catalog.small_leo(planted=0).elements[:50].copy()
    el[17, 1] = 1.5
    with pytest.raises(cd.CDError) as ei:
        cd.cd_validate_elements(cd.soa(el))
    assert ei.value.status == cd.CD_E_INVALID and "17" in str(ei.value)
    el[17, 1] = 0.01
    cd.cd_validate_elements(cd.soa(el))


def test_per_object_step_pairs_parity():
    """Variable steps on a cut of the tracked catalog (object-major boxes,
    device-wide key sort): exact parity with the literal oracle."""
    need_gpu()
    say("pairs per-object dt cut")
    sc = catalog.scaled(catalog.tracked_hour(seed=14, planted=8), n=2000, horizon_ticks=30_000)
    dt = oracle.dt_heuristic(sc.elements, sc.tick_s, 5.0, sc.horizon_ticks)
    bp, pairs = run_catalog(sc, dt_array=dt)
    lo, hi, t0, t1, obj = bp.boxes.to_host()
    ref = oracle.pairs(oracle.Boxes(lo, hi, t0, t1, obj))
    assert np.array_equal(pairs, ref)


@pytest.mark.parametrize("rule", [0, 2])
def test_tracked_hour_full_size_sampled(rule):
    """The benchmark workload (16 848 objects, 1 h, dt = 1 s, 60.65 M boxes, FP64),
    with the speed-bound box (0) and the eccentric-anomaly interval box (2):
    sampled exact parity, exact parity on a time window, planted recall."""
    need_gpu()
    say("tracked16848 1h full size, box rule", rule)
    sc = catalog.tracked_hour()
    bp, pairs = run_catalog(sc, box_rule=rule)
    N = bp.count
    assert N == 16848 * 3600
    lo, hi, t0, t1, obj = bp.boxes.to_host()
    ob = oracle.Boxes(lo, hi, t0, t1, obj)
    rng = np.random.default_rng(99)
    sample = rng.choice(N, 192, replace=False)
    # include boxes that do have partners, so the sample is not all-empty
    if len(pairs):
        pick = pairs[rng.choice(len(pairs), min(64, len(pairs)), replace=False)]
        pos = slab_positions(obj, 16848)
        extra = [pos[(int(t) // 1000) * 16848 + int(i)] for i, _, t, _ in pick]
        sample = np.unique(np.concatenate([sample, extra]))
    want = oracle.pairs_of(ob, sample)
    got = records_of_boxes(pairs, obj, t0, t1, sample)
    got = np.unique(got, axis=0) if len(got) else got.reshape(0, 4)
    assert np.array_equal(got, want)
    # exact parity on the first 3 slabs (time window [0, 3 s))
    w = 3 * 16848
    ref_w = oracle.pairs(ob.take(np.arange(w)))
    got_w = pairs[pairs[:, 2] < 3000]
    assert np.array_equal(got_w, ref_w)
    # planted conjunctions found at their times
    for i, j, tc in sc.planted:
        hit = pairs[(pairs[:, 0] == i) & (pairs[:, 1] == j)]
        assert np.any((hit[:, 2] <= tc) & (tc < hit[:, 3])), (i, j, tc)
    # box bounds of sampled boxes against the oracle's own construction
    ob_i = np.unique(obj[sample])[:16]
    sub = oracle.boxes(sc.elements[ob_i], 1000, sc.horizon_ticks, sc.tick_s, 1.0, rule=rule)
    pos = slab_positions(obj, 16848)
    g = np.concatenate([pos[np.arange(3600) * 16848 + i] for i in ob_i])
    assert_boxes_close(lo[g], hi[g], sub.lo, sub.hi, sc.elements[obj[g], 0])


def test_tracked_hour_heuristic_steps_full_size():
    """Per-object steps (each box's motion bounded by 5 km; 79.7 M boxes,
    object-major, device-wide sort path): sampled exact parity, planted
    recall, and the FP32 tree's list contains the FP64 list (extras counted)."""
    need_gpu()
    say("tracked16848 1h heuristic dt full size")
    import torch
    import paper_1901_10475_amd as cd
    sc = catalog.tracked_hour()
    el = cd.soa(sc.elements)
    p = cd.params_struct(sc.tick_s, sc.mu, sc.threshold_km, sc.horizon_ticks, 0)
    bp = cd.BroadPhase(sc.n, p, None, cd.CD_FP64, cd.CD_FP64, dt_heuristic_km=5.0, el_soa=el)
    pairs = bp.run(el).cpu().numpy().view(np.uint32).copy()
    dt = bp.dt.cpu().numpy().view(np.uint32)
    assert np.array_equal(dt, oracle.dt_heuristic(sc.elements, sc.tick_s, 5.0, sc.horizon_ticks))
    lo, hi, t0, t1, obj = bp.boxes.to_host()
    ob = oracle.Boxes(lo, hi, t0, t1, obj)
    rng = np.random.default_rng(7)
    sample = rng.choice(len(t0), 160, replace=False)
    if len(pairs):
        # boxes that have partners: object i's box containing t_lo
        K = -(-sc.horizon_ticks // dt.astype(np.int64))
        off = np.concatenate([[0], np.cumsum(K)[:-1]])
        pick = pairs[rng.choice(len(pairs), min(48, len(pairs)), replace=False)]
        extra = [off[i] + int(t) // int(dt[i]) for i, _, t, _ in pick]
        sample = np.unique(np.concatenate([sample, extra]))
    want = oracle.pairs_of(ob, sample)
    got = records_of_boxes(pairs, obj, t0, t1, sample)
    got = np.unique(got, axis=0) if len(got) else got.reshape(0, 4)
    assert np.array_equal(got, want)
    for i, j, tc in sc.planted:
        hit = pairs[(pairs[:, 0] == i) & (pairs[:, 1] == j)]
        assert np.any((hit[:, 2] <= tc) & (tc < hit[:, 3])), (i, j, tc)
    del bp
    torch.cuda.empty_cache()
    bp32 = cd.BroadPhase(sc.n, p, None, cd.CD_FP64, cd.CD_FP32, dt_heuristic_km=5.0, el_soa=el)
    p32 = bp32.run(el).cpu().numpy().view(np.uint32)
    s64 = {tuple(x) for x in pairs.tolist()}
    s32 = {tuple(x) for x in p32.tolist()}
    assert s64 <= s32
    say(f"heuristic dt: {len(s64)} FP64 records, {len(s32) - len(s64)} extra with an FP32 tree")


@pytest.mark.parametrize("start", [10_000, 1_234_567])
def test_window_boxes_and_pairs(start):
    """A horizon placed at absolute ticks [start, start + T]: boxes match the
    oracle's window boxes, records match the oracle on the same boxes."""
    need_gpu()
    say("window start", start)
    import torch
    import paper_1901_10475_amd as cd
    sc = catalog.scaled(catalog.small_leo(), n=600, horizon_ticks=60_000)
    el = cd.soa(sc.elements)
    for dt in (None, oracle.dt_heuristic(sc.elements, sc.tick_s, 5.0, sc.horizon_ticks)):
        p = cd.params_struct(sc.tick_s, sc.mu, sc.threshold_km, sc.horizon_ticks,
                             sc.dt_ticks if dt is None else 0, start_ticks=start)
        dtt = None if dt is None else torch.from_numpy(dt.view(np.int32)).cuda()
        bp = cd.BroadPhase(sc.n, p, dtt)
        pairs = bp.run(el).cpu().numpy().view(np.uint32)
        lo, hi, t0, t1, obj = bp.boxes.to_host()
        ob = oracle.boxes(sc.elements, sc.dt_ticks if dt is None else dt, sc.horizon_ticks,
                          sc.tick_s, sc.threshold_km, start=start)
        if dt is None:
            g = gpu_to_object_major(obj, sc.n, oracle.intervals(sc.dt_ticks, sc.horizon_ticks))
            lo, hi, t0, t1, obj = lo[g], hi[g], t0[g], t1[g], obj[g]
        assert np.array_equal(t0, ob.t0) and np.array_equal(t1, ob.t1)
        assert np.array_equal(obj, ob.obj)
        assert_boxes_close(lo, hi, ob.lo, ob.hi, sc.elements[ob.obj, 0])
        ref = oracle.pairs(oracle.Boxes(*bp.boxes.to_host()))
        assert np.array_equal(pairs, ref)


@pytest.mark.parametrize("heur", [None, 5.0])
def test_box_codes_change_tree_shape_not_records(heur):
    """Morton codes written with the boxes (orbit-frame) versus codes formed by
    the tree builder from the boxes: the same record list."""
    need_gpu()
    say("codes", heur)
    import torch
    import paper_1901_10475_amd as cd
    sc = catalog.scaled(catalog.tracked_hour(seed=14), n=4000, horizon_ticks=90_000)
    el = cd.soa(sc.elements)
    p = cd.params_struct(sc.tick_s, sc.mu, sc.threshold_km, sc.horizon_ticks,
                         sc.dt_ticks if heur is None else 0)
    out = []
    for codes in (True, False):
        for tp in (cd.CD_FP64, cd.CD_FP32):
            # boxes as arrays here, so that their codes can be read afterwards
            bp = cd.BroadPhase(sc.n, p, None, cd.CD_FP64, tp, codes=codes,
                               dt_heuristic_km=heur, el_soa=el, in_tree=False)
            out.append((codes, tp, bp.run(el).cpu().numpy().copy()))
            if codes:
                c = bp.boxes.code[:bp.count].cpu().numpy().view(np.uint32)
                assert bp.boxes.desc.code_valid == 1
                assert c.max() < (1 << 30) and len(np.unique(c)) > bp.count // 10
    by = {(c, tp): r for c, tp, r in out}
    assert np.array_equal(by[(True, cd.CD_FP64)], by[(False, cd.CD_FP64)])
    assert np.array_equal(by[(True, cd.CD_FP32)], by[(False, cd.CD_FP32)])
    assert len(by[(True, cd.CD_FP64)]) > 0
    # FP64 boxes written as the tree's own leaf records (uniform step only)
    bp = cd.BroadPhase(sc.n, p, None, cd.CD_FP64, cd.CD_FP64, dt_heuristic_km=heur, el_soa=el)
    assert bp.in_tree == (heur is None)
    assert np.array_equal(bp.run(el).cpu().numpy(), by[(True, cd.CD_FP64)])
