"""The graph-capturable query, graph replay of a batch, and the autotuner.

The device-count query must give, record for record, the list of the
synchronising query on the same tree (bit-exact: both are canonical lists),
in every traversal mode (one launch per node-pair level, every level in one
launch, the per-leaf walk) and with the per-leaf walk forced as fallback.  A
captured batch is replayed several times, with eager work and
synchronisation between replays and a changed input before the last one;
every replay is checked against eager runs.
"""
import json

import numpy as np
import pytest
import torch

import paper_1901_10475_amd as cd
from paper_1901_10475_amd import autotune, catalog
from paper_1901_10475_amd.batch import BatchRunner
from tests.gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu


def _async(bp, capacity, tuning=None):
    cd.cd_set_tuning(tuning)
    try:
        out = torch.empty((capacity, 4), dtype=torch.int32, device="cuda")
        ws = cd._bytes(cd.lib().cd_query_pairs_ws(bp.count, capacity), "cuda")
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        cd.cd_query_pairs_async(bp.tree, out, capacity, cnt, st, ws)
        torch.cuda.synchronize()
        c, s = int(cnt.item()), int(st.item())
        return out[:c].cpu().numpy() if s == 0 else None, c, s
    finally:
        cd.cd_set_tuning(None)


def _cases():
    leo = catalog.small_leo()
    hour = catalog.scaled(catalog.tracked_hour(), n=3000, horizon_ticks=120_000)
    debris = catalog.projected_debris(seed=91, n=4000, parents=2, horizon_ticks=120_000,
                                      planted=4)
    return [("leo1000", leo, None), ("tracked3000_120s", hour, None),
            ("debris4000_heur", debris, 5.0)]


@pytest.mark.parametrize("name,sc,heur", _cases(), ids=[c[0] for c in _cases()])
def test_async_query_equals_eager(name, sc, heur):
    need_gpu()
    say("async query", name)
    el = cd.soa(sc.elements)
    p = cd.params_struct(sc.tick_s, sc.mu, sc.threshold_km, sc.horizon_ticks,
                         sc.dt_ticks if heur is None else 0)
    bp = cd.BroadPhase(sc.n, p, dt_heuristic_km=heur, el_soa=el)
    ref = bp.run(el).cpu().numpy()
    P = len(ref)
    say("  records", P)
    assert P > 0
    for tun in (None, {"mode": 1}, {"mode": 1, "walk_threads": 64}, {"max_levels": 1},
                {"expand_blocks": 64, "expand_threads": 64},
                {"expand_blocks": 256, "expand_threads": 512},
                {"expand_blocks": 64, "expand_threads": 1024},
                {"mode": 2}, {"mode": 2, "expand_blocks": 64}, {"mode": 2, "expand_blocks": 4096}):
        for cap in (P, P + 1, 2 * P + 17):
            got, c, s = _async(bp, cap, tun)
            assert s == 0 and c == P, (tun, cap, c, s)
            assert np.array_equal(got, ref), (tun, cap)
    # too small: status bit 1 and at least the needed count
    if P >= 2:
        got, c, s = _async(bp, P - 1)
        assert s == 1 and c >= P


@pytest.mark.parametrize("name,sc,heur", _cases(), ids=[c[0] for c in _cases()])
def test_one_launch_traversal_equals_levels(name, sc, heur):
    """Every node-pair level in one launch of a resident grid (mode 2), in the
    synchronising query: the same canonical list as one launch per level."""
    need_gpu()
    say("one-launch traversal", name)
    el = cd.soa(sc.elements)
    p = cd.params_struct(sc.tick_s, sc.mu, sc.threshold_km, sc.horizon_ticks,
                         sc.dt_ticks if heur is None else 0)
    bp = cd.BroadPhase(sc.n, p, dt_heuristic_km=heur, el_soa=el)
    ref = bp.run(el).cpu().numpy()
    assert len(ref) > 0
    try:
        for tun in ({"mode": 2}, {"mode": 2, "expand_blocks": 64}, {"mode": 2, "expand_blocks": 4096}):
            cd.cd_set_tuning(tun)
            for rep in range(2):
                got = bp.run(el).cpu().numpy()
                assert np.array_equal(got, ref), (tun, rep)
    finally:
        cd.cd_set_tuning(None)


def test_last_query_levels_bound_the_async_levels():
    """cd_last_query_levels after a synchronising query is the number of
    node-pair levels the device-count query needs on that tree: with that
    many it never falls back to the per-leaf walk, with one fewer it does
    (counted by the counters build); the records are the same either way."""
    need_gpu()
    sc = catalog.scaled(catalog.tracked_hour(), n=3000, horizon_ticks=120_000)
    el = cd.soa(sc.elements)
    p = cd.params_struct(sc.tick_s, sc.mu, sc.threshold_km, sc.horizon_ticks, sc.dt_ticks)
    bp = cd.BroadPhase(sc.n, p)
    ref = bp.run(el).cpu().numpy()
    P = len(ref)
    with cd.counters_build():
        bp.query()
        lv = cd.cd_last_query_levels()
        say("levels", lv, "records", P)
        assert 1 < lv <= 400
        for levels, walks in ((lv, False), (lv + 3, False), (lv - 1, True)):
            cd.cd_counters_reset(None)
            got, c, s = _async(bp, P, {"max_levels": levels})
            cnt = cd.cd_counters_read()
            assert s == 0 and np.array_equal(got, ref), levels
            assert (cnt["walk_steps"] > 0) == walks, (levels, cnt)


def test_async_query_single_and_empty_trees():
    need_gpu()
    lo = np.zeros((1, 3))
    b = cd.Boxes.from_arrays(lo, lo + 1.0, [0], [1], [0], horizon_ticks=1, obj_count=1)
    tree = cd.Tree(1, cd.CD_FP64)
    ws = cd._bytes(cd.lib().cd_build_tree_ws(1), "cuda")
    cd.cd_build_tree(b, cd.CD_FP64, tree, ws)
    out = torch.empty((4, 4), dtype=torch.int32, device="cuda")
    wq = cd._bytes(cd.lib().cd_query_pairs_ws(1, 4), "cuda")
    cnt = torch.full((1,), 7, dtype=torch.int64, device="cuda")
    st = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    cd.cd_query_pairs_async(tree, out, 4, cnt, st, wq)
    torch.cuda.synchronize()
    assert cnt.item() == 0 and st.item() == 0


def _batch_scenarios():
    sizes = [2000, 2600, 3400, 2100, 5200, 2900]
    out = []
    for s, n in enumerate(sizes):
        sc = catalog.batch_member(s, n)
        out.append(catalog.scaled(sc, horizon_ticks=30_000))
    return out


def test_graph_replays_match_eager_runs():
    need_gpu()
    scs = _batch_scenarios()
    say("batch", [s.n for s in scs])
    br = BatchRunner(scs, min_capacity=1024)
    br.calibrate()
    with torch.cuda.stream(br.stream):
        eager = [br.run_eager(k).cpu().numpy() for k in range(len(scs))]
    br.stream.synchronize()
    assert sum(len(e) for e in eager) > 0
    br.capture()
    for rep in range(3):
        br.replay()
        res = br.results()
        for k, r in enumerate(res):
            assert np.array_equal(r.cpu().numpy(), eager[k]), (rep, k)
        # eager work and synchronisation between replays
        with torch.cuda.stream(br.stream):
            x = br.run_eager(rep % len(scs))
        br.stream.synchronize()
        assert np.array_equal(x.cpu().numpy(), eager[rep % len(scs)])
        torch.cuda.synchronize()
    # a replay rereads its inputs: new elements for scenario 0
    new = catalog.batch_member(40, scs[0].n)
    new = catalog.scaled(new, horizon_ticks=30_000)
    br.el[0].copy_(cd.soa(new.elements))
    torch.cuda.synchronize()
    br.replay()
    res = br.results()
    with torch.cuda.stream(br.stream):
        fresh = br.run_eager(0).cpu().numpy()
    br.stream.synchronize()
    assert np.array_equal(res[0].cpu().numpy(), fresh)
    for k in range(1, len(scs)):
        assert np.array_equal(res[k].cpu().numpy(), eager[k])
    br.close()


def test_graph_replay_recovers_from_exceeded_capacity():
    need_gpu()
    deb = catalog.projected_debris(seed=92, n=3000, parents=2, horizon_ticks=30_000, planted=0)
    dense = catalog.Scenario("debris3000_30s_dt1s", deb.elements, 1_000, 30_000, 1.0)
    scs = [_batch_scenarios()[0], dense, _batch_scenarios()[2]]
    br = BatchRunner(scs, min_capacity=1)
    br.calibrate()
    with torch.cuda.stream(br.stream):
        eager = [br.run_eager(k).cpu().numpy() for k in range(len(scs))]
    br.stream.synchronize()
    say("records", [len(e) for e in eager])
    assert len(eager[1]) >= 2
    br.capacity[1] = len(eager[1]) // 2    # too small on purpose
    br._alloc_outputs()
    br.capture()
    br.replay()
    res = br.results()      # scenario 1 is rerun eagerly
    for k in range(len(scs)):
        assert np.array_equal(res[k].cpu().numpy(), eager[k])
    assert br.capacity[1] > len(eager[1])
    br.close()


def test_autotuner_searches_checks_and_caches(tmp_path):
    need_gpu()
    sc = catalog.scaled(catalog.tracked_hour(), n=3000, horizon_ticks=60_000)
    el = cd.soa(sc.elements)
    p = cd.params_struct(sc.tick_s, sc.mu, sc.threshold_km, sc.horizon_ticks, sc.dt_ticks)
    bp = cd.BroadPhase(sc.n, p)
    bp.build(el)
    path = str(tmp_path / "tune.json")
    best, hit = autotune.tuned(bp.query, cd.CD_FP64, bp.count, "fixed", path=path, reps=2)
    assert not hit and best in autotune.candidates()
    cache = json.load(open(path))
    key = autotune.cache_key(cd.CD_FP64, bp.count, "fixed")
    assert cache[key]["tuning"] == best and len(cache[key]["ms"]) == len(autotune.candidates())
    again, hit = autotune.tuned(bp.query, cd.CD_FP64, bp.count, "fixed", path=path)
    assert hit and again == best
    say("autotuned", best)


def test_slab_tuner_keeps_the_record_list(tmp_path):
    need_gpu()
    sc = catalog.projected_debris(seed=93, n=3000, parents=2, horizon_ticks=120_000, planted=4)
    el = cd.soa(sc.elements)
    p = cd.params_struct(sc.tick_s, sc.mu, sc.threshold_km, sc.horizon_ticks, 0)
    bp = cd.BroadPhase(sc.n, p, dt_heuristic_km=5.0, el_soa=el)

    def run(w):
        bp.slab_ticks = w
        return bp.run(el)

    path = str(tmp_path / "tune.json")
    best, hit = autotune.tuned_slab(run, sc.horizon_ticks, cd.CD_FP64, bp.count, "heuristic",
                                    path=path, reps=2)
    assert not hit and best in autotune.slab_candidates(sc.horizon_ticks)
    again, hit = autotune.tuned_slab(run, sc.horizon_ticks, cd.CD_FP64, bp.count, "heuristic",
                                     path=path)
    assert hit and again == best
    say("slab tuned", best)
