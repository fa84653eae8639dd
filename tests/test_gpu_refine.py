"""Bulk interval refinement on the GPU against the oracle's refinement and
Alg. Brute Force, on the records the GPU broad phase returns.

Both sides halve the same spans and drop a span when the two objects' boxes
over it do not meet; the boxes differ by rounding only (and, for the interval
rules, by how the 1e-10 rad widening reaches the bounds: the oracle carries it
through interval operations, the kernels pad by 1e-10 R), so a span may be
kept by one side and dropped by the other only where the two boxes touch to
within 1e-5 km.  Every other leaf must agree.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1901_10475_amd as cd
from paper_1901_10475_amd import catalog
from tests.gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu
MU = oracle.MU_EARTH


def _planted_leo(seed, n, planted, T, dt, start=0):
    rng = np.random.default_rng(seed)
    el = catalog.leo_mix(rng, n)
    pl = catalog.plant_conjunctions(rng, el, planted, T, dt, 1.0)
    for i, j, _ in pl:
        for o in (i, j):
            nm = np.sqrt(MU / el[o, 0] ** 3)
            el[o, 5] = (el[o, 5] - nm * start * 1e-3) % (2 * np.pi)
    return catalog.Scenario(f"leo{n}_planted", el, dt, T, 1.0, planted=pl)


def _gap(sc, i, j, a, b, start, rule):
    """Largest axis gap between the oracle's boxes of i and j over the instants
    a .. b - 1 (negative: they overlap)."""
    ta, tb = (start + a) * sc.tick_s, (start + b - 1) * sc.tick_s
    if rule == 0:
        out = []
        for o in (i, j):
            pa = oracle.position(sc.elements[o], ta)
            pb = oracle.position(sc.elements[o], tb)
            g = oracle.vmax(*sc.elements[o, :2]) * (tb - ta) / 2 + sc.threshold_km / 2
            out.append((np.minimum(pa, pb) - g, np.maximum(pa, pb) + g))
        (li, hi), (lj, hj) = out
    else:
        li, hi = oracle.box_interval(sc.elements[i], ta, tb, sc.threshold_km, rule)
        lj, hj = oracle.box_interval(sc.elements[j], ta, tb, sc.threshold_km, rule)
    return float(np.max(np.maximum(li - hj, lj - hi)))


def _run(sc, rule, start, heur=None):
    el = cd.soa(sc.elements)
    p = cd.params_struct(sc.tick_s, sc.mu, sc.threshold_km, sc.horizon_ticks,
                         sc.dt_ticks if heur is None else 0, start_ticks=start, box_rule=rule)
    bp = cd.BroadPhase(sc.n, p, dt_heuristic_km=heur, el_soa=el)
    pairs = bp.run(el).clone()
    return el, p, pairs


@pytest.mark.parametrize("rule", [0, 1, 2])
@pytest.mark.parametrize("min_steps,delta", [(1, 1), (16, 1), (1, 7), (4, 25)])
def test_refine_matches_oracle(rule, min_steps, delta):
    need_gpu()
    start = 5_000 if delta == 7 else 0
    sc = _planted_leo(81 + rule, 150, 6, 40_000, 4_000, start)
    say("refine rule", rule, "min_steps", min_steps, "delta", delta, "start", start)
    el, p, pairs = _run(sc, rule, start)
    got = cd.cd_refine_records(el, p, delta, pairs, min_steps=min_steps)
    torch.cuda.synchronize()
    got = got.cpu().numpy().view(np.uint32)
    rec = pairs.cpu().numpy().view(np.uint32)
    want = oracle.refine(sc.elements, rec, sc.horizon_ticks, sc.tick_s, sc.threshold_km, delta,
                         min_steps, rule=rule, start=start)
    say("records", len(rec), "leaves gpu", len(got), "oracle", len(want))
    assert len(want) > 0
    g = {tuple(x) for x in got.tolist()}
    w = {tuple(x) for x in want.tolist()}
    for i, j, a, b in g ^ w:
        assert abs(_gap(sc, i, j, a, b, start, rule)) <= 1e-5, (i, j, a, b)
    assert len(g ^ w) <= max(2, len(w) // 1000)
    # sorted and unique
    assert np.array_equal(got, np.unique(got, axis=0))


def test_single_instant_leaves_are_brute_force_witnesses():
    need_gpu()
    sc = _planted_leo(91, 120, 6, 20_000, 2_000)
    say("refine vs brute force")
    el, p, pairs = _run(sc, 0, 0)
    got = cd.cd_refine_records(el, p, 1, pairs).cpu().numpy().view(np.uint32)
    W = oracle.brute_force(sc.elements, sc.threshold_km / 2, sc.horizon_ticks, 1, sc.tick_s)
    want = {(int(i), int(j), int(t)) for t, i, j in W.tolist()}
    have = {(int(i), int(j), int(a)) for i, j, a, b in got.tolist()}
    assert len(want) > 0
    for i, j, t in have ^ want:
        pi = oracle.position(sc.elements[i], t * sc.tick_s)
        pj = oracle.position(sc.elements[j], t * sc.tick_s)
        assert abs(np.max(np.abs(pi - pj)) - sc.threshold_km) <= 1e-9


@pytest.mark.parametrize("heur", [None, 20.0])
def test_first_leaf_is_the_first_witness(heur):
    need_gpu()
    sc = _planted_leo(92, 160, 6, 40_000, 2_000)
    say("refine vs first witness", heur)
    el, p, pairs = _run(sc, 2, 0, heur=heur)
    leaves = cd.cd_refine_records(el, p, 1, pairs).cpu().numpy().view(np.uint32)
    wit, first = cd.cd_first_witness(el, p, 1, pairs)
    wit = wit.cpu().numpy().view(np.uint32)
    rec = pairs.cpu().numpy().view(np.uint32)
    for r, (i, j, lo, hi) in enumerate(rec.tolist()):
        ts = [a for a_i, a_j, a, b in leaves.tolist() if (a_i, a_j) == (i, j) and lo <= a < hi]
        if wit[r] != cd.CD_NO_WITNESS:
            # the refinement holds every witness; its first leaf may precede the
            # witness only by an instant within the widening of the threshold
            assert wit[r] in ts
            if min(ts) < wit[r]:
                pi = oracle.position(sc.elements[i], min(ts) * sc.tick_s)
                pj = oracle.position(sc.elements[j], min(ts) * sc.tick_s)
                assert np.max(np.abs(pi - pj)) <= sc.threshold_km + 1e-5
    fc = cd.first_collision(pairs, first)
    assert fc is not None
    assert (fc[1], fc[2], fc[0]) in {(int(i), int(j), int(a)) for i, j, a, b in leaves.tolist()}


def test_capacity_retry_and_whole_horizon_records():
    need_gpu()
    sc = _planted_leo(93, 60, 4, 30_000, 1_000)
    say("refine capacity retry")
    el = cd.soa(sc.elements)
    p = cd.params_struct(sc.tick_s, sc.mu, sc.threshold_km, sc.horizon_ticks, sc.dt_ticks)
    # caller-built records: every planted pair over the whole horizon
    rec = np.array([[i, j, 0, sc.horizon_ticks + 1] for i, j, _ in sc.planted], np.uint32)
    pairs = torch.from_numpy(rec.view(np.int32)).cuda()
    big = cd.cd_refine_records(el, p, 1, pairs, capacity=1 << 20).cpu().numpy()
    small = cd.cd_refine_records(el, p, 1, pairs, capacity=1).cpu().numpy()
    assert np.array_equal(big, small) and len(big) > 0
    want = oracle.refine(sc.elements, rec, sc.horizon_ticks, sc.tick_s, sc.threshold_km, 1, 1)
    g = {tuple(x) for x in big.view(np.uint32).tolist()}
    w = {tuple(x) for x in want.tolist()}
    for i, j, a, b in g ^ w:
        assert abs(_gap(sc, i, j, a, b, 0, 0)) <= 1e-5
    for i, j, tc in sc.planted:
        assert any((x[0], x[1], x[2]) == (i, j, tc) for x in g)


def test_empty_records():
    need_gpu()
    sc = _planted_leo(94, 20, 0, 1000, 1000)
    el = cd.soa(sc.elements)
    p = cd.params_struct(sc.tick_s, sc.mu, sc.threshold_km, sc.horizon_ticks, sc.dt_ticks)
    none = torch.empty((0, 4), dtype=torch.int32, device="cuda")
    assert cd.cd_refine_records(el, p, 1, none).shape[0] == 0
    with pytest.raises(cd.CDError):
        cd.cd_refine_records(el, p, 0, none)
