"""Pins of the oracle's bulk interval refinement (the halving of Procedure
resolveCollisions applied to every candidate record at once).

Independent reference: Alg. Brute Force (every pair at every grid instant).
With the speed box and single-instant leaves the refinement must return
exactly the brute-force witnesses inside the records (a box over one instant
is the occupancy cube, Property 1); with the interval boxes the leaves hold
every witness and add only instants within their 1e-10 rad widening of the
threshold; with coarser leaves every witness lies in a leaf, every leaf in its
record.
"""
import numpy as np
import pytest

import oracle
from paper_1901_10475_amd import catalog


def _planted(seed, n, T, dt, planted=4, thr=1.0):
    rng = np.random.default_rng(seed)
    el = catalog.leo_mix(rng, n)
    pl = catalog.plant_conjunctions(rng, el, planted, T, dt, thr)
    return el, pl


def _witnesses(el, T, delta, thr, start=0):
    W = oracle.brute_force(el, thr / 2.0, start + T, delta, 1e-3)
    W = W[W[:, 0] >= start]
    return {(int(i), int(j), int(t) - start) for t, i, j in W.tolist()}


def _records(el, dt, T, thr, start=0, rule=0):
    b = oracle.boxes(el, dt, T, 1e-3, thr, start=start, rule=rule)
    return oracle.pairs(b)


@pytest.mark.parametrize("start,delta", [(0, 1), (0, 7), (12_345, 1), (12_345, 50)])
def test_single_instant_leaves_are_the_brute_force_witnesses(start, delta):
    T, dt, thr = 20_000, 2_000, 1.0
    el, pl = _planted(21, 40, T, dt, thr=thr)
    # shift the planted pairs so they meet at start + t_c
    n_mean = np.sqrt(oracle.MU_EARTH / el[:, 0] ** 3)
    for i, j, _ in pl:
        for o in (i, j):
            el[o, 5] = (el[o, 5] - n_mean[o] * start * 1e-3) % (2 * np.pi)
    rec = _records(el, dt, T, thr, start)
    leaves = oracle.refine(el, rec, T, 1e-3, thr, delta, 1, start=start)
    got = {(int(i), int(j), int(a)) for i, j, a, b in leaves.tolist()}
    assert all(b == a + 1 for _, _, a, b in leaves.tolist())
    want = _witnesses(el, T, delta, thr, start)
    assert len(want) > 0
    assert got == want


@pytest.mark.parametrize("rule", [1, 2])
def test_interval_rules_hold_every_witness(rule):
    T, dt, thr, delta = 20_000, 4_000, 1.0, 1
    el, _ = _planted(22, 40, T, dt, thr=thr)
    rec = _records(el, dt, T, thr, rule=rule)
    leaves = oracle.refine(el, rec, T, 1e-3, thr, delta, 1, rule=rule)
    got = {(int(i), int(j), int(a)) for i, j, a, b in leaves.tolist()}
    want = _witnesses(el, T, delta, thr)
    assert want <= got
    for i, j, t in got - want:
        pi = oracle.position(el[i], t * 1e-3)
        pj = oracle.position(el[j], t * 1e-3)
        assert np.max(np.abs(pi - pj)) <= thr + 1e-5


@pytest.mark.parametrize("rule", [0, 2])
def test_coarse_leaves_cover_witnesses_inside_records(rule):
    T, dt, thr, delta, ms = 20_000, 5_000, 1.0, 3, 8
    el, _ = _planted(23, 40, T, dt, thr=thr)
    rec = _records(el, dt, T, thr, rule=rule)
    leaves = oracle.refine(el, rec, T, 1e-3, thr, delta, ms, rule=rule)
    want = _witnesses(el, T, delta, thr)
    for i, j, t in want:
        assert any(a <= t < b for a_i, a_j, a, b in leaves.tolist() if (a_i, a_j) == (i, j))
    for i, j, a, b in leaves.tolist():
        # at most ms grid instants, all inside one of the pair's records
        assert a % delta == 0 and (b - 1) % delta == 0 and (b - 1 - a) // delta + 1 <= ms
        assert any(lo <= a and b <= hi for ri, rj, lo, hi in rec.tolist() if (ri, rj) == (i, j))
    # halving never emits more than the records' own instants
    assert len(leaves) <= sum((hi - lo) for _, _, lo, hi in rec.tolist())


def test_whole_horizon_record_of_a_planted_pair():
    """A caller's record spanning the whole horizon: the refinement finds the
    pair's brute-force instants by halving alone."""
    T, thr = 30_000, 1.0
    el, pl = _planted(24, 12, T, 1000, planted=3, thr=thr)
    want = _witnesses(el, T, 1, thr)
    for i, j, tc in pl:
        rec = np.array([[i, j, 0, T + 1]], np.uint32)
        leaves = oracle.refine(el, rec, T, 1e-3, thr, 1, 1)
        got = {(int(a), int(b), int(t)) for a, b, t, _ in leaves.tolist()}
        assert got == {w for w in want if w[:2] == (i, j)}
        assert (i, j, tc) in got


def test_empty_and_errors():
    el, _ = _planted(25, 10, 1000, 1000, planted=0)
    none = np.zeros((0, 4), np.uint32)
    assert len(oracle.refine(el, none, 1000, 1e-3, 1.0, 1)) == 0
    far = np.array([[0, 1, 0, 1001]], np.uint32)   # two unplanted objects, far apart
    assert len(oracle.refine(el, far, 1000, 1e-3, 1.0, 1)) == 0
    with pytest.raises(ValueError):
        oracle.refine(el, far, 1000, 1e-3, 1.0, 0)
    with pytest.raises(ValueError):
        oracle.refine(el, far, 1000, 1e-3, 1.0, 1, min_steps=0)
