"""Pins of the oracle's potential-collision graph by altitude bands (Def.
Potential-Collision Graph; the perigee/apogee test and the edge partitioning
of the orbit evaluation).

References independent of the band formula: a constructed pair of circular
orbits whose occupancy cubes touch corner to corner along the radial
direction (the largest radial gap a collision allows), Alg. Brute Force's
witnesses, and the literal all-pairs records of each band's own catalog.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1901_10475_amd import catalog

MU = oracle.MU_EARTH


def _corner_pair(R1, gap, t_s=100.0):
    """Two circular polar orbits (RAAN 45 deg) of radii R1 and R1 + gap that
    both point along (1, 1, 1)/sqrt(3) at time t_s."""
    alpha = math.atan(1.0 / math.sqrt(2.0))     # argument of latitude of (1,1,1)
    out = []
    for a in (R1, R1 + gap):
        n = math.sqrt(MU / a ** 3)
        out.append([a, 0.0, math.pi / 2, math.pi / 4, 0.0, (alpha - n * t_s) % (2 * math.pi)])
    return np.array(out)


def test_corner_touch_is_the_widest_compatible_gap():
    thr, t = 2.0, 100.0
    inside = _corner_pair(7000.0, math.sqrt(3) * thr * (1 - 1e-9), t)
    p1, p2 = oracle.position(inside[0], t), oracle.position(inside[1], t)
    u = np.ones(3) / math.sqrt(3)
    assert np.allclose(p1 / np.linalg.norm(p1), u, atol=1e-12)
    assert np.max(np.abs(p2 - p1)) <= thr                  # the cubes meet: a collision
    assert oracle.band_compatible(inside[0], inside[1], thr)
    outside = _corner_pair(7000.0, math.sqrt(3) * thr * (1 + 1e-6), t)
    q1, q2 = oracle.position(outside[0], t), oracle.position(outside[1], t)
    assert np.max(np.abs(q2 - q1)) > thr
    assert not oracle.band_compatible(outside[0], outside[1], thr)


def test_band_holds_every_position():
    rng = np.random.default_rng(31)
    el = catalog.tracked_population(rng, 300)
    for e6 in el[::7]:
        lo, hi = oracle.band(e6, 1.0)
        P = 2 * math.pi * math.sqrt(e6[0] ** 3 / MU)
        r = [np.linalg.norm(oracle.position(e6, t)) for t in np.linspace(0, P, 400)]
        assert lo <= min(r) - 0.5 * math.sqrt(3) + 1e-6 and max(r) + 0.5 * math.sqrt(3) <= hi + 1e-6


def _mixed(seed, n, T, dt, thr):
    rng = np.random.default_rng(seed)
    el = catalog.tracked_population(rng, n)
    k = n // 10    # some highly eccentric orbits crossing several bands
    el[:k, 0] = rng.uniform(15000.0, 26000.0, k)
    el[:k, 1] = rng.uniform(0.5, 0.7, k)
    pl = catalog.plant_conjunctions(rng, el, 4, T, dt, thr)
    return el, pl


def test_filter_keeps_every_witness_and_drops_only_incompatible_pairs():
    T, dt, thr = 20_000, 2_000, 40.0
    el, pl = _mixed(32, 200, T, dt, thr)
    rec = oracle.pairs(oracle.boxes(el, dt, T, 1e-3, thr))
    kept = oracle.band_filter(el, rec, thr)
    dropped = {tuple(x) for x in rec.tolist()} - {tuple(x) for x in kept.tolist()}
    assert len(kept) > 0
    for i, j, _, _ in dropped:
        assert not oracle.band_compatible(el[i], el[j], thr)
    W = oracle.brute_force(el, thr / 2, T, 1, 1e-3)
    assert len(W) > 0
    keys = {(int(i), int(j)) for i, j, _, _ in kept.tolist()}
    for t, i, j in W.tolist():
        assert (i, j) in keys


@pytest.mark.parametrize("p", [1, 2, 5, 16])
def test_partition_covers_every_compatible_pair_and_balances(p):
    thr = 40.0
    el, _ = _mixed(33, 400, 1000, 1000, thr)
    edges, bands = oracle.band_partition(el, thr, p)
    assert len(bands) == p and edges[0] == -np.inf and edges[-1] == np.inf
    assert np.all(np.diff(edges) >= 0)
    where = [set() for _ in range(len(el))]
    for k, ids in enumerate(bands):
        assert np.all(np.diff(ids.astype(np.int64)) > 0)
        for i in ids:
            where[i].add(k)
    for i in range(len(el)):
        assert where[i], i
        for j in range(i + 1, len(el)):
            if oracle.band_compatible(el[i], el[j], thr):
                assert where[i] & where[j], (i, j)
    # every band holds the objects whose semi-major axis falls in it: about n / p
    d = len(el) // p
    for k in range(p):
        own = np.sum((el[:, 0] >= edges[k]) & (el[:, 0] < edges[k + 1]))
        assert own <= d + 1 or k == p - 1


@pytest.mark.parametrize("p", [2, 4])
def test_union_of_band_problems_is_the_filtered_full_problem(p):
    T, dt, thr = 20_000, 2_000, 40.0
    el, _ = _mixed(34, 200, T, dt, thr)
    full = oracle.band_filter(el, oracle.pairs(oracle.boxes(el, dt, T, 1e-3, thr)), thr)
    _, bands = oracle.band_partition(el, thr, p)
    parts = []
    for ids in bands:
        if len(ids) < 2:
            continue
        r = oracle.pairs(oracle.boxes(el[ids], dt, T, 1e-3, thr))
        if len(r):
            i, j = ids[r[:, 0]], ids[r[:, 1]]
            r = np.stack([np.minimum(i, j), np.maximum(i, j), r[:, 2], r[:, 3]], axis=1)
            parts.append(r[[oracle.band_compatible(el[a], el[b], thr) for a, b in r[:, :2]]])
    union = np.unique(np.concatenate(parts), axis=0) if parts else np.zeros((0, 4), np.uint32)
    assert len(full) > 0
    assert np.array_equal(union.astype(np.uint32), full)
