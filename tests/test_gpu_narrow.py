"""Narrow phase: the first collision instant of every candidate record against
the oracle's Alg. Brute Force (every witness (t, i, j) at every instant).

Expected value of a record (i, j, t_lo, t_hi): the smallest brute-force
witness t of (i, j) with t_lo <= t < t_hi, or none.  The decision
||p_i - p_j||_inf <= thr is taken in FP64 on both sides from positions that
differ by rounding only, so an instant whose oracle distance lies within
1e-9 km of the threshold may go either way; every other instant must agree.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1901_10475_amd as cd
from paper_1901_10475_amd import catalog
from tests.gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu
NONE = 0xFFFFFFFF


def _planted_leo(seed, n, planted, T, dt):
    rng = np.random.default_rng(seed)
    el = catalog.leo_mix(rng, n)
    pl = catalog.plant_conjunctions(rng, el, planted, T, dt, 1.0)
    return catalog.Scenario(f"leo{n}_planted", el, dt, T, 1.0, planted=pl)


def _dist(sc, i, j, t_abs):
    pi = oracle.position(sc.elements[i], t_abs * sc.tick_s)
    pj = oracle.position(sc.elements[j], t_abs * sc.tick_s)
    return float(np.max(np.abs(np.asarray(pi) - np.asarray(pj))))


def _check(sc, start, delta, heur=None, box_rule=0):
    el = cd.soa(sc.elements)
    p = cd.params_struct(sc.tick_s, sc.mu, sc.threshold_km, sc.horizon_ticks,
                         sc.dt_ticks if heur is None else 0, start_ticks=start,
                         box_rule=box_rule)
    bp = cd.BroadPhase(sc.n, p, dt_heuristic_km=heur, el_soa=el)
    pairs = bp.run(el)
    wit, first = cd.cd_first_witness(el, p, delta, pairs)
    torch.cuda.synchronize()
    recs = pairs.cpu().numpy().view(np.uint32)
    got = wit.cpu().numpy().view(np.uint32)
    # oracle: every witness over absolute instants [0, start + T], kept in the window
    W = oracle.brute_force(sc.elements, sc.threshold_km / 2.0, start + sc.horizon_ticks, delta,
                           sc.tick_s)
    W = W[W[:, 0] >= start]
    wins = {}
    for t, i, j in W.tolist():
        wins.setdefault((i, j), []).append(t - start)
    say("records", len(recs), "witnesses", len(W), "with a witness", int((got != NONE).sum()))
    assert len(recs) > 0
    loose = 0
    for r, (i, j, tlo, thi) in enumerate(recs.tolist()):
        ts = [t for t in wins.get((i, j), []) if tlo <= t < thi]
        want = min(ts) if ts else NONE
        if got[r] != want:
            # only a threshold tie may differ
            for t in (got[r], want):
                if t != NONE:
                    assert abs(_dist(sc, i, j, start + t) - sc.threshold_km) <= 1e-9, (r, got[r],
                                                                                       want)
            loose += 1
    assert loose <= 1
    # every brute-force witness lies in some record (the broad phase is conservative)
    keyset = {}
    for i, j, tlo, thi in recs.tolist():
        keyset.setdefault((i, j), []).append((tlo, thi))
    for (i, j), ts in wins.items():
        for t in ts:
            assert any(a <= t < b for a, b in keyset.get((i, j), [])), (t, i, j)
    # the first collision
    fc = cd.first_collision(pairs, first)
    if len(W):
        t0, i0, j0 = W[0].tolist()
        assert fc == (t0 - start, i0, j0)
    else:
        assert fc is None
    return got


@pytest.mark.parametrize("delta", [1, 7, 50])
def test_first_witness_matches_brute_force(delta):
    need_gpu()
    T = 20_000 if delta == 1 else 60_000
    sc = _planted_leo(71, 120 if delta == 1 else 200, 6, T, 1000)
    say("narrow", sc.n, "T", T, "delta", delta)
    got = _check(sc, 0, delta)
    assert (got != NONE).sum() >= 1


def test_first_witness_window_and_per_object_steps():
    need_gpu()
    sc = _planted_leo(72, 160, 6, 40_000, 1000)
    say("narrow window + heuristic steps")
    _check(sc, 12_345, 10, heur=5.0)


@pytest.mark.parametrize("rule", [cd.CD_BOX_INTERVAL_NU, cd.CD_BOX_INTERVAL_E])
def test_first_witness_interval_boxes(rule):
    """Records from the interval-evaluation boxes still hold every brute-force
    witness, and the first collision is the brute-force answer."""
    need_gpu()
    sc = _planted_leo(74, 160, 6, 40_000, 2000)
    say("narrow interval boxes rule", rule)
    got = _check(sc, 3_000, 5, box_rule=rule)
    assert (got != NONE).sum() >= 1


def test_first_witness_empty_and_argument_errors():
    need_gpu()
    sc = _planted_leo(73, 20, 0, 1000, 1000)
    el = cd.soa(sc.elements)
    p = cd.params_struct(sc.tick_s, sc.mu, sc.threshold_km, sc.horizon_ticks, sc.dt_ticks)
    pairs = torch.empty((0, 4), dtype=torch.int32, device="cuda")
    wit, first = cd.cd_first_witness(el, p, 1, pairs)
    assert wit.numel() == 0 and cd.first_collision(pairs, first) is None
    with pytest.raises(cd.CDError):
        cd.cd_first_witness(el, p, 0, pairs)
