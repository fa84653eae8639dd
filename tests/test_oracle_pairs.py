"""Pins for the oracle's pair sets: hand cases, invariants, and recall against
the paper's Alg. Brute Force."""
import math

import numpy as np

import oracle
from paper_1901_10475_amd import catalog

MU = oracle.MU_EARTH
TICK = 1e-3


def _soup(lo, hi, t0, t1, obj):
    return oracle.Boxes(np.asarray(lo, float).reshape(-1, 3), np.asarray(hi, float).reshape(-1, 3),
                        np.asarray(t0, np.uint32), np.asarray(t1, np.uint32),
                        np.asarray(obj, np.uint32))


def test_closed_comparison_touching_boxes():
    """H9: closed cubes that only touch do intersect; one ulp apart they don't."""
    b = _soup([[0, 0, 0], [1, 0, 0]], [[1, 1, 1], [2, 1, 1]], [0, 0], [5, 5], [0, 1])
    assert oracle.pairs(b).tolist() == [[0, 1, 0, 5]]
    b2 = _soup([[0, 0, 0], [np.nextafter(1.0, 2.0), 0, 0]], [[1, 1, 1], [2, 1, 1]],
               [0, 0], [5, 5], [0, 1])
    assert len(oracle.pairs(b2)) == 0


def test_half_open_time_and_self_exclusion():
    lo = [[0, 0, 0]] * 4
    hi = [[1, 1, 1]] * 4
    # [0,10) vs [10,20): adjacent, no overlap; [0,10) vs [9,20): overlap [9,10)
    b = _soup(lo[:2], hi[:2], [0, 10], [10, 20], [0, 1])
    assert len(oracle.pairs(b)) == 0
    b = _soup(lo[:2], hi[:2], [0, 9], [10, 20], [3, 1])
    assert oracle.pairs(b).tolist() == [[1, 3, 9, 10]]
    # same object never pairs with itself
    b = _soup(lo[:2], hi[:2], [0, 0], [10, 10], [2, 2])
    assert len(oracle.pairs(b)) == 0


def test_invariance_under_permutation_and_exact_translation():
    rng = np.random.default_rng(0)
    lo, hi, t0, t1, obj = catalog.random_boxes(1, 600, 50, extent=64, size=8, T=50)
    # snap to a dyadic grid so that a translation by 256 is exact
    lo, hi = np.floor(lo * 8) / 8, np.ceil(hi * 8) / 8
    b = _soup(lo, hi, t0, t1, obj)
    ref = oracle.pairs(b)
    assert len(ref) > 50
    perm = rng.permutation(600)
    assert np.array_equal(oracle.pairs(b.take(perm)), ref)
    shift = np.array([256.0, -512.0, 1024.0])
    assert np.array_equal(oracle.pairs(_soup(lo + shift, hi + shift, t0, t1, obj)), ref)
    # shifting time by a constant shifts every record's interval
    rec = oracle.pairs(_soup(lo, hi, t0 + 7, t1 + 7, obj))
    assert np.array_equal(rec[:, 2:], ref[:, 2:] + 7) and np.array_equal(rec[:, :2], ref[:, :2])


def test_each_record_has_a_common_point():
    """Constructive check: for every record a point exists in both boxes at a
    time inside both tags; for every non-record pair an axis separates."""
    lo, hi, t0, t1, obj = catalog.random_boxes(2, 300, 40, extent=50, size=8, T=30)
    b = _soup(lo, hi, t0, t1, obj)
    rec = {tuple(r) for r in oracle.pairs(b).tolist()}
    found = set()
    for a in range(300):
        for c in range(a + 1, 300):
            if obj[a] == obj[c]:
                continue
            x = np.maximum(lo[a], lo[c])             # candidate common point
            t = max(t0[a], t0[c])
            inside = (np.all(lo[a] <= x) and np.all(x <= hi[a]) and np.all(lo[c] <= x)
                      and np.all(x <= hi[c]) and t0[a] <= t < t1[a] and t0[c] <= t < t1[c])
            key = (min(obj[a], obj[c]), max(obj[a], obj[c]), t, min(t1[a], t1[c]))
            if inside:
                found.add(key)
    assert found == rec


def test_sampled_partners_partition_the_full_set():
    lo, hi, t0, t1, obj = catalog.random_boxes(3, 500, 60, extent=40, size=6, T=40)
    b = _soup(lo, hi, t0, t1, obj)
    ref = oracle.pairs(b)
    assert np.array_equal(oracle.pairs_of(b, np.arange(500)), ref)
    parts = [oracle.pairs_of(b, np.arange(k, 500, 7)) for k in range(7)]
    u = np.unique(np.concatenate(parts), axis=0)
    assert np.array_equal(u, ref)


def test_time_overlap_count_fixed_step():
    """Aligned fixed steps: only boxes of the same step overlap in time, so the
    brute-force-equivalent count is K * C(n, 2)."""
    rng = np.random.default_rng(5)
    el = catalog.leo_mix(rng, 30)
    b = oracle.boxes(el, 10, 95, TICK, 1.0)
    assert oracle.time_overlapping_pairs(b) == 10 * (30 * 29 // 2)


def test_identical_elements_overlap_every_interval():
    """H1 / H7: duplicated elements (the docked vehicles of Sec. 7.2) give one
    record per interval, the last one closed at T."""
    el = np.array([[6800.0, 0.001, 0.9, 0.2, 0.3, 0.4]] * 2)
    b = oracle.boxes(el, 10_000, 25_000, TICK, 1.0)
    assert oracle.pairs(b).tolist() == [[0, 1, 0, 10000], [0, 1, 10000, 20000],
                                        [0, 1, 20000, 25001]]


def test_phased_and_concentric_orbits():
    """H2: one circular orbit, phased far apart -> nothing.  H3: coplanar
    circles closer than the threshold -> every interval; far -> nothing."""
    a = 7000.0
    el = np.array([[a, 0.0, 0.3, 0.1, 0.0, 0.0], [a, 0.0, 0.3, 0.1, 0.0, 0.5]])
    assert len(oracle.pairs(oracle.boxes(el, 10_000, 600_000, TICK, 1.0))) == 0
    el = np.array([[a, 0.0, 0.3, 0.1, 0.0, 0.0], [a + 0.4, 0.0, 0.3, 0.1, 0.0, 0.0]])
    rec = oracle.pairs(oracle.boxes(el, 10_000, 100_000, TICK, 1.0))
    assert len(rec) == 10
    el = np.array([[a, 0.0, 0.3, 0.1, 0.0, 0.0], [a + 200.0, 0.0, 0.3, 0.1, 0.0, 3.0]])
    assert len(oracle.pairs(oracle.boxes(el, 10_000, 600_000, TICK, 1.0))) == 0


def test_crossing_at_node_reported_at_the_right_time():
    """H5: equatorial and polar circles of one radius, phased to meet at the
    node at t_c: a record covers t_c and Alg. Brute Force finds a witness there."""
    a = 7000.0
    n = math.sqrt(MU / a ** 3)
    tc = 123_456                            # ticks
    m0 = (-n * tc * TICK) % (2 * math.pi)
    el = np.array([[a, 0.0, 0.0, 0.0, 0.0, m0], [a, 0.0, math.pi / 2, 0.0, 0.0, m0]])
    rec = oracle.pairs(oracle.boxes(el, 10_000, 300_000, TICK, 1.0))
    assert any(r[2] <= tc < r[3] for r in rec)
    # sampled every tick the pair meets at t_c; sampled every second it tunnels
    assert len(oracle.brute_force(el, 0.5, 300_000, 1_000, TICK)) == 0
    w = oracle.brute_force(el, 0.5, 300_000, 1, TICK)
    # perpendicular tracks at speed v: inf-norm gap v |t - t_c| <= thr, so the
    # witnesses are the ticks within thr / v of t_c (one tick of slack)
    half = 1.0 / math.sqrt(MU / a) / TICK
    ts = w[:, 0].astype(np.int64)
    assert len(ts) and np.all(np.diff(ts) == 1)
    assert abs((tc - ts[0]) - half) <= 1.5 and abs((ts[-1] - tc) - half) <= 1.5
    assert all(any(r[2] <= t < r[3] for r in rec) for t, _, _ in w)


def test_perigee_apogee_separation_gives_no_record():
    """Sec. 7.1's static test: apogee below the other's perigee (with margin for
    the box growth) means no collision and, here, no record."""
    rng = np.random.default_rng(12)
    leo = catalog.leo_mix(rng, 60)
    geo = catalog.tracked_population(rng, 400)[-60:]      # GEO ring
    el = np.concatenate([leo, geo])
    T, dt, thr = 60_000, 10_000, 1.0
    b = oracle.boxes(el, dt, T, TICK, thr)
    rec = oracle.pairs(b)
    for i, j, _, _ in rec:
        assert (i < 60) == (j < 60)           # never LEO with GEO
    # margin bound from the box geometry, checked explicitly
    for i in range(60):
        apo = leo[i][0] * (1 + leo[i][1])
        g = oracle.vmax(leo[i][0], leo[i][1]) * 10.0 / 2 + thr / 2
        assert apo + math.sqrt(3) * (g + 80.0) < 35000.0


def test_degenerate_sizes():
    """H8: n = 0 and n = 1 give no records."""
    b = oracle.boxes(np.zeros((0, 6)), 10, 100, TICK, 1.0)
    assert len(b) == 0 and len(oracle.pairs(b)) == 0
    b = oracle.boxes(np.array([[7000.0, 0, 0, 0, 0, 0]]), 10, 100, TICK, 1.0)
    assert len(b) == 10 and len(oracle.pairs(b)) == 0


def test_recall_against_brute_force_small_catalog():
    """Every collision Alg. Brute Force finds at a fine step (continuous
    sampling of the same horizon) is covered by a record."""
    sc = catalog.small_leo(seed=31, n=120, planted=12)
    sc = catalog.scaled(sc, horizon_ticks=60_000)          # 60 s, dt = 10 s
    b = oracle.boxes(sc.elements, sc.dt_ticks, sc.horizon_ticks, TICK, sc.threshold_km)
    rec = oracle.pairs(b)
    w = oracle.brute_force(sc.elements, sc.threshold_km / 2, sc.horizon_ticks, 100, TICK)
    assert len(w) > 0
    cover = {}
    for r in rec.tolist():
        cover.setdefault((r[0], r[1]), []).append((r[2], r[3]))
    for t, i, j in w.tolist():
        assert any(a <= t < b_ for a, b_ in cover.get((i, j), [])), (t, i, j)
    planted_in = [p for p in sc.planted if p[2] <= sc.horizon_ticks]
    hit = {(int(i), int(j)) for _, i, j in w.tolist()}
    for i, j, tc in planted_in:
        assert (i, j) in hit


# ---- the bucketed driver: the same set as the literal one ------------------

def _both(b):
    lit = oracle.pairs(b)
    buck = oracle.pairs_bucketed(b)
    assert np.array_equal(lit, buck), (len(lit), len(buck))
    return lit


def test_bucketed_equals_literal_on_box_soups():
    """Caller-built boxes with ragged tags (overlapping intervals of lengths
    1..max_len, so the active list carries boxes across blocks), in all five
    geometries and sizes around the block size."""
    for kind in ("uniform", "identical", "disjoint", "line", "huge"):
        for N in (0, 1, 2, 3, 63, 64, 65, 1023, 1024, 1025, 2049, 5000):
            if kind == "identical" and N > 2049:
                continue
            for max_len, T in ((1, 40), (12, 400), (300, 500)):
                lo, hi, t0, t1, obj = catalog.random_boxes(N + 7 * max_len, N, max(2, N // 4),
                                                           extent=200, size=6, T=T,
                                                           max_len=max_len, kind=kind)
                _both(_soup(lo, hi, t0, t1, obj))


def test_bucketed_equals_literal_on_orbit_boxes():
    """Uniform steps (slabs), per-object steps (sweep), windows, the T + 1
    sentinel, and dt not dividing T."""
    sc = catalog.scaled(catalog.small_leo(seed=41, n=700, planted=12), horizon_ticks=61_000)
    b = oracle.boxes(sc.elements, 10_000, sc.horizon_ticks, TICK, sc.threshold_km)
    assert len(_both(b)) > 0
    dt = oracle.dt_heuristic(sc.elements, TICK, 5.0, sc.horizon_ticks)
    b = oracle.boxes(sc.elements, dt, sc.horizon_ticks, TICK, sc.threshold_km)
    assert len(_both(b)) > 0
    b = oracle.boxes(sc.elements, dt * 7, sc.horizon_ticks, TICK, sc.threshold_km,
                     start=1_234_567)
    assert len(_both(b)) > 0
    # mixed populations: per-object steps from 1 tick to beyond T
    rng = np.random.default_rng(8)
    el = catalog.tracked_population(rng, 500)
    dt = rng.integers(1, 90_000, 500).astype(np.uint32)
    dt[:40] = rng.integers(1, 50, 40)
    b = oracle.boxes(el, dt, 70_000, TICK, 200.0)
    assert len(_both(b)) > 0


def test_bucketed_equals_literal_on_hand_cases():
    el = np.array([[6800.0, 0.001, 0.9, 0.2, 0.3, 0.4]] * 2)
    assert _both(oracle.boxes(el, 10_000, 25_000, TICK, 1.0)).tolist() == \
        [[0, 1, 0, 10000], [0, 1, 10000, 20000], [0, 1, 20000, 25001]]
    assert _both(oracle.boxes(el, 1_000, 0, TICK, 1.0)).tolist() == [[0, 1, 0, 1]]
    b = _soup([[0, 0, 0], [1, 0, 0]], [[1, 1, 1], [2, 1, 1]], [0, 0], [5, 5], [0, 1])
    assert _both(b).tolist() == [[0, 1, 0, 5]]
    lo = [[0, 0, 0]] * 2
    hi = [[1, 1, 1]] * 2
    assert len(_both(_soup(lo, hi, [0, 10], [10, 20], [0, 1]))) == 0
    assert _both(_soup(lo, hi, [0, 9], [10, 20], [3, 1])).tolist() == [[1, 3, 9, 10]]
    assert len(_both(_soup(lo, hi, [0, 0], [10, 10], [2, 2]))) == 0
    assert len(_both(oracle.boxes(np.zeros((0, 6)), 10, 100, TICK, 1.0))) == 0
    assert len(_both(oracle.boxes(np.array([[7000.0, 0, 0, 0, 0, 0]]), 10, 100, TICK,
                                  1.0))) == 0


def test_bucketed_result_does_not_depend_on_threads():
    lo, hi, t0, t1, obj = catalog.random_boxes(9, 3000, 400, extent=60, size=8, T=60,
                                               max_len=20)
    b = _soup(lo, hi, t0, t1, obj)
    ref = oracle.pairs_bucketed(b)
    nt = oracle.num_threads()
    try:
        oracle.set_num_threads(1)
        assert np.array_equal(oracle.pairs_bucketed(b), ref)
        oracle.set_num_threads(3)
        assert np.array_equal(oracle.pairs_bucketed(b), ref)
    finally:
        oracle.set_num_threads(nt)
    assert np.array_equal(oracle.pairs(b), ref)


def test_time_window_restriction_is_exact():
    """The records of the boxes that meet [ta, tb) are exactly the records of
    all boxes whose interval meets [ta, tb) (the reduction the full-size GPU
    tests use to check long horizons window by window)."""
    sc = catalog.scaled(catalog.tracked_hour(seed=17, planted=6), n=900, horizon_ticks=40_000)
    dt = oracle.dt_heuristic(sc.elements, TICK, 5.0, sc.horizon_ticks) * 3
    b = oracle.boxes(sc.elements, dt, sc.horizon_ticks, TICK, 400.0)
    full = oracle.pairs_bucketed(b)
    assert len(full) > 1000 and np.array_equal(full, oracle.pairs(b))
    for ta, tb in ((0, 1), (0, 5_000), (12_345, 12_346), (17_000, 23_500), (39_000, 40_001)):
        got = oracle.pairs_bucketed(oracle.window(b, ta, tb))
        want = oracle.records_in_window(full, ta, tb)
        assert np.array_equal(got, want), (ta, tb)
        assert len(want) > 0
