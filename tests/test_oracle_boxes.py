"""Pins for the oracle's 4D boxes (Def. Interval Occupancy Region, Def. 4D
Occupancy Region, advanceTime's clamp at T)."""
import math

import numpy as np
import pytest

import oracle

MU = oracle.MU_EARTH
TICK = 1e-3


def _el(rng, k):
    return np.stack([rng.uniform(6578, 42164, k), rng.uniform(0, 0.3, k),
                     rng.uniform(0, math.pi, k), rng.uniform(0, 2 * math.pi, k),
                     rng.uniform(0, 2 * math.pi, k), rng.uniform(0, 2 * math.pi, k)], 1)


def test_property1_single_instant_is_occ():
    """T = 0: one zero-length interval per object; the box is exactly the
    occupancy cube of radius thr/2 about pos(0)."""
    rng = np.random.default_rng(1)
    el = _el(rng, 25)
    b = oracle.boxes(el, 1000, 0, TICK, 1.0)
    assert len(b) == 25
    for i in range(25):
        p = oracle.position(el[i], 0.0)
        assert np.array_equal(b.lo[i], p - 0.5)
        assert np.array_equal(b.hi[i], p + 0.5)
        assert (b.t0[i], b.t1[i], b.obj[i]) == (0, 1, i)


def test_interval_count_tags_and_truncated_last_interval():
    el = np.array([[7000.0, 0.01, 0.5, 0.1, 0.2, 0.3]])
    # dt does not divide T: intervals [0,10) [10,20) [20, 25] -> tag [20, 26)
    b = oracle.boxes(el, 10, 25, TICK, 1.0)
    assert list(b.t0) == [0, 10, 20]
    assert list(b.t1) == [10, 20, 26]
    # the truncated interval's motion term uses its true length, 5 ticks
    p20 = oracle.position(el[0], 20 * TICK)
    p25 = oracle.position(el[0], 25 * TICK)
    g = oracle.vmax(7000.0, 0.01) * (5 * TICK) / 2 + 0.5
    assert np.allclose(b.lo[2], np.minimum(p20, p25) - g, rtol=0, atol=1e-12)
    assert np.allclose(b.hi[2], np.maximum(p20, p25) + g, rtol=0, atol=1e-12)
    # dt >= T gives one interval [0, T] with tag [0, T + 1)
    b1 = oracle.boxes(el, 1000, 700, TICK, 1.0)
    assert list(b1.t0) == [0] and list(b1.t1) == [701]
    # dt dividing T exactly
    b2 = oracle.boxes(el, 5, 20, TICK, 1.0)
    assert list(b2.t0) == [0, 5, 10, 15] and list(b2.t1) == [5, 10, 15, 21]


def test_object_major_order_and_counts():
    rng = np.random.default_rng(2)
    el = _el(rng, 7)
    dt = np.array([3, 7, 1, 100, 9, 10, 2], np.uint32)
    T = 40
    b = oracle.boxes(el, dt, T, TICK, 1.0)
    K = [math.ceil(T / d) for d in dt]
    assert len(b) == sum(K)
    assert list(b.obj) == [i for i in range(7) for _ in range(K[i])]
    off = 0
    for i in range(7):
        t0 = b.t0[off:off + K[i]]
        t1 = b.t1[off:off + K[i]]
        # tags tile [0, T] exactly, half-open, last one closed at T
        assert t0[0] == 0 and t1[-1] == T + 1
        assert np.all(t0[1:] == t1[:-1])
        off += K[i]


def test_invalid_inputs_rejected():
    el = np.array([[7000.0, 0.01, 0.5, 0.1, 0.2, 0.3]])
    with pytest.raises(ValueError):
        oracle.boxes(el, 0, 100, TICK, 1.0)
    with pytest.raises(ValueError):
        oracle.boxes(el, 10, 2 ** 32 - 1, TICK, 1.0)


def test_circular_equatorial_exact_bounds():
    """x(t) = a cos(theta): the interval straddling theta = 0 must reach x = a,
    and the box equals the closed form of its definition."""
    a = 7000.0
    n = math.sqrt(MU / a ** 3)
    dt_ticks = 60_000                      # 60 s
    phi = n * 30.0                         # half the swept angle
    el = np.array([[a, 0.0, 0.0, 0.0, 0.0, -phi]])   # theta(0) = -phi
    b = oracle.boxes(el, dt_ticks, dt_ticks, TICK, 1.0)
    v = math.sqrt(MU / a)
    g = v * 60.0 / 2 + 0.5
    want_lo = np.array([a * math.cos(phi) - g, -a * math.sin(phi) - g, -g])
    want_hi = np.array([a * math.cos(phi) + g, a * math.sin(phi) + g, g])
    assert np.allclose(b.lo[0], want_lo, rtol=0, atol=1e-9)
    assert np.allclose(b.hi[0], want_hi, rtol=0, atol=1e-9)
    assert b.hi[0][0] - 0.5 >= a          # true extremum inside the box


def test_boxes_contain_dense_samples():
    """Superset property of occ-int: every position inside the interval lies in
    the box shrunk by the radius (64 samples per interval)."""
    rng = np.random.default_rng(4)
    el = _el(rng, 30)
    T, dt = 600_000, 97_000
    b = oracle.boxes(el, dt, T, TICK, 1.0)
    for k in range(len(b)):
        i = b.obj[k]
        t_end = min(b.t1[k], T)
        for s in np.linspace(b.t0[k], t_end, 64):
            p = oracle.position(el[i], s * TICK)
            assert np.all(p >= b.lo[k] + 0.5 - 1e-9) and np.all(p <= b.hi[k] - 0.5 + 1e-9)


def test_motion_term_is_needed():
    """Without the vmax term some sampled position would leave the endpoint
    hull: the growth is not decorative."""
    rng = np.random.default_rng(6)
    el = _el(rng, 4)
    el[:, 0] = rng.uniform(6578, 8000, 4)         # LEO: several turning points
    T, dt = 6_000_000, 200_000
    b = oracle.boxes(el, dt, T, TICK, 0.0)
    worst = 0.0
    for k in range(len(b)):
        i = b.obj[k]
        pa = oracle.position(el[i], b.t0[k] * TICK)
        pb = oracle.position(el[i], min(b.t1[k], T) * TICK)
        hull_lo, hull_hi = np.minimum(pa, pb), np.maximum(pa, pb)
        for s in np.linspace(b.t0[k], min(b.t1[k], T), 33):
            p = oracle.position(el[i], s * TICK)
            worst = max(worst, np.max(hull_lo - p), np.max(p - hull_hi))
            assert np.all(p >= b.lo[k] - 1e-9) and np.all(p <= b.hi[k] + 1e-9)
    assert worst > 1.0


def test_outward_rounding_f32():
    rng = np.random.default_rng(8)
    xs = np.concatenate([rng.uniform(-45000, 45000, 20000), [0.0, 1.0, -1.0, 0.1, 1e-30]])
    for x in xs:
        d = oracle.round_down_f32(x)
        u = oracle.round_up_f32(x)
        assert float(d) <= x <= float(u)
        # tight: the next float beyond each bound is on the other side of x
        assert float(np.nextafter(d, np.float32(np.inf))) > x or float(d) == x
        assert float(np.nextafter(u, np.float32(-np.inf))) < x or float(u) == x
        if float(np.float32(x)) == x:
            assert d == u


def test_dt_heuristic_bound():
    rng = np.random.default_rng(9)
    el = _el(rng, 500)
    dt = oracle.dt_heuristic(el, TICK, 5.0, 3_600_000)
    for i in range(500):
        v = oracle.vmax(el[i][0], el[i][1])
        assert dt[i] >= 1
        assert v * dt[i] * TICK <= 5.0 + 1e-12          # displacement bound holds
        assert v * (dt[i] + 1) * TICK > 5.0             # and is the largest such step


def test_window_boxes_are_the_shifted_tail_of_the_long_horizon():
    """A horizon [S, S + T] with S a multiple of every step is the tail of the
    horizon [0, S + T]: same positions (same absolute ticks), tags shifted by S."""
    import numpy as np
    import oracle
    from paper_1901_10475_amd import catalog
    sc = catalog.scaled(catalog.small_leo(), n=20)
    dt = np.array([1000, 2000, 500, 4000] * 5, np.uint32)
    S, T = 8000, 6000
    long = oracle.boxes(sc.elements, dt, S + T, sc.tick_s, sc.threshold_km)
    win = oracle.boxes(sc.elements, dt, T, sc.tick_s, sc.threshold_km, start=S)
    keep = long.t0 >= S
    assert keep.sum() == len(win.t0)
    np.testing.assert_array_equal(long.lo[keep], win.lo)
    np.testing.assert_array_equal(long.hi[keep], win.hi)
    np.testing.assert_array_equal(long.t0[keep] - S, win.t0)
    np.testing.assert_array_equal(long.t1[keep] - S, win.t1)
    np.testing.assert_array_equal(long.obj[keep], win.obj)
