"""Pins of the oracle's interval arithmetic and interval-evaluation boxes
(Sec. 4.5, Def. Interval Occupancy Region with Properties 1 and 2).

Each check rests on something other than the oracle's own formulas: the
paper's two worked examples, dense sampling of the functions and of the
propagated path, and nesting.
"""
import math

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.filterwarnings("ignore")

ULP4 = 4 * np.finfo(float).eps


def _contains(outer, inner, slack=0.0):
    return outer[0] <= inner[0] + slack and inner[1] <= outer[1] + slack


# ---- the worked examples of Sec. 4.5 --------------------------------------

def test_linear_example_2x_plus_y():
    # f(x, y) = 2x + y, x in [1, 2], y in [2, 4]  ->  [4, 8]
    two_x = oracle.iv_op("mul", (2.0, 2.0), (1.0, 2.0))
    f = oracle.iv_op("add", two_x, (2.0, 4.0))
    assert _contains(f, (4.0, 8.0))
    assert abs(f[0] - 4.0) <= 4 * ULP4 * 4 and abs(f[1] - 8.0) <= 4 * ULP4 * 8


def test_dependency_example_x_times_x():
    # x * x over [-1, 1]: the naive product gives [-1, 1], the true range is [0, 1]
    naive = oracle.iv_op("mul", (-1.0, 1.0), (-1.0, 1.0))
    assert _contains(naive, (-1.0, 1.0)) and naive[0] <= -1.0 + 1e-15
    sq = oracle.iv_op("sqr", (-1.0, 1.0))
    assert sq[0] == 0.0 and 1.0 <= sq[1] <= 1.0 + 1e-15


# ---- every operation contains the values at sampled points -----------------

def _rand_iv(rng, scale, avoid_zero=False):
    a, b = np.sort(rng.uniform(-scale, scale, 2))
    if avoid_zero:
        if a <= 0.0 <= b:
            a, b = (b + 0.1, b + 1.0) if rng.random() < 0.5 else (a - 1.0, a - 0.1)
    return (float(a), float(b))


@pytest.mark.parametrize("op", ["add", "sub", "mul", "div"])
def test_operations_contain_samples(op):
    rng = np.random.default_rng(11)
    fn = {"add": np.add, "sub": np.subtract, "mul": np.multiply, "div": np.divide}[op]
    for _ in range(300):
        A = _rand_iv(rng, 10.0)
        B = _rand_iv(rng, 10.0, avoid_zero=(op == "div"))
        r = oracle.iv_op(op, A, B)
        xs = np.concatenate([[A[0], A[1]], rng.uniform(*A, 40)])
        ys = np.concatenate([[B[0], B[1]], rng.uniform(*B, 40)])
        vals = fn(xs[:, None], ys[None, :])
        assert r[0] <= vals.min() and vals.max() <= r[1], (op, A, B, r)
        # and the bounds are attained at corners (up to the outward step)
        span = max(abs(vals.min()), abs(vals.max()), 1.0)
        assert vals.min() - r[0] <= 1e-14 * span and r[1] - vals.max() <= 1e-14 * span


@pytest.mark.parametrize("fn", ["cos", "sin"])
def test_cos_sin_range_against_dense_sampling(fn):
    rng = np.random.default_rng(12)
    f = getattr(np, fn)
    cases = [(0.0, 0.0), (1.0, 1.0), (-0.1, 0.1), (3.0, 3.3), (math.pi / 2 - 1e-3, math.pi / 2 + 1e-3),
             (0.0, 2 * math.pi), (-7.0, 0.5), (100.0, 103.0), (1e3, 1e3 + 1e-4)]
    for _ in range(200):
        c = rng.uniform(-50.0, 50.0)
        w = 10 ** rng.uniform(-6, 0.9)
        cases.append((c, c + w))
    for lo, hi in cases:
        r = oracle.iv_op(fn, (lo, hi))
        xs = np.linspace(lo, hi, 200_001)
        v = f(xs)
        step = (hi - lo) / 200_000
        assert r[0] <= v.min() and v.max() <= r[1], (fn, lo, hi, r)
        # tight: within the sampling error (step^2 / 2) of the sampled extremes
        tol = step * step / 2 + 1e-15
        assert v.min() - r[0] <= tol and r[1] - v.max() <= tol, (fn, lo, hi, r, v.min(), v.max())


# ---- interval-evaluation boxes ----------------------------------------------

MU = oracle.MU_EARTH
ORBITS = [
    np.array([6900.0, 0.0005, 0.9, 0.3, 0.5, 0.2]),      # low, near-circular
    np.array([7200.0, 0.02, 1.7, 4.0, 2.5, 5.9]),        # retrograde, mean anomaly near 2 pi
    np.array([12000.0, 0.3, 0.5, 1.0, 4.0, 3.0]),        # eccentric, near apogee
    np.array([26600.0, 0.7, 1.1, 2.0, 1.0, 6.1]),        # highly eccentric, near perigee
    np.array([42164.0, 0.0, 0.0, 0.0, 0.0, 1.0]),        # equatorial geostationary
]


def _period(el):
    return 2 * math.pi * math.sqrt(el[0] ** 3 / MU)


def _path(el, ta, tb, m=4001):
    ts = np.linspace(ta, tb, m)
    return np.stack([oracle.position(el, t) for t in ts])


def _intervals(el):
    P = _period(el)
    return [(10.0, 11.0), (100.0, 160.0), (0.0, 0.1 * P), (0.37 * P, 0.93 * P),
            (5.0, 5.0 + 1.5 * P)]


@pytest.mark.parametrize("rule", [0, 1, 2])
def test_box_contains_the_path(rule):
    thr = 2.0
    for el in ORBITS:
        vmax = oracle.vmax(el[0], el[1])
        for ta, tb in _intervals(el):
            if rule == 0:
                pa, pb = oracle.position(el, ta), oracle.position(el, tb)
                g = vmax * (tb - ta) / 2 + thr / 2
                lo, hi = np.minimum(pa, pb) - g, np.maximum(pa, pb) + g
            else:
                lo, hi = oracle.box_interval(el, ta, tb, thr, rule)
            pts = _path(el, ta, tb)
            assert np.all(pts - thr / 2 >= lo - 1e-9) and np.all(pts + thr / 2 <= hi + 1e-9), \
                (rule, el, ta, tb)


def test_eccentric_rule_is_the_exact_hull():
    """Rule 2 evaluates a single-occurrence form: its box is the hull of the
    path itself, up to sampling and its 1e-10 rad widening."""
    thr = 1.0
    for el in ORBITS:
        n = math.sqrt(MU / el[0] ** 3)
        for ta, tb in _intervals(el):
            lo, hi = oracle.box_interval(el, ta, tb, thr, 2)
            m = 20001
            pts = _path(el, ta, min(tb, ta + _period(el)), m)
            # sampling error: the path's curvature between samples (E moves at
            # most n (tb-ta)/(m-1)/(1-e) per sample)
            dE = n * (tb - ta) / (m - 1) / (1 - el[1])
            tol = el[0] * (1 + el[1]) * dE * dE / 2 + 1e-6 * el[0] / 7000.0
            assert np.all(np.abs(lo - (pts.min(0) - thr / 2)) <= tol), (el, ta, tb)
            assert np.all(np.abs(hi - (pts.max(0) + thr / 2)) <= tol), (el, ta, tb)


def test_full_turn_is_the_orbit_bounding_box():
    """Over a period or more, rule 2 gives the orbit's bounding box, which for
    a Kepler ellipse has the closed form centre_d +- sqrt((a P_d)^2 + (b Q_d)^2)
    with centre -a e P; P, Q built here from the three rotation matrices."""
    for el in ORBITS:
        a, e, inc, raan, argp = el[:5]
        Rz = lambda t: np.array([[math.cos(t), -math.sin(t), 0], [math.sin(t), math.cos(t), 0],
                                 [0, 0, 1]])
        Rx = lambda t: np.array([[1, 0, 0], [0, math.cos(t), -math.sin(t)],
                                 [0, math.sin(t), math.cos(t)]])
        M = Rz(raan) @ Rx(inc) @ Rz(argp)
        P, Q = M[:, 0], M[:, 1]
        b = a * math.sqrt(1 - e * e)
        half = np.sqrt((a * P) ** 2 + (b * Q) ** 2)
        ctr = -a * e * P
        lo, hi = oracle.box_interval(el, 3.0, 3.0 + 1.01 * _period(el), 0.0, 2)
        assert np.allclose(lo, ctr - half, atol=1e-6) and np.allclose(hi, ctr + half, atol=1e-6)
        # the true-anomaly rule contains it
        lo1, hi1 = oracle.box_interval(el, 3.0, 3.0 + 1.01 * _period(el), 0.0, 1)
        assert np.all(lo1 <= lo + 1e-6) and np.all(hi <= hi1 + 1e-6)


@pytest.mark.parametrize("rule", [1, 2])
def test_property1_single_instant(rule):
    thr = 3.0
    for el in ORBITS:
        for t in (0.0, 17.25, 0.5 * _period(el)):
            lo, hi = oracle.box_interval(el, t, t, thr, rule)
            p = oracle.position(el, t)
            assert np.allclose(lo, p - thr / 2, atol=1e-5) and np.allclose(hi, p + thr / 2,
                                                                           atol=1e-5)


@pytest.mark.parametrize("rule", [1, 2])
def test_property2_nested_intervals(rule):
    rng = np.random.default_rng(13)
    for el in ORBITS:
        P = _period(el)
        for _ in range(20):
            a2, b2 = np.sort(rng.uniform(0, 1.2 * P, 2))
            a1, b1 = np.sort(rng.uniform(a2, b2, 2))
            lo1, hi1 = oracle.box_interval(el, a1, b1, 1.0, rule)
            lo2, hi2 = oracle.box_interval(el, a2, b2, 1.0, rule)
            assert np.all(lo2 <= lo1 + 1e-9) and np.all(hi1 <= hi2 + 1e-9), (el, a1, b1, a2, b2)


def test_rules_tighten_in_order_on_short_steps():
    """On one-second intervals of a near-circular orbit: the exact hull (rule
    2) lies inside the true-anomaly evaluation (rule 1), which is smaller than
    the speed-bound box (rule 0)."""
    el = ORBITS[0]
    vmax = oracle.vmax(el[0], el[1])
    for t in np.arange(0.0, 600.0, 37.0):
        lo2, hi2 = oracle.box_interval(el, t, t + 1.0, 0.0, 2)
        lo1, hi1 = oracle.box_interval(el, t, t + 1.0, 0.0, 1)
        pa, pb = oracle.position(el, t), oracle.position(el, t + 1.0)
        g = vmax / 2
        lo0, hi0 = np.minimum(pa, pb) - g, np.maximum(pa, pb) + g
        assert np.all(lo1 <= lo2 + 1e-9) and np.all(hi2 <= hi1 + 1e-9)
        assert np.prod(hi1 - lo1) < np.prod(hi0 - lo0)


def test_boxes_take_the_rule():
    rng = np.random.default_rng(14)
    el = np.stack(ORBITS)
    dt = np.array([1000, 7000, 30000, 60000, 250000], np.uint32)
    T, start = 600_000, 12_345
    ref = oracle.boxes(el, dt, T, 1e-3, 2.0, start=start)
    for rule in (1, 2):
        b = oracle.boxes(el, dt, T, 1e-3, 2.0, start=start, rule=rule)
        assert np.array_equal(b.t0, ref.t0) and np.array_equal(b.t1, ref.t1)
        assert np.array_equal(b.obj, ref.obj)
        for k in rng.choice(len(b), 40, replace=False):
            i = b.obj[k]
            ta = (start + int(b.t0[k])) * 1e-3
            tb = (start + min(int(b.t1[k]), T)) * 1e-3
            lo, hi = oracle.box_interval(el[i], ta, tb, 2.0, rule)
            assert np.array_equal(lo, b.lo[k]) and np.array_equal(hi, b.hi[k])
    with pytest.raises(ValueError):
        oracle.boxes(el, dt, T, 1e-3, 2.0, rule=3)
