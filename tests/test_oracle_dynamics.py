"""Pins for the oracle's dynamics: g(t) = nu(t) and h(nu) (Sec. 4.5, 7.1).

Each check compares the oracle with something other than itself: closed forms,
orbital invariants, an independent bisection solve, the paper's own ODE
(Eq. nu-dot) integrated numerically, and the figures the paper prints.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle

MU = oracle.MU_EARTH
GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_figures.json")


def _rand_elements(rng, k, a=(6578.0, 42000.0), e=(0.0, 0.3)):
    return np.stack([rng.uniform(*a, k), rng.uniform(*e, k), rng.uniform(0, math.pi, k),
                     rng.uniform(0, 2 * math.pi, k), rng.uniform(0, 2 * math.pi, k),
                     rng.uniform(0, 2 * math.pi, k)], 1)


def _bisect_kepler(M, e):
    lo, hi = M - 1.0, M + 1.0       # |E - M| <= e < 1
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid - e * math.sin(mid) - M < 0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def test_kepler_special_cases():
    # e = 0: E = M exactly; M in {0, pi}: E = M for every e
    for M in np.linspace(0, 2 * math.pi, 17):
        assert oracle.eccentric_anomaly(M, 0.0) == M
    for e in (0.0, 0.1, 0.3, 0.7, 0.95):
        assert oracle.eccentric_anomaly(0.0, e) == 0.0
        assert abs(oracle.eccentric_anomaly(math.pi, e) - math.pi) < 1e-15


def test_kepler_residual_and_bisection():
    rng = np.random.default_rng(7)
    for _ in range(2000):
        M = rng.uniform(0, 2 * math.pi)
        e = rng.uniform(0, 0.95)
        E = oracle.eccentric_anomaly(M, e)
        assert abs(E - e * math.sin(E) - M) <= 1e-15 * (1 + abs(M)) * 4
        assert abs(E - _bisect_kepler(M, e)) <= 1e-12


def test_circular_equatorial_closed_form():
    rng = np.random.default_rng(3)
    for _ in range(50):
        a = rng.uniform(6578, 42164)
        m0 = rng.uniform(0, 2 * math.pi)
        el = [a, 0.0, 0.0, 0.0, 0.0, m0]
        n = math.sqrt(MU / a ** 3)
        for t in (0.0, 1.0, 137.25, 3600.0, 21600.0):
            th = m0 + n * t
            want = np.array([a * math.cos(th), a * math.sin(th), 0.0])
            got = oracle.position(el, t)
            assert np.max(np.abs(got - want)) <= 1e-9 * a


def test_radius_is_orbit_equation():
    rng = np.random.default_rng(11)
    els = _rand_elements(rng, 200)
    for el in els:
        a, e = el[0], el[1]
        for t in rng.uniform(0, 20000, 5):
            p = oracle.position(el, t)
            r = np.linalg.norm(p)
            assert a * (1 - e) * (1 - 1e-13) <= r <= a * (1 + e) * (1 + 1e-13)
            M = (el[5] + math.sqrt(MU / a ** 3) * t) % (2 * math.pi)
            E = _bisect_kepler(M, e)
            assert abs(r - a * (1 - e * math.cos(E))) <= 1e-9 * a


def test_orbit_normal_and_node_and_perigee():
    """Plane orientation pins i and Omega; perigee direction pins omega."""
    rng = np.random.default_rng(5)
    els = _rand_elements(rng, 100, e=(0.01, 0.3))
    for el in els:
        a, e, inc, raan, argp, _ = el
        el0 = el.copy()
        el0[5] = 0.0                        # at perigee at t = 0
        p1 = oracle.position(el0, 0.0)
        p2 = oracle.position(el0, 60.0)
        h = np.cross(p1, p2)
        h /= np.linalg.norm(h)
        want = np.array([math.sin(raan) * math.sin(inc), -math.cos(raan) * math.sin(inc),
                         math.cos(inc)])
        assert np.max(np.abs(h - want)) < 1e-10
        rp = a * (1 - e)
        node = np.array([math.cos(raan), math.sin(raan), 0.0])
        assert abs(np.linalg.norm(p1) - rp) < 1e-9 * a
        assert abs(p1 @ node - rp * math.cos(argp)) < 1e-9 * a
        assert abs(p1[2] - rp * math.sin(argp) * math.sin(inc)) < 1e-9 * a


def test_nudot_equation_finite_difference():
    """The propagated path obeys the paper's ODE for the true anomaly."""
    rng = np.random.default_rng(13)
    els = _rand_elements(rng, 60)
    hstep = 0.05
    for el in els:
        a, e = el[0], el[1]
        p_ = a * (1 - e * e)
        for t in rng.uniform(10, 20000, 4):
            pm = oracle.position(el, t - hstep)
            pp = oracle.position(el, t + hstep)
            p0 = oracle.position(el, t)
            swept = math.atan2(np.linalg.norm(np.cross(pm, pp)), pm @ pp)
            nudot_fd = swept / (2 * hstep)
            one_plus_ecos = p_ / np.linalg.norm(p0)
            nudot_eq = math.sqrt(MU / p_ ** 3) * one_plus_ecos ** 2
            assert abs(nudot_fd - nudot_eq) <= 1e-7 * nudot_eq


def test_nudot_equation_runge_kutta():
    """Integrating Eq. (nu-dot) by RK4, as the paper's simulation would,
    reaches the oracle's closed-form nu(t)."""
    rng = np.random.default_rng(17)
    els = _rand_elements(rng, 12)
    for el in els:
        a, e = el[0], el[1]
        k = math.sqrt(MU / (a * (1 - e * e)) ** 3)

        def f(nu):
            return k * (1 + e * math.cos(nu)) ** 2
        nu = oracle.true_anomaly(el, 0.0)
        h, steps = 0.5, 1200
        for _ in range(steps):
            k1 = f(nu)
            k2 = f(nu + 0.5 * h * k1)
            k3 = f(nu + 0.5 * h * k2)
            k4 = f(nu + h * k3)
            nu += h * (k1 + 2 * k2 + 2 * k3 + k4) / 6
        want = oracle.true_anomaly(el, h * steps)
        d = (nu - want + math.pi) % (2 * math.pi) - math.pi
        assert abs(d) < 1e-9


def test_vis_viva_angular_momentum_and_vmax():
    rng = np.random.default_rng(19)
    els = _rand_elements(rng, 80)
    for el in els:
        a, e = el[0], el[1]
        vmax = oracle.vmax(a, e)
        assert abs(vmax - math.sqrt(MU * (2 / (a * (1 - e)) - 1 / a))) <= 1e-12 * vmax
        for t in rng.uniform(1, 20000, 4):
            hs = 1e-3
            pm, p0, pp = (oracle.position(el, t + d) for d in (-hs, 0.0, hs))
            v = (pp - pm) / (2 * hs)
            r = np.linalg.norm(p0)
            assert abs(v @ v - MU * (2 / r - 1 / a)) <= 1e-6 * (v @ v)
            hmag = np.linalg.norm(np.cross(p0, v))
            assert abs(hmag - math.sqrt(MU * a * (1 - e * e))) <= 1e-6 * hmag
            assert np.linalg.norm(v) <= vmax * (1 + 1e-6)
        el0 = el.copy()
        el0[5] = 0.0
        v_peri = (oracle.position(el0, 1e-3) - oracle.position(el0, -1e-3)) / 2e-3
        assert abs(np.linalg.norm(v_peri) - vmax) <= 1e-6 * vmax


def test_paper_leo_speed_and_step_displacement():
    g = json.load(open(GOLD))
    # low LEO circular orbit: speed and distance per delta as the paper states
    el = [6578.0, 0.0, 0.9, 0.3, 0.0, 0.2]
    d = g["leo_step_displacement"]["delta_s"]
    p0 = oracle.position(el, 100.0)
    p1 = oracle.position(el, 100.0 + 1.0)
    speed_m_s = np.linalg.norm(p1 - p0) * 1000.0
    assert abs(speed_m_s - g["leo_speed"]["speed_m_s"]) < 0.01 * g["leo_speed"]["speed_m_s"]
    step_m = np.linalg.norm(oracle.position(el, 100.0 + d) - p0) * 1000.0
    assert abs(step_m - g["leo_step_displacement"]["displacement_m"]) < 0.01


def test_planted_conjunction_meets_at_planted_time():
    """Planted pairs are built in element space only (common line of nodes,
    timed arrival); the oracle must place them within the threshold at t_c."""
    from paper_1901_10475_amd import catalog
    rng = np.random.default_rng(23)
    el = catalog.leo_mix(rng, 40)
    pl = catalog.plant_conjunctions(rng, el, 10, 600_000, 10_000, 1.0)
    for i, j, tc in pl:
        pi = oracle.position(el[i], tc * 1e-3)
        pj = oracle.position(el[j], tc * 1e-3)
        assert np.max(np.abs(pi - pj)) <= 0.5
        # and far apart a quarter orbit later (different planes)
        tq = tc * 1e-3 + 1500.0
        assert np.max(np.abs(oracle.position(el[i], tq) - oracle.position(el[j], tq))) > 50.0
