"""Seeded synthetic catalogs (inputs only).

This module produces orbital-element catalogs and run parameters for the
broad phase; both the HIP path and the CPU oracle read its output.  It holds
none of the broad phase's arithmetic: no propagation, no boxes, no overlap
tests.  The space-track catalog the paper evaluates on (Sec. 7.2) is not
available, so these seeded catalogs stand in for it, shaped like the tracked
population: clustered in LEO, with MEO and a GEO ring.

Elements are rows ``[a km, e, i rad, raan rad, argp rad, m0 rad]`` where m0 is
the mean anomaly at t = 0.  Time is counted in integer ticks of ``tick_s``
seconds (1 ms by default).  Random numbers come from numpy's PCG64
(``default_rng(seed)``), drawn per class in the order a, e, i, raan, argp, m0.

Fragment clouds (the projected-debris catalog) are also built in element
space: each fragment takes its parent's elements changed by the first-order
effect of a small impulse on a near-circular orbit (Gauss's variational
equations), and its phase drifts at its own mean motion from the breakup
epoch to t = 0.

Planted conjunctions are built in element space only.  Two objects share a,
e, raan and argp but sit in planes of different inclination, so both orbits
pass through the same point on the common line of nodes.  Their mean anomaly
at t = 0 is chosen so that both reach the ascending node at the planted time
t_c, one of them offset along track by a small fraction of the threshold.
"""
import math
from dataclasses import dataclass, field

import numpy as np

MU_EARTH = 398600.4418     # km^3 / s^2
TICK_S = 1e-3              # seconds per tick
TWO_PI = 2.0 * math.pi
DEG = math.pi / 180.0


@dataclass
class Scenario:
    name: str
    elements: np.ndarray          # [n, 6] float64
    dt_ticks: object              # int (uniform step), np.ndarray[n] uint32, or None
                                  # (the step is chosen per object by a rule)
    horizon_ticks: int            # T
    threshold_km: float           # thr = 2 r
    tick_s: float = TICK_S
    mu: float = MU_EARTH
    planted: list = field(default_factory=list)   # [(i, j, t_c ticks)]

    @property
    def n(self):
        return int(self.elements.shape[0])

    @property
    def uniform_dt(self):
        return self.dt_ticks is not None and (np.isscalar(self.dt_ticks)
                                              or np.ndim(self.dt_ticks) == 0)


def _draw(rng, n, a_lo, a_hi, e_lo, e_hi, i_lo, i_hi, a_normal=None):
    """One class of objects; a is uniform unless a_normal=(mean, sd)."""
    if a_normal is None:
        a = rng.uniform(a_lo, a_hi, n)
    else:
        a = rng.normal(a_normal[0], a_normal[1], n)
    e = rng.uniform(e_lo, e_hi, n)
    inc = rng.uniform(i_lo, i_hi, n)
    raan = rng.uniform(0.0, TWO_PI, n)
    argp = rng.uniform(0.0, TWO_PI, n)
    m0 = rng.uniform(0.0, TWO_PI, n)
    return np.stack([a, e, inc, raan, argp, m0], axis=1)


def leo_mix(rng, n):
    """The 10-minute test population: a ~ U[6778, 8378] km, e ~ U[0, 0.02]."""
    return _draw(rng, n, 6778.0, 8378.0, 0.0, 0.02, 0.0, math.pi)


def tracked_population(rng, n=16848):
    """75 % LEO, 10 % MEO, 15 % GEO (counts rounded, LEO takes the rest)."""
    n_meo = int(round(0.10 * n))
    n_geo = int(round(0.15 * n))
    n_leo = n - n_meo - n_geo
    leo = _draw(rng, n_leo, 6578.0, 8378.0, 0.0, 0.05, 0.0, math.pi)
    meo = _draw(rng, n_meo, 20000.0, 30000.0, 0.0, 0.3, 0.0, math.pi)
    geo = _draw(rng, n_geo, 0.0, 0.0, 0.0, 0.01, 0.0, 15.0 * DEG,
                a_normal=(42164.0, 50.0))
    return np.concatenate([leo, meo, geo], axis=0)


def _mean_anomaly_at_true(nu, e):
    """Mean anomaly of true anomaly nu (closed form, the inverse direction of
    Kepler's equation; used only to place planted objects)."""
    E = 2.0 * math.atan2(math.sqrt(1.0 - e) * math.sin(0.5 * nu),
                         math.sqrt(1.0 + e) * math.cos(0.5 * nu))
    return E - e * math.sin(E)


def plant_conjunctions(rng, elements, count, horizon_ticks, dt_ticks, thr_km,
                       tick_s=TICK_S, mu=MU_EARTH, a_range=(6778.0, 8378.0),
                       e_range=(0.0, 0.02)):
    """Overwrite the last 2*count rows with `count` conjunction pairs.

    Returns [(i, j, t_c)] with t_c in ticks.  Planted times cycle through a
    step boundary, the middle of a step, the horizon T itself and t = 0.
    """
    n = elements.shape[0]
    if 2 * count > n:
        raise ValueError("not enough objects to plant into")
    out = []
    step = int(dt_ticks) if np.ndim(dt_ticks) == 0 else int(np.max(dt_ticks))
    for p in range(count):
        i, j = n - 2 * count + 2 * p, n - 2 * count + 2 * p + 1
        a = rng.uniform(*a_range)
        e = rng.uniform(*e_range)
        raan = rng.uniform(0.0, TWO_PI)
        argp = rng.uniform(0.0, TWO_PI)
        inc_a = rng.uniform(0.0, math.pi)
        inc_b = (inc_a + rng.uniform(20.0, 160.0) * DEG) % math.pi
        kind = p % 4
        if kind == 0:       # on a step boundary
            t_c = int(rng.integers(0, max(1, horizon_ticks // max(step, 1)) + 1)) * step
        elif kind == 1:     # middle of a step
            t_c = int(rng.integers(0, max(1, horizon_ticks // max(step, 1)))) * step + step // 2
        elif kind == 2:     # the horizon itself
            t_c = horizon_ticks
        else:               # initially in conjunction
            t_c = 0
        t_c = int(min(max(t_c, 0), horizon_ticks))
        # ascending node: argument of latitude 0, true anomaly -argp
        m_node = _mean_anomaly_at_true(-argp, e)
        n_mean = math.sqrt(mu / a ** 3)
        m0 = (m_node - n_mean * t_c * tick_s) % TWO_PI
        # along-track offset of the partner, at most 0.3 thr
        dm = rng.uniform(-0.3, 0.3) * thr_km / a
        elements[i] = [a, e, inc_a, raan, argp, m0]
        elements[j] = [a, e, inc_b, raan, argp, (m0 + dm) % TWO_PI]
        out.append((i, j, t_c))
    return out


# ---- the workloads ---------------------------------------------------------

def small_leo(seed=1001, n=1000, planted=16):
    """n = 1000 LEO objects, 10-minute horizon, dt = 10 s, threshold 1 km."""
    rng = np.random.default_rng(seed)
    el = leo_mix(rng, n)
    T, dt, thr = 600_000, 10_000, 1.0
    pl = plant_conjunctions(rng, el, planted, T, dt, thr) if planted else []
    return Scenario("leo1000_600s_dt10s", el, dt, T, thr, planted=pl)


def tracked_hour(seed=2001, n=16848, planted=16):
    """n = 16848 tracked-population catalog, 1-hour horizon, dt = 1 s."""
    rng = np.random.default_rng(seed)
    el = tracked_population(rng, n)
    T, dt, thr = 3_600_000, 1_000, 1.0
    pl = plant_conjunctions(rng, el, planted, T, dt, thr) if planted else []
    return Scenario("tracked16848_1h_dt1s", el, dt, T, thr, planted=pl)


def scaled(sc, n=None, horizon_ticks=None, dt_ticks=None):
    """Same recipe with a smaller n / horizon / step (parity-sized cases).
    Keeps the first n rows and any planted pair that survives the cut."""
    el = sc.elements if n is None else sc.elements[:n].copy()
    T = sc.horizon_ticks if horizon_ticks is None else int(horizon_ticks)
    dt = sc.dt_ticks if dt_ticks is None else dt_ticks
    pl = [(i, j, t) for (i, j, t) in sc.planted if j < el.shape[0] and t <= T]
    return Scenario(sc.name + "_cut", el, dt, T, sc.threshold_km, sc.tick_s, sc.mu, pl)


def batch_sizes(seed=4000, count=64, lo=2000, hi=50000):
    """Scenario sizes n ~ logU[lo, hi] (the log drawn uniformly, n rounded)."""
    rng = np.random.default_rng(seed)
    return [int(round(math.exp(x))) for x in rng.uniform(math.log(lo), math.log(hi), count)]


def batch_member(s, n, seed_base=4001):
    """Scenario s of the uneven batch: n LEO objects, 30-minute horizon, dt = 1 s."""
    rng = np.random.default_rng(seed_base + s)
    return Scenario(f"batch{s}_n{n}", leo_mix(rng, n), 1_000, 1_800_000, 1.0)


def fragment_clouds(rng, parents, per_parent, dv_sigma_kms, age_range_s, mu=MU_EARTH):
    """Fragments of impulsive breakups of near-circular parents.

    For each parent (a row of elements) and each fragment: an impulse with
    radial, along-track and normal parts R, S, W ~ N(0, dv_sigma^2); the
    breakup happened `age` seconds before t = 0, age ~ U[age_range], at the
    parent's argument of latitude u_b at that epoch.  With v = sqrt(mu / a)
    the first-order element changes of a circular orbit are
        da = 2 a S / v,
        d(e cos w) = (R sin u_b + 2 S cos u_b) / v,
        d(e sin w) = (-R cos u_b + 2 S sin u_b) / v,
        di = W cos u_b / v,   draan = W sin u_b / (v sin i),
    and the fragment's mean argument of latitude at t = 0 is
    u_b + n_frag * age.  Returns [len(parents) * per_parent, 6].
    """
    out = []
    for par in parents:
        a, e, inc, raan, argp, m0 = (float(v) for v in par)
        n_par = math.sqrt(mu / a ** 3)
        v = math.sqrt(mu / a)
        age = rng.uniform(age_range_s[0], age_range_s[1])
        u_b = (argp + m0 - n_par * age) % TWO_PI
        R, S, W = (rng.normal(0.0, dv_sigma_kms, per_parent) for _ in range(3))
        su, cu = math.sin(u_b), math.cos(u_b)
        fa = a + 2.0 * a * S / v
        ex = e * math.cos(argp) + (R * su + 2.0 * S * cu) / v
        ey = e * math.sin(argp) + (-R * cu + 2.0 * S * su) / v
        fe = np.minimum(np.hypot(ex, ey), 0.9)
        fw = np.arctan2(ey, ex) % TWO_PI
        fi = np.clip(inc + W * cu / v, 0.0, math.pi)
        fO = (raan + W * su / (v * max(math.sin(inc), 1e-3))) % TWO_PI
        n_frag = np.sqrt(mu / fa ** 3)
        fm = (u_b + n_frag * age - fw) % TWO_PI
        out.append(np.stack([fa, fe, fi, fO, fw, fm], axis=1))
    return np.concatenate(out, axis=0) if out else np.zeros((0, 6))


def projected_debris(seed=5001, n=100_000, fragment_share=0.2, parents=50,
                     horizon_ticks=21_600_000, planted=16, dv_sigma_kms=0.05,
                     age_days=(1.0, 30.0)):
    """Projected-debris catalog: (1 - fragment_share) n objects of the
    10-minute test population plus fragment clouds of `parents` breakups
    (parents drawn among those objects, an equal share of fragments each,
    impulses N(0, 50 m/s) per axis, breakups 1-30 days before t = 0).
    Threshold 1 km; the step is chosen per object (dt_ticks None)."""
    rng = np.random.default_rng(seed)
    per = int(round(n * fragment_share / parents)) if parents else 0
    n_base = n - per * parents
    base = leo_mix(rng, n_base)
    pidx = rng.choice(n_base, size=parents, replace=False) if parents else []
    frag = fragment_clouds(rng, base[pidx], per, dv_sigma_kms,
                           (age_days[0] * 86400.0, age_days[1] * 86400.0))
    el = np.concatenate([base, frag], axis=0)
    # planted pairs replace rows of the base population (fragments stay whole)
    pl = []
    if planted:
        head = el[:n_base]
        pl = plant_conjunctions(rng, head, planted, horizon_ticks, 1_000, 1.0)
        el[:n_base] = head
    hours = horizon_ticks / 3_600_000
    name = f"debris{n}_{hours:g}h" if hours >= 1 else f"debris{n}_{horizon_ticks // 1000}s"
    return Scenario(name, el, None, int(horizon_ticks), 1.0, planted=pl)


def random_boxes(seed, N, n_obj, extent=100.0, size=5.0, T=100, max_len=10,
                 kind="uniform"):
    """Box soups for box-level tests (caller-built boxes): lo/hi [N,3] float64,
    t0/t1/obj uint32.  kinds: uniform, identical, disjoint, line, huge."""
    rng = np.random.default_rng(seed)
    if kind == "identical":
        c = np.zeros((N, 3))
        h = np.full((N, 3), size)
    elif kind == "disjoint":
        c = np.stack([np.arange(N) * (4.0 * size), np.zeros(N), np.zeros(N)], 1)
        h = np.full((N, 3), size)
    elif kind == "line":
        c = np.stack([np.arange(N) * size * 1.5, np.zeros(N), np.zeros(N)], 1)
        h = np.full((N, 3), size)
    else:
        c = rng.uniform(-extent, extent, (N, 3))
        h = rng.uniform(0.1 * size, size, (N, 3))
    if kind == "huge" and N > 0:
        c[0] = 0.0
        h[0] = 10.0 * extent
    lo = c - h
    hi = c + h
    t0 = rng.integers(0, T, N).astype(np.uint32)
    t1 = (t0 + rng.integers(1, max_len + 1, N)).astype(np.uint32)
    obj = rng.integers(0, max(n_obj, 1), N).astype(np.uint32)
    return lo, hi, t0, t1, obj
