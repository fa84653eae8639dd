"""CPU oracle for the 4D-AABB broad phase -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never links,
loads or calls it; it shares no code with the HIP path.

The arithmetic lives in plain C (``cd_oracle.c``, FP64), reached here through
ctypes with numpy arrays.  See ``cd_oracle.c`` for the passages of Bak & Hobbs
that each function follows and for the readings taken where the paper is
silent.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_u32p = ctypes.POINTER(ctypes.c_uint32)
_u32pp = ctypes.POINTER(_u32p)
_dp = ctypes.c_void_p


class _Iv(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_double), ("hi", ctypes.c_double)]


def build(verbose=False):
    """Compile the oracle (gcc, -O2, OpenMP; no fast-math, no FMA contraction)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC",
           "-shared", _SRC, "-o", _LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        L.or_eccentric_anomaly.restype = ctypes.c_double
        L.or_eccentric_anomaly.argtypes = [ctypes.c_double, ctypes.c_double]
        L.or_true_anomaly.restype = ctypes.c_double
        L.or_true_anomaly.argtypes = [_dp, ctypes.c_double, ctypes.c_double]
        L.or_position_from_nu.restype = None
        L.or_position_from_nu.argtypes = [_dp, ctypes.c_double, _dp]
        L.or_position.restype = None
        L.or_position.argtypes = [_dp, ctypes.c_double, ctypes.c_double, _dp]
        L.or_vmax.restype = ctypes.c_double
        L.or_vmax.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.or_intervals.restype = ctypes.c_uint64
        L.or_intervals.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        L.or_box_count.restype = ctypes.c_int64
        L.or_box_count.argtypes = [ctypes.c_int64, _dp, ctypes.c_uint32]
        L.or_boxes.restype = ctypes.c_int
        L.or_boxes.argtypes = [ctypes.c_int64, _dp, _dp, ctypes.c_uint32, ctypes.c_uint32,
                               ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                               _dp, _dp, _dp, _dp, _dp]
        for nm in ("add", "sub", "mul", "div"):
            f = getattr(L, "or_iv_" + nm)
            f.restype = _Iv
            f.argtypes = [_Iv, _Iv]
        for nm in ("sqr", "cos", "sin"):
            f = getattr(L, "or_iv_" + nm)
            f.restype = _Iv
            f.argtypes = [_Iv]
        L.or_box_interval.restype = None
        L.or_box_interval.argtypes = [_dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_int, _dp, _dp]
        L.or_pairs.restype = ctypes.c_int64
        L.or_pairs.argtypes = [ctypes.c_int64, _dp, _dp, _dp, _dp, _dp, _u32pp]
        L.or_pairs_bucketed.restype = ctypes.c_int64
        L.or_pairs_bucketed.argtypes = [ctypes.c_int64, _dp, _dp, _dp, _dp, _dp, _u32pp]
        L.or_pairs_of.restype = ctypes.c_int64
        L.or_pairs_of.argtypes = [ctypes.c_int64, _dp, _dp, _dp, _dp, _dp,
                                  ctypes.c_int64, _dp, _u32pp]
        L.or_time_overlapping_pairs.restype = ctypes.c_int64
        L.or_time_overlapping_pairs.argtypes = [ctypes.c_int64, _dp, _dp, _dp]
        L.or_brute_force.restype = ctypes.c_int64
        L.or_brute_force.argtypes = [ctypes.c_int64, _dp, _dp, ctypes.c_uint32,
                                     ctypes.c_uint32, ctypes.c_double,
                                     ctypes.c_double, _u32pp]
        L.or_round_down_f32.restype = ctypes.c_float
        L.or_round_down_f32.argtypes = [ctypes.c_double]
        L.or_round_up_f32.restype = ctypes.c_float
        L.or_round_up_f32.argtypes = [ctypes.c_double]
        L.or_outward_f32.restype = None
        L.or_outward_f32.argtypes = [ctypes.c_int64, _dp, _dp, _dp, _dp]
        L.or_dt_heuristic.restype = None
        L.or_dt_heuristic.argtypes = [ctypes.c_int64, _dp, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double,
                                      ctypes.c_uint32, _dp]
        L.or_refine.restype = ctypes.c_int64
        L.or_refine.argtypes = [ctypes.c_int64, _dp, ctypes.c_uint32, ctypes.c_uint32,
                                ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int64, _dp, _u32pp]
        L.or_band.restype = None
        L.or_band.argtypes = [_dp, ctypes.c_double, _dp, _dp]
        L.or_band_compatible.restype = ctypes.c_int
        L.or_band_compatible.argtypes = [_dp, _dp, ctypes.c_double]
        L.or_band_filter.restype = ctypes.c_int64
        L.or_band_filter.argtypes = [ctypes.c_int64, _dp, ctypes.c_double, ctypes.c_int64, _dp,
                                     _u32pp]
        L.or_band_partition.restype = ctypes.c_int64
        L.or_band_partition.argtypes = [ctypes.c_int64, _dp, ctypes.c_double, ctypes.c_int,
                                        _dp, _dp, _dp]
        L.or_free.restype = None
        L.or_free.argtypes = [ctypes.c_void_p]
        L.or_num_threads.restype = ctypes.c_int
        L.or_num_threads.argtypes = []
        L.or_set_num_threads.restype = None
        L.or_set_num_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


MU_EARTH = 398600.4418  # km^3 / s^2 (the paper names mu but gives no value)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def eccentric_anomaly(M, e):
    return lib().or_eccentric_anomaly(float(M), float(e))


def true_anomaly(el, t_s, mu=MU_EARTH):
    el = _c(el, np.float64)
    return lib().or_true_anomaly(_ptr(el), float(t_s), float(mu))


def position_from_nu(el, nu):
    el = _c(el, np.float64)
    out = np.zeros(3)
    lib().or_position_from_nu(_ptr(el), float(nu), _ptr(out))
    return out


def position(el, t_s, mu=MU_EARTH):
    el = _c(el, np.float64)
    out = np.zeros(3)
    lib().or_position(_ptr(el), float(t_s), float(mu), _ptr(out))
    return out


def positions(elements, t_s, mu=MU_EARTH):
    """Positions of all objects [n,6] at one time: [n,3]."""
    elements = _c(elements, np.float64)
    return np.stack([position(elements[i], t_s, mu) for i in range(len(elements))]) \
        if len(elements) else np.zeros((0, 3))


def vmax(a, e, mu=MU_EARTH):
    return lib().or_vmax(float(a), float(e), float(mu))


def intervals(dt, T):
    return int(lib().or_intervals(int(dt), int(T)))


class Boxes:
    """Object-major FP64 boxes: lo/hi [N,3], t0/t1/obj [N] uint32."""

    def __init__(self, lo, hi, t0, t1, obj):
        self.lo, self.hi, self.t0, self.t1, self.obj = lo, hi, t0, t1, obj

    def __len__(self):
        return len(self.t0)

    def take(self, idx):
        return Boxes(self.lo[idx], self.hi[idx], self.t0[idx], self.t1[idx], self.obj[idx])


BOX_SPEED, BOX_INTERVAL_NU, BOX_INTERVAL_E = 0, 1, 2


def boxes(elements, dt, T, tick_s, thr_km, mu=MU_EARTH, start=0, rule=BOX_SPEED):
    """Boxes over absolute ticks [start, start + T], tags relative to start.
    rule: BOX_SPEED (endpoint hull + vmax growth) or an interval evaluation
    over the true (BOX_INTERVAL_NU) or eccentric (BOX_INTERVAL_E) anomaly."""
    el = _c(elements, np.float64).reshape(-1, 6)
    n = len(el)
    dt = _c(np.broadcast_to(np.asarray(dt, dtype=np.uint32), (n,)), np.uint32)
    N = lib().or_box_count(n, _ptr(dt), int(T))
    if N < 0:
        raise ValueError("dt must be >= 1 tick")
    lo = np.zeros((N, 3))
    hi = np.zeros((N, 3))
    t0 = np.zeros(N, np.uint32)
    t1 = np.zeros(N, np.uint32)
    obj = np.zeros(N, np.uint32)
    rc = lib().or_boxes(n, _ptr(el), _ptr(dt), int(T), int(start), float(tick_s), float(mu),
                        float(thr_km), int(rule), _ptr(lo), _ptr(hi), _ptr(t0), _ptr(t1),
                        _ptr(obj))
    if rc != 0:
        raise ValueError("invalid box parameters")
    return Boxes(lo, hi, t0, t1, obj)


def iv(lo, hi=None):
    return _Iv(float(lo), float(lo if hi is None else hi))


def iv_op(name, *args):
    """Interval operation or_iv_<name> on (lo, hi) pairs; returns (lo, hi)."""
    r = getattr(lib(), "or_iv_" + name)(*[iv(*a) for a in args])
    return (r.lo, r.hi)


def box_interval(el, ta_s, tb_s, thr_km, var, mu=MU_EARTH):
    """occ-int of one object over [ta_s, tb_s] by interval evaluation over the
    true (var=1) or eccentric (var=2) anomaly: (lo[3], hi[3])."""
    el = _c(el, np.float64)
    lo = np.zeros(3)
    hi = np.zeros(3)
    lib().or_box_interval(_ptr(el), float(ta_s), float(tb_s), float(mu), float(thr_km),
                          int(var), _ptr(lo), _ptr(hi))
    return lo, hi


def _take_records(n, ptr, width):
    if n > 0:
        arr = np.ctypeslib.as_array(ptr, shape=(n * width,)).reshape(n, width).copy()
    else:
        arr = np.zeros((0, width), np.uint32)
    lib().or_free(ctypes.cast(ptr, ctypes.c_void_p))
    return arr


def _box_args(b):
    lo = _c(b.lo, np.float64)
    hi = _c(b.hi, np.float64)
    t0 = _c(b.t0, np.uint32)
    t1 = _c(b.t1, np.uint32)
    obj = _c(b.obj, np.uint32)
    return (lo, hi, t0, t1, obj)


def pairs(b):
    """Canonical record set [P,4] uint32 of all overlapping box pairs (literal)."""
    arrs = _box_args(b)
    out = _u32p()
    n = lib().or_pairs(len(b.t0), *[_ptr(x) for x in arrs], ctypes.byref(out))
    return _take_records(n, out, 4)


def pairs_bucketed(b):
    """The same canonical set as pairs(b), testing only box pairs whose time
    tags overlap (a t0-ordered sweep with a t1-ordered active list; with a
    uniform step, all pairs within each time slab)."""
    arrs = _box_args(b)
    out = _u32p()
    n = lib().or_pairs_bucketed(len(b.t0), *[_ptr(x) for x in arrs], ctypes.byref(out))
    return _take_records(n, out, 4)


def window(b, ta, tb):
    """The boxes whose time tags meet the ticks [ta, tb).  Two time intervals
    that meet each other and both meet [ta, tb) have a common point inside it
    (intervals on a line), so pairs(window(b, ta, tb)) is exactly the records
    of pairs(b) whose [t_lo, t_hi) meets [ta, tb)."""
    keep = np.nonzero((b.t0 < tb) & (b.t1 > ta))[0]
    return b.take(keep)


def records_in_window(rec, ta, tb):
    """Rows of a record list whose [t_lo, t_hi) meets the ticks [ta, tb)."""
    rec = np.asarray(rec).reshape(-1, 4)
    return rec[(rec[:, 2] < tb) & (rec[:, 3] > ta)]


def pairs_of(b, sample):
    """Canonical records that involve at least one sampled box."""
    arrs = _box_args(b)
    s = _c(sample, np.int64)
    out = _u32p()
    n = lib().or_pairs_of(len(b.t0), *[_ptr(x) for x in arrs], len(s), _ptr(s),
                          ctypes.byref(out))
    return _take_records(n, out, 4)


def time_overlapping_pairs(b):
    t0 = _c(b.t0, np.uint32)
    t1 = _c(b.t1, np.uint32)
    obj = _c(b.obj, np.uint32)
    return int(lib().or_time_overlapping_pairs(len(t0), _ptr(t0), _ptr(t1), _ptr(obj)))


def brute_force(elements, r, T, delta, tick_s, mu=MU_EARTH):
    """All witnesses [W,3] (t, i, j) of Alg. Brute Force; row 0 is its answer."""
    el = _c(elements, np.float64).reshape(-1, 6)
    n = len(el)
    rr = _c(np.broadcast_to(np.asarray(r, dtype=np.float64), (n,)), np.float64)
    out = _u32p()
    w = lib().or_brute_force(n, _ptr(el), _ptr(rr), int(T), int(delta), float(tick_s),
                             float(mu), ctypes.byref(out))
    return _take_records(w, out, 3)


def refine(elements, records, T, tick_s, thr_km, delta, min_steps=1, rule=BOX_SPEED,
           mu=MU_EARTH, start=0):
    """Bulk interval refinement of candidate records [R,4] (i, j, t_lo, t_hi):
    the canonical leaves [L,4] (i, j, first instant, last instant + 1)."""
    el = _c(elements, np.float64).reshape(-1, 6)
    rec = _c(np.asarray(records, dtype=np.uint32).reshape(-1, 4), np.uint32)
    out = _u32p()
    m = lib().or_refine(len(el), _ptr(el), int(T), int(start), float(tick_s), float(mu),
                        float(thr_km), int(rule), int(delta), int(min_steps), len(rec),
                        _ptr(rec), ctypes.byref(out))
    if m < 0:
        raise ValueError("invalid refinement arguments")
    return _take_records(m, out, 4)


def band(el, thr_km):
    """Radial band [lo, hi] of one object (perigee/apogee widened by sqrt(3) r)."""
    el = _c(el, np.float64)
    lo, hi = ctypes.c_double(0), ctypes.c_double(0)
    lib().or_band(_ptr(el), float(thr_km), ctypes.byref(lo), ctypes.byref(hi))
    return lo.value, hi.value


def band_compatible(el_i, el_j, thr_km):
    a = _c(el_i, np.float64)
    b = _c(el_j, np.float64)
    return bool(lib().or_band_compatible(_ptr(a), _ptr(b), float(thr_km)))


def band_filter(elements, records, thr_km):
    el = _c(elements, np.float64).reshape(-1, 6)
    rec = _c(np.asarray(records, dtype=np.uint32).reshape(-1, 4), np.uint32)
    out = _u32p()
    m = lib().or_band_filter(len(el), _ptr(el), float(thr_km), len(rec), _ptr(rec),
                             ctypes.byref(out))
    return _take_records(m, out, 4)


def band_partition(elements, thr_km, p):
    """(edges [p+1], per-band object id arrays) of the altitude-band edge partition."""
    el = _c(elements, np.float64).reshape(-1, 6)
    edges = np.zeros(p + 1)
    count = np.zeros(p, np.int64)
    total = lib().or_band_partition(len(el), _ptr(el), float(thr_km), int(p), _ptr(edges),
                                    _ptr(count), None)
    if total < 0:
        raise ValueError("p must be >= 1")
    members = np.zeros(max(total, 1), np.uint32)
    lib().or_band_partition(len(el), _ptr(el), float(thr_km), int(p), _ptr(edges),
                            _ptr(count), _ptr(members))
    off = np.concatenate([[0], np.cumsum(count)])
    return edges, [members[off[k]:off[k + 1]] for k in range(p)]


def round_down_f32(x):
    return np.float32(lib().or_round_down_f32(float(x)))


def round_up_f32(x):
    return np.float32(lib().or_round_up_f32(float(x)))


def outward_f32(b):
    """FP64 boxes rounded outward to FP32 (returned as exact float64 values)."""
    lo = _c(b.lo, np.float64)
    hi = _c(b.hi, np.float64)
    lo32 = np.zeros(lo.shape, np.float32)
    hi32 = np.zeros(hi.shape, np.float32)
    lib().or_outward_f32(lo.size, _ptr(lo), _ptr(hi), _ptr(lo32), _ptr(hi32))
    return Boxes(lo32.astype(np.float64), hi32.astype(np.float64), b.t0.copy(),
                 b.t1.copy(), b.obj.copy())


def dt_heuristic(elements, tick_s, max_disp_km, T, mu=MU_EARTH):
    el = _c(elements, np.float64).reshape(-1, 6)
    out = np.zeros(len(el), np.uint32)
    lib().or_dt_heuristic(len(el), _ptr(el), float(mu), float(tick_s),
                          float(max_disp_km), int(T), _ptr(out))
    return out


def num_threads():
    return int(lib().or_num_threads())


def set_num_threads(n):
    """OpenMP threads of later oracle calls."""
    lib().or_set_num_threads(int(n))
