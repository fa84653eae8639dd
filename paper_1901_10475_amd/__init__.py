"""MI355X (gfx950) 4D-AABB broad phase for n-to-n orbital collision detection.

Python binding of the C ABI in ``include/cd4d.h`` (library ``libcd4d.so``,
hand-written HIP kernels).  This module only marshals arguments: PyTorch
supplies device memory and the current HIP stream, every step of the path runs
in the library's kernels, and there is no CPU fallback -- importing the module
without the built library raises.

The functions below keep the C names (``cd_build_boxes``, ``cd_build_tree``,
``cd_query_pairs``, ...).  ``BroadPhase`` holds one set of buffers and runs the
three steps in order for repeated queries.
"""
import contextlib
import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime the library binds to)

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libcd4d.so")
# the same library built with the traversal's executed-work counters
_COUNTERS_LIB_PATH = os.path.join(_HERE, "libcd4d_counters.so")

CD_OK, CD_E_INVALID, CD_E_WORKSPACE, CD_E_CAPACITY, CD_E_OVERFLOW, CD_E_DEVICE = range(6)
CD_FP64, CD_FP32 = 0, 1
CD_BOX_SPEED, CD_BOX_INTERVAL_NU, CD_BOX_INTERVAL_E = 0, 1, 2
CD_LAYOUT_OBJECT, CD_LAYOUT_SORTED = 0, 1
CD_SORTED_MAX_ARRAYS, CD_SORTED_MAX_RECORDS = 17408, 278528

_vp = ctypes.c_void_p


class cd_elements(ctypes.Structure):
    _fields_ = [("a", _vp), ("e", _vp), ("inc", _vp), ("raan", _vp), ("argp", _vp),
                ("m0", _vp), ("n", ctypes.c_int64)]


class cd_params(ctypes.Structure):
    _fields_ = [("tick_s", ctypes.c_double), ("mu", ctypes.c_double),
                ("threshold_km", ctypes.c_double), ("horizon_ticks", ctypes.c_uint32),
                ("dt_ticks", ctypes.c_uint32), ("start_ticks", ctypes.c_uint32),
                ("box_rule", ctypes.c_uint32)]


class cd_boxes(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int64), ("precision", ctypes.c_int), ("lo", _vp * 3),
                ("hi", _vp * 3), ("t0", _vp), ("t1", _vp), ("obj", _vp),
                ("slab_ticks", ctypes.c_uint32), ("slab_size", ctypes.c_int64),
                ("horizon_ticks", ctypes.c_uint32), ("obj_count", ctypes.c_uint32),
                ("code", _vp), ("code_valid", ctypes.c_int), ("layout", ctypes.c_int),
                ("records", _vp)]


class cd_tree(ctypes.Structure):
    _fields_ = [("mem", _vp), ("bytes", ctypes.c_size_t), ("count", ctypes.c_int64),
                ("precision", ctypes.c_int), ("slab_ticks", ctypes.c_uint32),
                ("horizon_ticks", ctypes.c_uint32), ("obj_count", ctypes.c_uint32)]


class cd_tuning(ctypes.Structure):
    _fields_ = [("expand_blocks", ctypes.c_uint32), ("expand_threads", ctypes.c_uint32),
                ("walk_threads", ctypes.c_uint32), ("mode", ctypes.c_uint32),
                ("max_levels", ctypes.c_uint32)]


class cd_counters(ctypes.Structure):
    _fields_ = [("tests", ctypes.c_uint64), ("leaf_tests", ctypes.c_uint64),
                ("mixed_tests", ctypes.c_uint64), ("leaf_hits", ctypes.c_uint64),
                ("pairs", ctypes.c_uint64), ("walk_steps", ctypes.c_uint64)]


class CDError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{_status_name(status)} ({status}): {message}")
        self.status = status


def _status_name(s):
    return {0: "CD_OK", 1: "CD_E_INVALID", 2: "CD_E_WORKSPACE", 3: "CD_E_CAPACITY",
            4: "CD_E_OVERFLOW", 5: "CD_E_DEVICE"}.get(s, "CD_E_?")


_libs = {}
_active = _LIB_PATH


def lib():
    """The loaded libcd4d.so (raises if it has not been built); inside
    ``counters_build()``, libcd4d_counters.so."""
    return _load(_active)


@contextlib.contextmanager
def counters_build():
    """Route the enclosed calls of this module through libcd4d_counters.so,
    the library built with CD_COUNTERS (same calls, same results, plus the
    executed-work counters of cd_counters_reset / cd_counters_read).  Launch
    shapes set with cd_set_tuning are per library."""
    global _active
    prev = _active
    _active = _COUNTERS_LIB_PATH
    try:
        yield lib()
    finally:
        _active = prev


def _load(path):
    if path not in _libs:
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with "
                              "`python -m paper_1901_10475_amd.build`")
        L = ctypes.CDLL(path)
        P = ctypes.POINTER
        i64, u32, sz, dbl = ctypes.c_int64, ctypes.c_uint32, ctypes.c_size_t, ctypes.c_double
        flt = ctypes.c_float
        sig = {
            "cd_status_string": (ctypes.c_char_p, [ctypes.c_int]),
            "cd_last_error": (ctypes.c_char_p, []),
            "cd_version": (ctypes.c_int, []),
            "cd_stream_copy": (ctypes.c_int, [_vp, _vp, sz, _vp]),
            "cd_profile_enable": (ctypes.c_int, [ctypes.c_int]),
            "cd_profile_read": (ctypes.c_int, [P(ctypes.c_char_p), P(dbl), P(i64), ctypes.c_int,
                                               ctypes.c_int]),
            "cd_box_count_ws": (sz, [i64]),
            "cd_box_count": (ctypes.c_int, [_vp, i64, P(cd_params), P(i64), _vp, sz, _vp]),
            "cd_validate_ws": (sz, [i64]),
            "cd_validate_elements": (ctypes.c_int, [P(cd_elements), P(i64), _vp, sz, _vp]),
            "cd_dt_heuristic": (ctypes.c_int, [P(cd_elements), P(cd_params), dbl, _vp, _vp]),
            "cd_build_boxes_ws": (sz, [i64]),
            "cd_build_boxes": (ctypes.c_int, [P(cd_elements), _vp, P(cd_params), P(cd_boxes),
                                              _vp, sz, _vp]),
            "cd_tree_bytes": (sz, [i64, ctypes.c_int]),
            "cd_tree_leaf_records": (_vp, [_vp, i64]),
            "cd_build_tree_ws": (sz, [i64]),
            "cd_build_tree": (ctypes.c_int, [P(cd_boxes), ctypes.c_int, u32, P(cd_tree), _vp,
                                             sz, _vp]),
            "cd_query_pairs_ws": (sz, [i64, i64]),
            "cd_query_pairs": (ctypes.c_int, [P(cd_tree), _vp, i64, P(i64), _vp, sz, _vp]),
            "cd_query_pairs_async": (ctypes.c_int, [P(cd_tree), _vp, i64, _vp, _vp, _vp, sz,
                                                    _vp]),
            "cd_noalloc_scratch_bytes": (sz, []),
            "cd_query_pairs_async_noalloc": (ctypes.c_int, [P(cd_tree), _vp, i64, _vp, _vp,
                                                            _vp]),
            "cd_set_tuning": (ctypes.c_int, [P(cd_tuning)]),
            "cd_get_tuning": (ctypes.c_int, [P(cd_tuning)]),
            "cd_graph_begin": (ctypes.c_int, [_vp]),
            "cd_graph_end": (ctypes.c_int, [_vp, P(_vp)]),
            "cd_graph_launch": (ctypes.c_int, [_vp, _vp]),
            "cd_graph_destroy": (ctypes.c_int, [_vp]),
            "cd_first_witness": (ctypes.c_int, [P(cd_elements), P(cd_params), u32, _vp, i64, _vp,
                                                _vp, _vp]),
            "cd_refine_records_ws": (sz, [i64, i64, i64]),
            "cd_band_filter_ws": (sz, [i64]),
            "cd_band_filter": (ctypes.c_int, [P(cd_elements), P(cd_params), _vp, i64, _vp,
                                              P(ctypes.c_int64), _vp, sz, _vp]),
            "cd_band_partition_ws": (sz, [i64, ctypes.c_int32]),
            "cd_band_partition": (ctypes.c_int, [P(cd_elements), P(cd_params), ctypes.c_int32,
                                                 _vp, _vp, _vp, i64, P(ctypes.c_int64), _vp,
                                                 sz, _vp]),
            "cd_gather_elements": (ctypes.c_int, [P(cd_elements), _vp, i64, _vp, _vp]),
            "cd_remap_records": (ctypes.c_int, [_vp, i64, _vp, i64, _vp, _vp]),
            "cd_canonical_records_ws": (sz, [i64]),
            "cd_canonical_records": (ctypes.c_int, [_vp, i64, u32, u32, _vp,
                                                    P(ctypes.c_int64), _vp, sz, _vp]),
            "cd_refine_records": (ctypes.c_int, [P(cd_elements), P(cd_params), u32, u32, _vp,
                                                 i64, _vp, i64, P(ctypes.c_int64), _vp, sz,
                                                 _vp]),
            "cd_mlp_features": (ctypes.c_int, [P(cd_elements), P(cd_params), _vp, _vp]),
            "cd_dt_mlp": (ctypes.c_int, [P(cd_elements), _vp, dbl, P(cd_params), _vp, _vp,
                                         _vp]),
            "cd_mlp_forward": (ctypes.c_int, [_vp, _vp, i64, _vp, _vp]),
            "cd_mlp_grad_ws": (sz, [i64]),
            "cd_mlp_grad": (ctypes.c_int, [_vp, _vp, _vp, i64, _vp, _vp, _vp, sz, _vp]),
            "cd_mlp_adam": (ctypes.c_int, [_vp, _vp, _vp, _vp, i64, flt, flt, flt, flt, _vp,
                                           _vp]),
            "cd_pair_object_counts": (ctypes.c_int, [_vp, i64, i64, _vp, _vp]),
            "cd_counters_available": (ctypes.c_int, []),
            "cd_last_query_levels": (ctypes.c_int, []),
            "cd_counters_reset": (ctypes.c_int, [_vp, i64, _vp]),
            "cd_counters_read": (ctypes.c_int, [P(cd_counters), _vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _libs[path] = L
    return _libs[path]


EXPORTED = ("cd_status_string", "cd_last_error", "cd_version", "cd_stream_copy",
            "cd_profile_enable",
            "cd_profile_read", "cd_box_count_ws",
            "cd_box_count", "cd_validate_ws", "cd_validate_elements", "cd_dt_heuristic",
            "cd_build_boxes_ws", "cd_build_boxes", "cd_tree_bytes", "cd_tree_leaf_records",
            "cd_build_tree_ws",
            "cd_build_tree", "cd_query_pairs_ws", "cd_query_pairs", "cd_query_pairs_async",
            "cd_noalloc_scratch_bytes", "cd_query_pairs_async_noalloc",
            "cd_set_tuning", "cd_get_tuning", "cd_graph_begin", "cd_graph_end",
            "cd_graph_launch", "cd_graph_destroy", "cd_first_witness", "cd_refine_records_ws",
            "cd_refine_records", "cd_band_filter_ws", "cd_band_filter", "cd_band_partition_ws",
            "cd_band_partition", "cd_gather_elements", "cd_remap_records",
            "cd_canonical_records_ws", "cd_canonical_records", "cd_mlp_features",
            "cd_dt_mlp", "cd_mlp_forward", "cd_mlp_grad_ws", "cd_mlp_grad", "cd_mlp_adam",
            "cd_pair_object_counts", "cd_counters_available", "cd_counters_reset",
            "cd_counters_read", "cd_last_query_levels")


def cd_counters_available():
    return int(lib().cd_counters_available())


def cd_counters_reset(visits=None):
    """Zero the executed-work totals and bind `visits` (an int32 device tensor
    of per-object counts that the caller has zeroed, or None)."""
    # the plain library refuses the call before it would touch a stream
    s = _stream() if cd_counters_available() else None
    if visits is not None:
        if visits.dtype != torch.int32 or not visits.is_cuda or not visits.is_contiguous():
            raise ValueError("visits must be a contiguous int32 device tensor")
        _check(lib().cd_counters_reset(_ptr(visits), visits.numel(), s))
    else:
        _check(lib().cd_counters_reset(None, 0, s))


def cd_counters_read():
    """Executed-work totals since the last reset, as a dict (syncs)."""
    c = cd_counters()
    s = _stream() if cd_counters_available() else None
    _check(lib().cd_counters_read(ctypes.byref(c), s))
    return {k: int(getattr(c, k)) for k, _ in cd_counters._fields_}


def cd_stream_copy(dst, src, nbytes=None):
    """Streaming copy of nbytes (default: all of src) between device tensors."""
    n = src.numel() * src.element_size() if nbytes is None else int(nbytes)
    if dst.numel() * dst.element_size() < n:
        raise ValueError("dst is smaller than the copy")
    _check(lib().cd_stream_copy(_ptr(dst), _ptr(src), n, _stream()))


def cd_profile_enable(on=True):
    lib().cd_profile_enable(1 if on else 0)


def cd_profile_read(reset=True):
    """{stage: (total_ms, launches)} accumulated since the last reset (syncs)."""
    m = 32
    names = (ctypes.c_char_p * m)()
    ms = (ctypes.c_double * m)()
    ln = (ctypes.c_int64 * m)()
    k = lib().cd_profile_read(names, ms, ln, m, 1 if reset else 0)
    if k < 0:
        _check(k)
    return {names[i].decode(): (ms[i], ln[i]) for i in range(min(k, m))}


def _check(rc):
    if rc != CD_OK:
        raise CDError(rc, lib().cd_last_error().decode())
    return rc


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def _bytes(nbytes, device):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


# ---- argument marshalling -----------------------------------------------------

def elements_struct(el_soa):
    """el_soa: float64 CUDA tensor [6, n] (rows a, e, inc, raan, argp, m0)."""
    assert el_soa.dtype == torch.float64 and el_soa.is_cuda and el_soa.dim() == 2
    assert el_soa.shape[0] == 6 and el_soa.is_contiguous()
    n = el_soa.shape[1]
    base, row = el_soa.data_ptr(), el_soa.stride(0) * el_soa.element_size()
    rows = [ctypes.c_void_p(base + k * row if n else 0) for k in range(6)]
    return cd_elements(*rows, n)


def params_struct(tick_s, mu, threshold_km, horizon_ticks, dt_ticks=0, start_ticks=0,
                  box_rule=0):
    """box_rule: CD_BOX_SPEED, CD_BOX_INTERVAL_NU or CD_BOX_INTERVAL_E."""
    return cd_params(float(tick_s), float(mu), float(threshold_km), int(horizon_ticks),
                     int(dt_ticks), int(start_ticks), int(box_rule))


class Boxes:
    """Device box arrays (SoA) plus the cd_boxes descriptor.  codes=True adds
    the per-box Morton code array that cd_build_boxes fills for the tree."""

    def __init__(self, count, precision, device="cuda", codes=False, layout=CD_LAYOUT_OBJECT):
        ft = torch.float64 if precision == CD_FP64 else torch.float32
        self.count, self.precision = int(count), precision
        self.lo = torch.empty((3, max(count, 1)), dtype=ft, device=device)
        self.hi = torch.empty((3, max(count, 1)), dtype=ft, device=device)
        self.t0 = torch.empty(max(count, 1), dtype=torch.int32, device=device)
        self.t1 = torch.empty(max(count, 1), dtype=torch.int32, device=device)
        self.obj = torch.empty(max(count, 1), dtype=torch.int32, device=device)
        self.code = (torch.empty(max(count, 1), dtype=torch.int32, device=device)
                     if codes else None)
        self.desc = cd_boxes()
        self.desc.count = self.count
        self.desc.precision = precision
        for d in range(3):
            self.desc.lo[d] = self.lo[d].data_ptr()
            self.desc.hi[d] = self.hi[d].data_ptr()
        self.desc.t0 = self.t0.data_ptr()
        self.desc.t1 = self.t1.data_ptr()
        self.desc.obj = self.obj.data_ptr()
        self.desc.code = self.code.data_ptr() if codes else None
        self.desc.code_valid = 0
        self.desc.layout = layout

    @classmethod
    def in_tree(cls, tree, count, device="cuda", code=None):
        """FP64 box records written straight into an FP64 tree's leaf-record
        area (cd_boxes.records = cd_tree_leaf_records; tree: anything with the
        tree's byte tensor as .mem): lo/hi/t0/t1/obj are strided views of the
        records; codes also go to a packed array (`code`, at least count
        int32 entries, or a new one)."""
        b = cls.__new__(cls)
        b.count, b.precision = int(count), CD_FP64
        N = max(int(count), 1)
        base = lib().cd_tree_leaf_records(_ptr(tree.mem), N)
        off = base - tree.mem.data_ptr()
        recs = tree.mem[off:off + 64 * N]
        f64 = recs.view(torch.float64).view(N, 8)
        u32 = recs.view(torch.int32).view(N, 16)
        b.lo = f64[:, 0:3].t()
        b.hi = f64[:, 3:6].t()
        b.t0, b.t1, b.obj = u32[:, 12], u32[:, 13], u32[:, 14]
        b.code = torch.empty(N, dtype=torch.int32, device=device) if code is None else code[:N]
        b.desc = cd_boxes()
        b.desc.count = b.count
        b.desc.precision = CD_FP64
        b.desc.records = base
        b.desc.code = b.code.data_ptr()
        b.desc.code_valid = 0
        b.desc.layout = CD_LAYOUT_SORTED
        b.tree_ref = tree
        return b

    @classmethod
    def from_arrays(cls, lo, hi, t0, t1, obj, precision=CD_FP64, horizon_ticks=0,
                    obj_count=0, slab_ticks=0, slab_size=0, device="cuda"):
        """Caller-built boxes from host arrays lo/hi [N,3], t0/t1/obj [N]."""
        import numpy as np
        N = len(t0)
        b = cls(N, precision, device)
        npf = np.float64 if precision == CD_FP64 else np.float32
        if N:
            b.lo[:, :N].copy_(torch.from_numpy(np.ascontiguousarray(np.asarray(lo, npf).T)))
            b.hi[:, :N].copy_(torch.from_numpy(np.ascontiguousarray(np.asarray(hi, npf).T)))
            b.t0[:N].copy_(torch.from_numpy(np.asarray(t0, np.uint32).view(np.int32)))
            b.t1[:N].copy_(torch.from_numpy(np.asarray(t1, np.uint32).view(np.int32)))
            b.obj[:N].copy_(torch.from_numpy(np.asarray(obj, np.uint32).view(np.int32)))
        b.desc.horizon_ticks = int(horizon_ticks) if horizon_ticks else int(
            np.max(np.asarray(t0, np.uint64)) if N else 0)
        b.desc.obj_count = int(obj_count) if obj_count else int(
            np.max(np.asarray(obj, np.uint64)) + 1 if N else 0)
        b.desc.slab_ticks = int(slab_ticks)
        b.desc.slab_size = int(slab_size)
        return b

    def to_host(self):
        """(lo [N,3] f64, hi [N,3] f64, t0, t1, obj uint32) as numpy arrays."""
        import numpy as np
        N = self.count
        lo = self.lo[:, :N].T.double().cpu().numpy()
        hi = self.hi[:, :N].T.double().cpu().numpy()
        u = lambda t: t[:N].cpu().numpy().view(np.uint32)
        return lo, hi, u(self.t0), u(self.t1), u(self.obj)


class Tree:
    def __init__(self, count, precision, device="cuda"):
        nbytes = lib().cd_tree_bytes(int(count), precision)
        self.mem = _bytes(nbytes, device)
        self.desc = cd_tree()
        self.desc.mem = self.mem.data_ptr()
        self.desc.bytes = nbytes


# ---- the C functions, marshalled ----------------------------------------------------

def cd_box_count(dt_ticks, n, params, device="cuda"):
    """Box count for per-object steps (int32/uint32 CUDA tensor) or, with
    dt_ticks None, for the uniform params.dt_ticks."""
    out = ctypes.c_int64(0)
    if dt_ticks is None:
        _check(lib().cd_box_count(None, int(n), ctypes.byref(params), ctypes.byref(out), None, 0,
                                  _stream()))
    else:
        ws = _bytes(lib().cd_box_count_ws(int(n)), device)
        _check(lib().cd_box_count(_ptr(dt_ticks), int(n), ctypes.byref(params),
                                  ctypes.byref(out), _ptr(ws), ws.numel(), _stream()))
    return out.value


def cd_validate_elements(el_soa, device="cuda"):
    el = elements_struct(el_soa)
    ws = _bytes(lib().cd_validate_ws(el.n), device)
    bad = ctypes.c_int64(-1)
    rc = lib().cd_validate_elements(ctypes.byref(el), ctypes.byref(bad), _ptr(ws), ws.numel(),
                                    _stream())
    if rc == CD_E_INVALID and bad.value >= 0:
        raise CDError(rc, lib().cd_last_error().decode())
    _check(rc)


def cd_dt_heuristic(el_soa, params, max_disp_km, dt_out):
    el = elements_struct(el_soa)
    _check(lib().cd_dt_heuristic(ctypes.byref(el), ctypes.byref(params), float(max_disp_km),
                                 _ptr(dt_out), _stream()))


def cd_build_boxes(el_soa, dt_ticks, params, boxes, ws):
    el = elements_struct(el_soa)
    _check(lib().cd_build_boxes(ctypes.byref(el), _ptr(dt_ticks) if dt_ticks is not None else None,
                                ctypes.byref(params), ctypes.byref(boxes.desc), _ptr(ws),
                                ws.numel(), _stream()))


def cd_build_tree(boxes, precision, tree, ws, slab_ticks=0):
    _check(lib().cd_build_tree(ctypes.byref(boxes.desc), precision, int(slab_ticks),
                               ctypes.byref(tree.desc), _ptr(ws), ws.numel(), _stream()))


def cd_query_pairs(tree, out, capacity, ws):
    """Returns (status, count).  CD_E_CAPACITY is returned, not raised, with the
    number of records needed."""
    cnt = ctypes.c_int64(0)
    rc = lib().cd_query_pairs(ctypes.byref(tree.desc), _ptr(out), int(capacity),
                              ctypes.byref(cnt), _ptr(ws), ws.numel(), _stream())
    if rc not in (CD_OK, CD_E_CAPACITY):
        _check(rc)
    return rc, cnt.value


def cd_query_pairs_async(tree, out, capacity, count_dev, status_dev, ws):
    """Enqueue the graph-capturable query; count_dev (int64 [1]) and
    status_dev (int32 [1]) are CUDA tensors written by the device."""
    if capacity < 1 or out.shape[0] < capacity:
        raise ValueError("out must hold `capacity` records")
    _check(lib().cd_query_pairs_async(ctypes.byref(tree.desc), _ptr(out), int(capacity),
                                      _ptr(count_dev), _ptr(status_dev), _ptr(ws), ws.numel(),
                                      _stream()))


TUNING_DEFAULTS = {"expand_blocks": 2048, "expand_threads": 256, "walk_threads": 256,
                   "mode": 0, "max_levels": 96}


def cd_query_pairs_async_noalloc(tree, out, capacity, count_dev, status_dev):
    """cd_query_pairs_async with the library's fixed scratch as workspace."""
    if capacity < 1 or out.shape[0] < capacity:
        raise ValueError("out must hold `capacity` records")
    _check(lib().cd_query_pairs_async_noalloc(ctypes.byref(tree.desc), _ptr(out), int(capacity),
                                              _ptr(count_dev), _ptr(status_dev), _stream()))


def cd_set_tuning(t=None):
    """t: dict of cd_tuning fields (missing or 0 -> default), or None for defaults."""
    if t is None:
        _check(lib().cd_set_tuning(None))
        return
    v = cd_tuning(*(int(t.get(k, 0)) for k, _ in cd_tuning._fields_))
    _check(lib().cd_set_tuning(ctypes.byref(v)))


def cd_last_query_levels():
    return int(lib().cd_last_query_levels())


def cd_get_tuning():
    v = cd_tuning()
    _check(lib().cd_get_tuning(ctypes.byref(v)))
    return {k: int(getattr(v, k)) for k, _ in cd_tuning._fields_}


class Graph:
    """Work recorded from the current stream between begin() and end(),
    replayed by launch() (cd_graph_*)."""

    def __init__(self):
        self.h = ctypes.c_void_p(0)

    def begin(self):
        _check(lib().cd_graph_begin(_stream()))

    def end(self):
        _check(lib().cd_graph_end(_stream(), ctypes.byref(self.h)))

    def launch(self):
        _check(lib().cd_graph_launch(self.h, _stream()))

    def close(self):
        if self.h:
            lib().cd_graph_destroy(self.h)
            self.h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


CD_NO_WITNESS = 0xFFFFFFFF


def cd_first_witness(el_soa, params, delta_ticks, pairs):
    """Narrow phase over records (int32 [P, 4] CUDA tensor): (witness int32 [P]
    -- CD_NO_WITNESS read as uint32 where none --, first int64 [1] on the
    device = min over records of (t << 32 | record))."""
    if not (pairs.is_cuda and pairs.dtype == torch.int32 and pairs.dim() == 2
            and pairs.shape[1] == 4 and pairs.is_contiguous()):
        raise ValueError("pairs: need a contiguous int32 CUDA tensor [P, 4]")
    el = elements_struct(el_soa)
    P = int(pairs.shape[0])
    wit = torch.empty(max(P, 1), dtype=torch.int32, device=pairs.device)
    first = torch.empty(1, dtype=torch.int64, device=pairs.device)
    _check(lib().cd_first_witness(ctypes.byref(el), ctypes.byref(params), int(delta_ticks),
                                  _ptr(pairs), P, _ptr(wit), _ptr(first), _stream()))
    return wit[:P], first


def cd_refine_records(el_soa, params, delta_ticks, pairs, min_steps=1, capacity=None):
    """Bulk interval refinement of records (int32 [P, 4] CUDA tensor): the
    canonical leaves, int32 [L, 4] (i, j, first instant, last instant + 1; read
    as uint32).  Grows the output and work buffers and repeats when they are
    too small."""
    if not (pairs.is_cuda and pairs.dtype == torch.int32 and pairs.dim() == 2
            and pairs.shape[1] == 4 and pairs.is_contiguous()):
        raise ValueError("pairs: need a contiguous int32 CUDA tensor [P, 4]")
    el = elements_struct(el_soa)
    P = int(pairs.shape[0])
    cap = int(capacity) if capacity is not None else max(4 * P, 1 << 16)
    for _ in range(8):
        out = torch.empty((max(cap, 1), 4), dtype=torch.int32, device=pairs.device)
        ws = _bytes(lib().cd_refine_records_ws(el.n, P, cap), pairs.device)
        cnt = ctypes.c_int64(0)
        rc = lib().cd_refine_records(ctypes.byref(el), ctypes.byref(params), int(delta_ticks),
                                     int(min_steps), _ptr(pairs), P, _ptr(out), cap,
                                     ctypes.byref(cnt), _ptr(ws), ws.numel(), _stream())
        if rc != CD_E_CAPACITY:
            _check(rc)
            return out[:cnt.value]
        cap = max(int(cnt.value * 1.25) + 1024, 2 * cap)
    _check(rc)


def _need_pairs(pairs):
    if not (pairs.is_cuda and pairs.dtype == torch.int32 and pairs.dim() == 2
            and pairs.shape[1] == 4 and pairs.is_contiguous()):
        raise ValueError("pairs: need a contiguous int32 CUDA tensor [P, 4]")


def cd_band_filter(el_soa, params, pairs):
    """The records whose objects' radial bands meet (int32 [K, 4], input order)."""
    _need_pairs(pairs)
    el = elements_struct(el_soa)
    P = int(pairs.shape[0])
    out = torch.empty((max(P, 1), 4), dtype=torch.int32, device=pairs.device)
    ws = _bytes(lib().cd_band_filter_ws(P), pairs.device)
    cnt = ctypes.c_int64(0)
    _check(lib().cd_band_filter(ctypes.byref(el), ctypes.byref(params), _ptr(pairs), P,
                                _ptr(out), ctypes.byref(cnt), _ptr(ws), ws.numel(), _stream()))
    return out[:cnt.value]


def cd_band_partition(el_soa, params, nbands):
    """(edges float64 [p+1], offsets int32 [p+1], members int32 [M]) on the device:
    band k's objects are members[offsets[k]:offsets[k+1]]."""
    el = elements_struct(el_soa)
    dev = el_soa.device
    edges = torch.empty(int(nbands) + 1, dtype=torch.float64, device=dev)
    offsets = torch.empty(int(nbands) + 1, dtype=torch.int32, device=dev)
    cap = max(2 * el.n, 1)
    ws = _bytes(lib().cd_band_partition_ws(el.n, int(nbands)), dev)
    for _ in range(2):
        members = torch.empty(cap, dtype=torch.int32, device=dev)
        cnt = ctypes.c_int64(0)
        rc = lib().cd_band_partition(ctypes.byref(el), ctypes.byref(params), int(nbands),
                                     _ptr(edges), _ptr(offsets), _ptr(members), cap,
                                     ctypes.byref(cnt), _ptr(ws), ws.numel(), _stream())
        if rc != CD_E_CAPACITY:
            _check(rc)
            return edges, offsets, members[:cnt.value]
        cap = int(cnt.value)
    _check(rc)


def cd_gather_elements(el_soa, ids):
    """Elements [6, len(ids)] of objects ids (int32 CUDA tensor)."""
    el = elements_struct(el_soa)
    out = torch.empty((6, max(int(ids.numel()), 1)), dtype=torch.float64, device=el_soa.device)
    _check(lib().cd_gather_elements(ctypes.byref(el), _ptr(ids), int(ids.numel()), _ptr(out),
                                    _stream()))
    return out[:, :int(ids.numel())]


def cd_remap_records(pairs, ids, out=None):
    """Local ids of records mapped through ids (int32 CUDA tensor) into out."""
    _need_pairs(pairs)
    if out is None:
        out = torch.empty_like(pairs)
    _check(lib().cd_remap_records(_ptr(pairs), int(pairs.shape[0]), _ptr(ids),
                                  int(ids.numel()), _ptr(out), _stream()))
    return out


def cd_canonical_records(pairs, horizon_ticks, obj_count):
    """The canonical list (sorted, repeats removed) of any records."""
    _need_pairs(pairs)
    P = int(pairs.shape[0])
    out = torch.empty((max(P, 1), 4), dtype=torch.int32, device=pairs.device)
    ws = _bytes(lib().cd_canonical_records_ws(P), pairs.device)
    cnt = ctypes.c_int64(0)
    _check(lib().cd_canonical_records(_ptr(pairs), P, int(horizon_ticks), int(obj_count),
                                      _ptr(out), ctypes.byref(cnt), _ptr(ws), ws.numel(),
                                      _stream()))
    return out[:cnt.value]


def first_collision(pairs, first):
    """(t, i, j) of the earliest collision from cd_first_witness's result, or None."""
    v = int(first.item()) & 0xFFFFFFFFFFFFFFFF
    if v == 0xFFFFFFFFFFFFFFFF:
        return None
    t, r = v >> 32, v & 0xFFFFFFFF
    i, j = (int(x) & 0xFFFFFFFF for x in pairs[r, :2].tolist())
    return t, i, j


class BroadPhase:
    """Buffers for repeated queries over one catalog shape.

    ``run(el_soa)`` builds the boxes, the tree and the canonical pair list;
    returns an int32 CUDA tensor [P, 4] (i, j, t_lo, t_hi; read as uint32).
    Buffers are allocated here and grown only when the pair count exceeds the
    current capacity (then the query alone is repeated).
    """

    def __init__(self, n, params, dt_ticks=None, box_precision=CD_FP64,
                 tree_precision=CD_FP64, capacity=None, slab_ticks=0, device="cuda",
                 dt_heuristic_km=None, el_soa=None, dt_mlp=None, codes=True,
                 layout=CD_LAYOUT_SORTED, in_tree=True):
        """dt_heuristic_km: per-object steps from cd_dt_heuristic; dt_mlp:
        (bfloat16 weight tensor, fallback_disp_km) for steps from cd_dt_mlp.
        Either is recomputed by every build from the elements (el_soa is
        needed here to size the buffers).  layout: the box order requested
        from cd_build_boxes for a uniform step (CD_LAYOUT_SORTED needs codes;
        the layout written is in boxes.desc.layout after a build).  in_tree:
        FP64 boxes of a sorted uniform step are written as the FP64 tree's
        leaf records (boxes then views those records)."""
        self.dt_heuristic_km = dt_heuristic_km
        self.dt_mlp = dt_mlp
        if dt_heuristic_km is not None or dt_mlp is not None:
            dt_ticks = torch.empty(int(n), dtype=torch.int32, device=device)
            self._steps(el_soa, params, dt_ticks)
        self.n, self.params, self.dt = int(n), params, dt_ticks
        self.device = device
        self.count = cd_box_count(dt_ticks, n, params, device)
        self.layout = layout if codes else CD_LAYOUT_OBJECT
        self.tree_precision = tree_precision
        self.tree = Tree(self.count, tree_precision, device)
        # FP64 boxes of a uniform step in Morton order go straight into the
        # FP64 tree's leaf records (no sort, no copy in the tree build)
        self.in_tree = (in_tree and dt_ticks is None and box_precision == CD_FP64
                        and tree_precision == CD_FP64 and self.layout == CD_LAYOUT_SORTED
                        and self.n <= CD_SORTED_MAX_RECORDS and self.count > 0)
        if self.in_tree:
            self.boxes = Boxes.in_tree(self.tree, self.count, device)
        else:
            self.boxes = Boxes(self.count, box_precision, device, codes=codes,
                               layout=self.layout)
        self.ws_boxes = _bytes(lib().cd_build_boxes_ws(self.n), device)
        self.ws_tree = _bytes(lib().cd_build_tree_ws(self.count), device)
        self.slab_ticks = slab_ticks
        self._alloc_query(capacity if capacity is not None else max(1 << 16, self.count // 64))

    def _alloc_query(self, cap):
        self.capacity = int(cap)
        self.out = torch.empty((max(self.capacity, 1), 4), dtype=torch.int32, device=self.device)
        self.ws_query = _bytes(lib().cd_query_pairs_ws(self.count, self.capacity), self.device)

    def _steps(self, el_soa, params, dt):
        if self.dt_mlp is not None:
            el = elements_struct(el_soa)
            w, fallback = self.dt_mlp
            _check(lib().cd_dt_mlp(ctypes.byref(el), _ptr(w), float(fallback),
                                   ctypes.byref(params), _ptr(dt), None, _stream()))
        else:
            cd_dt_heuristic(el_soa, params, self.dt_heuristic_km, dt)

    def build(self, el_soa):
        if self.dt_heuristic_km is not None or self.dt_mlp is not None:
            self._steps(el_soa, self.params, self.dt)
        self.boxes.desc.layout = self.layout
        cd_build_boxes(el_soa, self.dt, self.params, self.boxes, self.ws_boxes)
        cd_build_tree(self.boxes, self.tree_precision, self.tree, self.ws_tree, self.slab_ticks)

    def query(self):
        rc, cnt = cd_query_pairs(self.tree, self.out, self.capacity, self.ws_query)
        if rc == CD_E_CAPACITY:
            self._alloc_query(int(cnt * 1.25) + 1024)
            rc, cnt = cd_query_pairs(self.tree, self.out, self.capacity, self.ws_query)
            _check(rc)
        return self.out[:cnt]

    def run(self, el_soa):
        self.build(el_soa)
        return self.query()


def query_boxes(boxes, tree_precision=CD_FP64, slab_ticks=0, capacity=1 << 16):
    """Tree + canonical pairs over caller-built ``Boxes``."""
    tree = Tree(boxes.count, tree_precision, boxes.lo.device)
    ws = _bytes(lib().cd_build_tree_ws(boxes.count), boxes.lo.device)
    cd_build_tree(boxes, tree_precision, tree, ws, slab_ticks)
    while True:
        out = torch.empty((max(capacity, 1), 4), dtype=torch.int32, device=boxes.lo.device)
        wsq = _bytes(lib().cd_query_pairs_ws(boxes.count, capacity), boxes.lo.device)
        rc, cnt = cd_query_pairs(tree, out, capacity, wsq)
        if rc == CD_OK:
            return out[:cnt]
        capacity = int(cnt * 1.25) + 1024


def soa(elements_np, device="cuda"):
    """Host [n, 6] element rows -> device [6, n] float64 (the library's layout)."""
    import numpy as np
    a = np.ascontiguousarray(np.asarray(elements_np, np.float64).reshape(-1, 6).T)
    return torch.from_numpy(a).to(device)
