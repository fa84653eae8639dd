"""C-ABI checks that need no GPU: the library loads, exports every function
include/cd4d.h declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "cd4d.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cd_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import paper_1901_10475_amd as cd
    L = cd.lib()
    decl = _declared()
    assert len(decl) >= 15
    for name in decl:
        assert hasattr(L, name), name
    assert set(decl) == set(cd.EXPORTED)


def test_counters_build_exports_the_same_symbols():
    """libcd4d_counters.so (CD_COUNTERS) is the same ABI; only it answers the
    counter calls, the plain library refuses them without touching a device."""
    import paper_1901_10475_amd as cd
    assert cd.cd_counters_available() == 0
    with pytest.raises(cd.CDError) as ei:
        cd.cd_counters_read()
    assert ei.value.status == cd.CD_E_INVALID
    with pytest.raises(cd.CDError) as ei:
        cd.cd_counters_reset(None)
    assert ei.value.status == cd.CD_E_INVALID
    with cd.counters_build() as L:
        for name in _declared():
            assert hasattr(L, name), name
        assert cd.cd_counters_available() == 1
        assert L is not cd._load(cd._LIB_PATH)
    assert cd.lib() is cd._load(cd._LIB_PATH)
    assert cd.cd_counters_available() == 0


def test_header_constants_match_the_binding():
    """Every #define CD_* integer constant of include/cd4d.h has the same value
    in the Python binding."""
    import paper_1901_10475_amd as cd
    src = open(os.path.join(ROOT, "include", "cd4d.h")).read()
    defs = dict(re.findall(r"#define\s+(CD_[A-Z_0-9]+)\s+(-?\d+)\b", src))
    assert "CD_SORTED_MAX_RECORDS" in defs and "CD_LAYOUT_SORTED" in defs
    for name, value in defs.items():
        if hasattr(cd, name):
            assert getattr(cd, name) == int(value), name
    assert cd.CD_SORTED_MAX_ARRAYS == int(defs["CD_SORTED_MAX_ARRAYS"])
    assert cd.CD_SORTED_MAX_RECORDS == int(defs["CD_SORTED_MAX_RECORDS"])


def test_status_strings_and_version():
    import paper_1901_10475_amd as cd
    L = cd.lib()
    assert L.cd_version() >= 1
    for s in range(6):
        assert L.cd_status_string(s).decode()
    assert L.cd_status_string(99).decode() == "unknown status"


def test_sizes_are_host_only_and_monotone():
    import paper_1901_10475_amd as cd
    L = cd.lib()
    assert L.cd_tree_bytes(0, cd.CD_FP64) == 256
    # header, 2N-1 node records, children of the N-1 inner nodes, and room for
    # the overlapping sibling pairs the refit records
    seeds = (10 // 4 + 4096) * 8
    # (FP64: plus a skip link per leaf, for leaf records written in place)
    assert L.cd_tree_bytes(10, cd.CD_FP64) == 256 + 19 * 64 + 9 * 8 + seeds + 10 * 4
    assert L.cd_tree_bytes(10, cd.CD_FP32) == 256 + 19 * 40 + 9 * 8 + seeds
    assert L.cd_build_tree_ws(1000) < L.cd_build_tree_ws(100000)
    assert L.cd_query_pairs_ws(10, 1000) < L.cd_query_pairs_ws(10, 100000)


def test_uniform_box_count_and_argument_errors():
    import paper_1901_10475_amd as cd
    L = cd.lib()
    out = ctypes.c_int64(-1)
    p = cd.params_struct(1e-3, 398600.4418, 1.0, 600_000, 10_000)
    assert L.cd_box_count(None, 1000, ctypes.byref(p), ctypes.byref(out), None, 0, None) == 0
    assert out.value == 60_000
    p = cd.params_struct(1e-3, 398600.4418, 1.0, 25, 10)
    assert L.cd_box_count(None, 3, ctypes.byref(p), ctypes.byref(out), None, 0, None) == 0
    assert out.value == 9
    p = cd.params_struct(1e-3, 398600.4418, 1.0, 0, 10)          # T = 0: one instant
    assert L.cd_box_count(None, 4, ctypes.byref(p), ctypes.byref(out), None, 0, None) == 0
    assert out.value == 4
    bad = [cd.params_struct(1e-3, 398600.4418, 1.0, 600, 0),        # dt = 0
           cd.params_struct(0.0, 398600.4418, 1.0, 600, 1),         # tick 0
           cd.params_struct(1e-3, 398600.4418, -1.0, 600, 1),       # thr < 0
           cd.params_struct(1e-3, float("nan"), 1.0, 600, 1),
           cd.params_struct(1e-3, 398600.4418, 1.0, 600, 1, box_rule=3)]  # unknown rule
    for q in bad:
        assert L.cd_box_count(None, 5, ctypes.byref(q), ctypes.byref(out), None, 0,
                              None) == cd.CD_E_INVALID
        assert L.cd_last_error().decode()
    q = cd.params_struct(1e-3, 398600.4418, 1.0, 2 ** 32 - 1, 1)
    assert L.cd_box_count(None, 5, ctypes.byref(q), ctypes.byref(out), None, 0,
                          None) == cd.CD_E_OVERFLOW
    q = cd.params_struct(1e-3, 398600.4418, 1.0, 2 ** 31, 1)     # 2^31 boxes per object
    assert L.cd_box_count(None, 5, ctypes.byref(q), ctypes.byref(out), None, 0,
                          None) == cd.CD_E_OVERFLOW
    assert L.cd_box_count(None, -1, ctypes.byref(p), ctypes.byref(out), None, 0,
                          None) == cd.CD_E_INVALID
    assert L.cd_box_count(None, 5, None, ctypes.byref(out), None, 0, None) == cd.CD_E_INVALID


def test_null_and_workspace_errors_before_any_launch():
    import paper_1901_10475_amd as cd
    L = cd.lib()
    p = cd.params_struct(1e-3, 398600.4418, 1.0, 600, 10)
    el = cd.cd_elements(None, None, None, None, None, None, 5)     # n > 0, NULL arrays
    b = cd.cd_boxes()
    b.count = 300
    assert L.cd_build_boxes(ctypes.byref(el), None, ctypes.byref(p), ctypes.byref(b), None, 0,
                            None) == cd.CD_E_INVALID
    tree = cd.cd_tree()
    b.precision = 7
    assert L.cd_build_tree(ctypes.byref(b), cd.CD_FP64, 0, ctypes.byref(tree), None, 0,
                           None) == cd.CD_E_INVALID
    b.precision = cd.CD_FP32
    assert L.cd_build_tree(ctypes.byref(b), cd.CD_FP64, 0, ctypes.byref(tree), None, 0,
                           None) == cd.CD_E_INVALID                  # FP64 tree of FP32 boxes
    cnt = ctypes.c_int64(0)
    assert L.cd_query_pairs(ctypes.byref(tree), None, 0, ctypes.byref(cnt), None, 0,
                            None) == cd.CD_E_INVALID                 # tree not built


def test_step_network_argument_errors_before_any_launch():
    import paper_1901_10475_amd as cd
    L = cd.lib()
    p = cd.params_struct(1e-3, 398600.4418, 1.0, 600, 10)
    el = cd.cd_elements(None, None, None, None, None, None, 5)     # n > 0, NULL arrays
    assert L.cd_mlp_features(ctypes.byref(el), ctypes.byref(p), None, None) == cd.CD_E_INVALID
    el0 = cd.cd_elements(None, None, None, None, None, None, 0)
    assert L.cd_mlp_features(ctypes.byref(el0), ctypes.byref(p), None, None) == cd.CD_OK
    assert L.cd_dt_mlp(ctypes.byref(el0), None, 0.0, ctypes.byref(p), None, None,
                       None) == cd.CD_E_INVALID                      # fallback <= 0
    assert L.cd_dt_mlp(ctypes.byref(el0), None, 5.0, ctypes.byref(p), None, None,
                       None) == cd.CD_OK                             # n = 0: nothing to do
    fake = ctypes.c_void_p(16)                                       # never dereferenced
    assert L.cd_mlp_forward(fake, fake, -1, fake, None) == cd.CD_E_INVALID
    assert L.cd_mlp_forward(None, None, 0, None, None) == cd.CD_OK
    assert L.cd_mlp_grad(fake, fake, fake, 0, fake, None, fake, 1 << 30,
                         None) == cd.CD_E_INVALID                    # empty batch
    assert L.cd_mlp_grad(fake, fake, fake, 10, fake, None, fake, 16,
                         None) == cd.CD_E_WORKSPACE
    assert L.cd_mlp_adam(fake, fake, fake, fake, 0, 1e-3, 0.9, 0.999, 1e-8, None,
                         None) == cd.CD_E_INVALID                    # step counts from 1
    assert L.cd_mlp_adam(fake, fake, fake, fake, 1, 1e-3, 1.0, 0.999, 1e-8, None,
                         None) == cd.CD_E_INVALID                    # beta1 = 1
    assert L.cd_pair_object_counts(None, 3, 5, fake, None) == cd.CD_E_INVALID
    assert L.cd_pair_object_counts(None, 0, 0, None, None) == cd.CD_OK
    # workspace grows with the batch: activations + one partial row per 128 samples
    w1, w2 = L.cd_mlp_grad_ws(1), L.cd_mlp_grad_ws(5000)
    assert w2 >= 258 * 4 * 5000 + 40 * 4610 * 4 > w1 > 0


def test_refine_argument_errors_before_any_launch():
    import paper_1901_10475_amd as cd
    L = cd.lib()
    p = cd.params_struct(1e-3, 398600.4418, 1.0, 600, 10)
    el0 = cd.cd_elements(None, None, None, None, None, None, 0)
    fake = ctypes.c_void_p(16)                                       # never dereferenced
    cnt = ctypes.c_int64(7)
    ws_bytes = L.cd_refine_records_ws(0, 0, 0)
    assert ws_bytes > 0
    # delta or min_steps 0, negative count, NULL pairs, missing workspace
    assert L.cd_refine_records(ctypes.byref(el0), ctypes.byref(p), 0, 1, None, 0, None, 0,
                               ctypes.byref(cnt), fake, ws_bytes, None) == cd.CD_E_INVALID
    assert L.cd_refine_records(ctypes.byref(el0), ctypes.byref(p), 1, 0, None, 0, None, 0,
                               ctypes.byref(cnt), fake, ws_bytes, None) == cd.CD_E_INVALID
    assert L.cd_refine_records(ctypes.byref(el0), ctypes.byref(p), 1, 1, None, -1, None, 0,
                               ctypes.byref(cnt), fake, ws_bytes, None) == cd.CD_E_INVALID
    assert L.cd_refine_records(ctypes.byref(el0), ctypes.byref(p), 1, 1, None, 5, fake, 5,
                               ctypes.byref(cnt), fake, 1 << 30, None) == cd.CD_E_INVALID
    assert L.cd_refine_records(ctypes.byref(el0), ctypes.byref(p), 1, 1, fake, 5, fake, 5,
                               ctypes.byref(cnt), fake, 16, None) == cd.CD_E_WORKSPACE
    bad = cd.params_struct(1e-3, 398600.4418, 1.0, 600, 10, box_rule=9)
    assert L.cd_refine_records(ctypes.byref(el0), ctypes.byref(bad), 1, 1, None, 0, None, 0,
                               ctypes.byref(cnt), fake, ws_bytes, None) == cd.CD_E_INVALID
    # nothing to refine: no launch, zero leaves
    assert L.cd_refine_records(ctypes.byref(el0), ctypes.byref(p), 1, 1, None, 0, None, 0,
                               ctypes.byref(cnt), fake, ws_bytes, None) == cd.CD_OK
    assert cnt.value == 0
    # the work queue is sized from the records and the capacity
    assert L.cd_refine_records_ws(100, 10**6, 0) > L.cd_refine_records_ws(100, 10, 0)


def test_band_argument_errors_before_any_launch():
    import paper_1901_10475_amd as cd
    L = cd.lib()
    p = cd.params_struct(1e-3, 398600.4418, 1.0, 600, 10)
    el0 = cd.cd_elements(None, None, None, None, None, None, 0)
    el5 = cd.cd_elements(None, None, None, None, None, None, 5)     # n > 0, NULL arrays
    fake = ctypes.c_void_p(16)                                       # never dereferenced
    cnt = ctypes.c_int64(7)
    assert L.cd_band_filter(ctypes.byref(el5), ctypes.byref(p), fake, 1, fake,
                            ctypes.byref(cnt), fake, 1 << 20, None) == cd.CD_E_INVALID
    assert L.cd_band_filter(ctypes.byref(el0), ctypes.byref(p), fake, 10, fake,
                            ctypes.byref(cnt), fake, 8, None) == cd.CD_E_WORKSPACE
    assert L.cd_band_filter(ctypes.byref(el0), ctypes.byref(p), None, 0, None,
                            ctypes.byref(cnt), fake, L.cd_band_filter_ws(0), None) == cd.CD_OK
    assert cnt.value == 0
    ws = L.cd_band_partition_ws(0, 4)
    for bands in (0, 4097):
        assert L.cd_band_partition(ctypes.byref(el0), ctypes.byref(p), bands, fake, fake, fake,
                                   0, ctypes.byref(cnt), fake, 1 << 30, None) == cd.CD_E_INVALID
    assert L.cd_band_partition(ctypes.byref(el0), ctypes.byref(p), 4, None, fake, fake, 0,
                               ctypes.byref(cnt), fake, ws, None) == cd.CD_E_INVALID
    assert L.cd_band_partition_ws(1000, 8) > L.cd_band_partition_ws(1000, 2)
    assert L.cd_gather_elements(ctypes.byref(el0), None, -1, None, None) == cd.CD_E_INVALID
    assert L.cd_gather_elements(ctypes.byref(el0), None, 3, None, None) == cd.CD_E_INVALID
    assert L.cd_remap_records(None, 2, None, 5, None, None) == cd.CD_E_INVALID
    assert L.cd_remap_records(None, 0, None, 0, None, None) == cd.CD_OK
    assert L.cd_canonical_records(None, 3, 10, 10, None, ctypes.byref(cnt), fake, 1 << 20,
                                  None) == cd.CD_E_INVALID
    assert L.cd_canonical_records(fake, 3, 10, 10, fake, ctypes.byref(cnt), fake, 8,
                                  None) == cd.CD_E_WORKSPACE


def test_tuning_ranges():
    """Launch shapes: node-pair workgroups of 64 to 1024 lanes (powers of 2),
    per-leaf-walk workgroups of 64, 128 or 256, traversal modes 0 to 2;
    anything else is rejected and changes nothing."""
    import paper_1901_10475_amd as cd
    cd.cd_set_tuning(None)
    base = cd.cd_get_tuning()
    for bad in ({"expand_threads": 384}, {"expand_threads": 2048}, {"walk_threads": 512},
                {"expand_blocks": 32}, {"mode": 3}):
        with pytest.raises(cd.CDError):
            cd.cd_set_tuning(bad)
        assert cd.cd_get_tuning() == base
    for ok in (512, 1024, 64):
        cd.cd_set_tuning({"expand_threads": ok})
        assert cd.cd_get_tuning()["expand_threads"] == ok
    for mode in (0, 1, 2):
        cd.cd_set_tuning({"mode": mode})
        assert cd.cd_get_tuning()["mode"] == mode
    cd.cd_set_tuning(None)
    assert cd.cd_get_tuning() == base


def test_stream_copy_argument_errors():
    """Checked on the host before any launch: misaligned sizes or addresses,
    overlap, NULL pointers; a zero-byte copy does nothing."""
    import paper_1901_10475_amd as cd
    L = cd.lib()
    assert L.cd_stream_copy(None, None, 0, None) == cd.CD_OK
    assert L.cd_stream_copy(None, ctypes.c_void_p(4096), 16, None) == cd.CD_E_INVALID
    assert L.cd_stream_copy(ctypes.c_void_p(8192), ctypes.c_void_p(4096), 17, None) == \
        cd.CD_E_INVALID
    assert L.cd_stream_copy(ctypes.c_void_p(8200), ctypes.c_void_p(4096), 16, None) == \
        cd.CD_E_INVALID
    assert L.cd_stream_copy(ctypes.c_void_p(4096 + 16), ctypes.c_void_p(4096), 64, None) == \
        cd.CD_E_INVALID
    assert "overlap" in L.cd_last_error().decode()


def test_tuning_is_per_thread():
    """Launch shapes set by one thread are not seen by another (no shared
    state between concurrent callers); NULL restores the defaults."""
    import threading
    import paper_1901_10475_amd as cd
    cd.cd_set_tuning({"expand_blocks": 512, "expand_threads": 128})
    try:
        seen = {}

        def other():
            seen["t"] = cd.cd_get_tuning()
            cd.cd_set_tuning({"walk_threads": 64})

        th = threading.Thread(target=other)
        th.start()
        th.join()
        assert seen["t"]["expand_blocks"] == 2048 and seen["t"]["expand_threads"] == 256
        mine = cd.cd_get_tuning()
        assert mine["expand_blocks"] == 512 and mine["expand_threads"] == 128
        assert mine["walk_threads"] == 256
    finally:
        cd.cd_set_tuning(None)
    assert cd.cd_get_tuning()["expand_blocks"] == 2048


def test_tree_leaf_records_and_record_argument_errors():
    """The leaf-record area of an FP64 tree buffer (pure pointer arithmetic),
    and box records refused before any launch where they cannot be used."""
    import paper_1901_10475_amd as cd
    L = cd.lib()
    L.cd_tree_leaf_records.restype = ctypes.c_void_p
    assert L.cd_tree_leaf_records(ctypes.c_void_p(1 << 20), 10) == (1 << 20) + 256 + 9 * 64
    assert L.cd_tree_leaf_records(ctypes.c_void_p(1 << 20), 0) is None
    assert L.cd_tree_leaf_records(None, 10) is None
    el = cd.cd_elements()
    el.n = 0
    p = cd.params_struct(1e-3, 398600.4418, 1.0, 100, 10)
    b = cd.cd_boxes()
    b.precision = cd.CD_FP32
    b.records = 1 << 20
    # n = 0 is accepted before the record checks; n = 1 with FP32 records is not
    for name in ("a", "e", "inc", "raan", "argp", "m0"):
        setattr(el, name, 4096)
    el.n = 1
    b.count = 10
    rc = L.cd_build_boxes(ctypes.byref(el), None, ctypes.byref(p), ctypes.byref(b), None, 0,
                          None)
    assert rc == cd.CD_E_INVALID and "FP64" in L.cd_last_error().decode()
