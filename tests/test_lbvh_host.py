"""Pre-flight of the LBVH index arithmetic (cd_logic.h, run on the CPU through
libcd4d_hostcheck.so): the Karras topology is a binary tree over the sorted
leaves, skip links follow pre-order, and the stackless walk that the traversal
kernel performs terminates and finds exactly the oracle's pair set."""
import ctypes
import os

import numpy as np
import pytest

import oracle
from paper_1901_10475_amd import catalog

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(os.path.dirname(HERE), "paper_1901_10475_amd", "libcd4d_hostcheck.so")
END = 0xFFFFFFFF


def _lib():
    L = ctypes.CDLL(LIB)
    vp = ctypes.c_void_p
    L.hc_karras.argtypes = [vp, ctypes.c_int64, vp, vp, vp, vp, vp, vp]
    L.hc_morton30.restype = ctypes.c_uint32
    L.hc_morton30.argtypes = [ctypes.c_double] * 3 + [vp, vp]
    L.hc_traverse.restype = ctypes.c_int64
    L.hc_traverse.argtypes = [ctypes.c_int64, vp, vp, vp, vp, vp, vp, ctypes.c_uint32, vp,
                              ctypes.c_int64]
    return L


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def sorted_keys(lo, hi, t0, slab_ticks):
    L = _lib()
    c = 0.5 * (lo + hi)
    mn = c.min(0) if len(c) else np.zeros(3)
    ext = (c.max(0) - mn) if len(c) else np.zeros(3)
    inv = np.where(ext > 0, 1.0 / np.where(ext > 0, ext, 1.0), 0.0)
    mn, inv = np.ascontiguousarray(mn), np.ascontiguousarray(inv)
    m = np.array([L.hc_morton30(x, y, z, _p(mn), _p(inv)) for x, y, z in c], np.uint64)
    key = ((t0.astype(np.uint64) // np.uint64(slab_ticks)) << np.uint64(32)) | m
    order = np.argsort(key, kind="stable")
    return np.ascontiguousarray(key[order]), order


def build_host_tree(lo, hi, t0, t1, obj, slab_ticks):
    L = _lib()
    N = len(t0)
    keys, order = sorted_keys(lo, hi, t0, slab_ticks)
    left = np.zeros(max(N - 1, 1), np.uint32)
    right = np.zeros_like(left)
    first = np.zeros(max(N - 1, 1), np.int64)
    last = np.zeros_like(first)
    esc_in = np.zeros(max(N - 1, 1), np.uint32)
    esc_leaf = np.zeros(N, np.uint32)
    L.hc_karras(_p(keys), N, _p(left), _p(right), _p(first), _p(last), _p(esc_in), _p(esc_leaf))
    M = 2 * N - 1
    nlo = np.zeros((M, 3))
    nhi = np.zeros((M, 3))
    nt0 = np.zeros(M, np.uint32)
    nt1 = np.zeros(M, np.uint32)
    link = np.zeros(M, np.uint32)
    esc = np.zeros(M, np.uint32)
    nlo[N - 1:] = lo[order]
    nhi[N - 1:] = hi[order]
    nt0[N - 1:] = t0[order]
    nt1[N - 1:] = t1[order]
    link[N - 1:] = obj[order]
    esc[N - 1:] = esc_leaf
    if N > 1:
        link[:N - 1] = left[:N - 1]
        esc[:N - 1] = esc_in[:N - 1]
        # unions, children before parents (post-order)
        def post(u):
            stack, out = [(u, False)], []
            while stack:
                x, done = stack.pop()
                if x >= N - 1:
                    continue
                if done:
                    out.append(x)
                else:
                    stack += [(x, True), (int(right[x]), False), (int(left[x]), False)]
            return out
        for x in post(0):
            l, r = int(left[x]), int(right[x])
            nlo[x] = np.minimum(nlo[l], nlo[r])
            nhi[x] = np.maximum(nhi[l], nhi[r])
            nt0[x] = min(nt0[l], nt0[r])
            nt1[x] = max(nt1[l], nt1[r])
    topo = dict(left=left, right=right, first=first, last=last, esc=esc, N=N)
    return (nlo, nhi, nt0, nt1, link, esc), topo


def check_topology(topo):
    N = topo["N"]
    if N == 1:
        assert topo["esc"][0] == END
        return
    left, right, first, last, esc = (topo[k] for k in ("left", "right", "first", "last", "esc"))
    parent = {}
    for i in range(N - 1):
        for c in (int(left[i]), int(right[i])):
            assert c not in parent, "node has two parents"
            parent[c] = i
    assert len(parent) == 2 * N - 2 and 0 not in parent          # all but the root
    rng = lambda x: (x - (N - 1), x - (N - 1)) if x >= N - 1 else (first[x], last[x])
    assert rng(0) == (0, N - 1)
    for i in range(N - 1):
        a, b = rng(int(left[i])), rng(int(right[i]))
        assert a[0] == first[i] and b[1] == last[i] and a[1] + 1 == b[0]
    # skip links: next node in pre-order after the node's subtree
    pre, stack = [], [0]
    while stack:
        x = stack.pop()
        pre.append(x)
        if x < N - 1:
            stack += [int(right[x]), int(left[x])]
    size = {}
    for x in reversed(pre):
        size[x] = 1 if x >= N - 1 else 1 + size[int(left[x])] + size[int(right[x])]
    where = {x: k for k, x in enumerate(pre)}
    for x in pre:
        k = where[x] + size[x]
        want = pre[k] if k < len(pre) else END
        assert int(esc[x]) == want


CASES = [(kind, N, w) for kind in ("uniform", "identical", "disjoint", "line", "huge")
         for N in (1, 2, 3, 5, 17, 64, 65, 300) for w in (1, 7)] + \
        [("uniform", 1000, 3), ("uniform", 4097, 5), ("identical", 700, 1)]


@pytest.mark.parametrize("kind,N,w", CASES)
def test_host_walk_matches_oracle(kind, N, w):
    lo, hi, t0, t1, obj = catalog.random_boxes(N * 7 + len(kind), N, max(2, N // 3),
                                               extent=40, size=6, T=30, max_len=8, kind=kind)
    nodes, topo = build_host_tree(lo, hi, t0, t1, obj, w)
    check_topology(topo)
    L = _lib()
    nlo, nhi, nt0, nt1, link, esc = (np.ascontiguousarray(a) for a in nodes)
    cap = N * N + 16
    out = np.zeros((cap, 4), np.uint32)
    cnt = L.hc_traverse(N, _p(nlo), _p(nhi), _p(nt0), _p(nt1), _p(link), _p(esc), w, _p(out), cap)
    assert cnt >= 0, "walk did not terminate"
    got = np.unique(out[:cnt], axis=0) if cnt else np.zeros((0, 4), np.uint32)
    ref = oracle.pairs(oracle.Boxes(lo, hi, t0, t1, obj))
    assert np.array_equal(got, ref)


def test_host_walk_on_orbital_boxes():
    sc = catalog.scaled(catalog.small_leo(seed=5, n=200, planted=8), horizon_ticks=60_000)
    b = oracle.boxes(sc.elements, sc.dt_ticks, sc.horizon_ticks, sc.tick_s, sc.threshold_km)
    nodes, topo = build_host_tree(b.lo, b.hi, b.t0, b.t1, b.obj, sc.dt_ticks)
    check_topology(topo)
    L = _lib()
    nlo, nhi, nt0, nt1, link, esc = (np.ascontiguousarray(a) for a in nodes)
    N = len(b)
    out = np.zeros((100000, 4), np.uint32)
    cnt = L.hc_traverse(N, _p(nlo), _p(nhi), _p(nt0), _p(nt1), _p(link), _p(esc),
                        sc.dt_ticks, _p(out), 100000)
    ref = oracle.pairs(b)
    assert len(ref) > 0
    # an object's tags partition time, so every record comes from one box pair:
    # the walk reports each unordered pair exactly once
    assert cnt == len(ref)
    assert np.array_equal(np.unique(out[:cnt], axis=0), ref)


def node_pair_pairs(nodes, topo):
    """The node-pair self-traversal in plain Python over a host-built tree:
    seeds = overlapping sibling pairs, expanded level by level."""
    nlo, nhi, nt0, nt1, link, esc = nodes
    N = topo["N"]
    left, right = topo["left"], topo["right"]

    def ov(a, c):
        return (nt0[a] < nt1[c] and nt0[c] < nt1[a] and np.all(nlo[a] <= nhi[c])
                and np.all(nlo[c] <= nhi[a]))
    level = [(int(left[p]), int(right[p])) for p in range(N - 1)
             if ov(int(left[p]), int(right[p]))]
    recs, levels = [], 0
    while level:
        nxt = []
        for a, c in level:
            A = [a] if a >= N - 1 else [int(left[a]), int(right[a])]
            C = [c] if c >= N - 1 else [int(left[c]), int(right[c])]
            for x in A:
                for y in C:
                    if not ov(x, y):
                        continue
                    if x >= N - 1 and y >= N - 1:
                        if link[x] != link[y]:
                            o1, o2 = sorted((int(link[x]), int(link[y])))
                            recs.append((o1, o2, max(nt0[x], nt0[y]), min(nt1[x], nt1[y])))
                    else:
                        nxt.append((x, y))
        level, levels = nxt, levels + 1
    return recs, levels


@pytest.mark.parametrize("kind,N,w", [("uniform", 300, 7), ("identical", 65, 1), ("huge", 500, 3),
                                      ("line", 257, 1), ("uniform", 2, 1), ("uniform", 1, 1)])
def test_node_pair_traversal_matches_oracle(kind, N, w):
    lo, hi, t0, t1, obj = catalog.random_boxes(N + 3, N, max(2, N // 3), extent=40, size=6,
                                               T=30, max_len=8, kind=kind)
    nodes, topo = build_host_tree(lo, hi, t0, t1, obj, w)
    recs, _ = node_pair_pairs(nodes, topo) if N > 1 else ([], 0)
    got = np.unique(np.array(recs, np.uint32).reshape(-1, 4), axis=0)
    ref = oracle.pairs(oracle.Boxes(lo, hi, t0, t1, obj))
    assert np.array_equal(got, ref)


def test_node_pair_traversal_reports_each_box_pair_once():
    sc = catalog.scaled(catalog.small_leo(seed=5, n=200, planted=8), horizon_ticks=60_000)
    b = oracle.boxes(sc.elements, sc.dt_ticks, sc.horizon_ticks, sc.tick_s, sc.threshold_km)
    nodes, topo = build_host_tree(b.lo, b.hi, b.t0, b.t1, b.obj, sc.dt_ticks)
    recs, levels = node_pair_pairs(nodes, topo)
    ref = oracle.pairs(b)
    assert len(recs) == len(ref) > 0
    assert np.array_equal(np.unique(np.array(recs, np.uint32), axis=0), ref)


def _topology(fn, keys, *extra):
    N = len(keys)
    out = [np.zeros(max(N - 1, 1), np.uint32), np.zeros(max(N - 1, 1), np.uint32),
           np.zeros(max(N - 1, 1), np.int64), np.zeros(max(N - 1, 1), np.int64),
           np.zeros(max(N - 1, 1), np.uint32), np.zeros(N, np.uint32)]
    assert fn(_p(keys), N, *extra, *[_p(a) for a in out]) == 0
    return out


@pytest.mark.parametrize("seed,N,bits,slab", [(0, 2, 30, 0), (1, 1000, 8, 0), (2, 5000, 40, 0),
                                              (3, 20000, 64, 0), (4, 3000, 4, 300),
                                              (5, 4000, 30, 1), (6, 6000, 30, 2),
                                              (7, 17408 * 2, 30, 17408), (8, 900, 2, 3)])
def test_32bit_views_give_the_64bit_topology(seed, N, bits, slab):
    """The kernels' Karras passes run in 32-bit position arithmetic, over the
    64-bit keys or over one time-major slab's 32-bit codes (slab bits taken
    from the position): same children, ranges and skip links as the 64-bit
    reference, also with many equal keys and with one- and two-key slabs."""
    L = _lib()
    vp = ctypes.c_void_p
    L.hc_karras32.argtypes = [vp, ctypes.c_int64, ctypes.c_uint32, vp, vp, vp, vp, vp, vp]
    rng = np.random.default_rng(seed)
    if slab:
        codes = rng.integers(0, 1 << bits, N, dtype=np.uint64) if bits < 64 else \
            rng.integers(0, 1 << 30, N, dtype=np.uint64)
        codes = np.sort(codes.reshape(N // slab, slab), axis=1).ravel()
        keys = (np.repeat(np.arange(N // slab, dtype=np.uint64), slab) << np.uint64(32)) | codes
    else:
        hi = (1 << bits) - 1 if bits < 64 else (1 << 63) - 1
        keys = np.sort(rng.integers(0, hi, N, dtype=np.uint64, endpoint=True))
    keys = np.ascontiguousarray(keys)
    ref = _topology(L.hc_karras, keys)
    got = _topology(L.hc_karras32, keys, slab)
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("seed,N,bits,slab,chunk", [
    (0, 1, 30, 1, 1024), (1, 2, 30, 1, 1024), (2, 3, 30, 3, 1024), (3, 1000, 8, 1000, 1024),
    (4, 1024, 30, 512, 1024), (5, 1025, 30, 25, 1024), (6, 3000, 4, 300, 1024),
    (7, 4000, 30, 1, 1024), (8, 6000, 30, 2, 512), (9, 17408 * 3, 30, 17408, 1024),
    (10, 16848 * 20, 30, 16848, 1024), (11, 900, 2, 3, 64), (12, 70000, 1, 7000, 256),
    (13, 16384 * 17 + 5, 30, 16384 * 17 + 5, 1024)])
def test_bottom_up_build_gives_the_karras_tree(seed, N, bits, slab, chunk):
    """The bottom-up build (one pass that finds each node's parent from the
    keys next to its range, and meets its sibling at their split) replayed on
    the CPU with the kernels' chunk and level structure, lanes in shuffled
    orders: its key-window reads stay in bounds, every meeting finds the
    sibling's box where the kernel looks for it, every level meeting's count
    was cleared, and the tree (children, skip links, leaf skip links) is the
    top-down Karras tree over the same keys, also with many equal codes, one-
    to three-key slabs, and sizes that reach level 2 of the queued passes."""
    L = _lib()
    vp = ctypes.c_void_p
    L.hc_agglo.argtypes = [vp, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                           vp, vp, vp, vp]
    rng = np.random.default_rng(seed)
    codes = rng.integers(0, 1 << bits, N, dtype=np.uint64)
    codes = np.sort(codes.reshape(N // slab, slab), axis=1).ravel()
    keys = np.ascontiguousarray(
        (np.repeat(np.arange(N // slab, dtype=np.uint64), slab) << np.uint64(32)) | codes)
    ref = _topology(L.hc_karras, keys)
    c32 = np.ascontiguousarray(codes.astype(np.uint32))
    for order_seed in (1, 2):
        left = np.zeros(max(N - 1, 1), np.uint32)
        right, esc_in = np.zeros_like(left), np.zeros_like(left)
        esc_leaf = np.zeros(N, np.uint32)
        rc = L.hc_agglo(_p(c32), N, slab, chunk, order_seed, _p(left), _p(right), _p(esc_in),
                        _p(esc_leaf))
        assert rc == 0
        assert np.array_equal(left[:N - 1], ref[0][:N - 1])
        assert np.array_equal(right[:N - 1], ref[1][:N - 1])
        assert np.array_equal(esc_in[:N - 1], ref[4][:N - 1])
        assert np.array_equal(esc_leaf, ref[5])
