"""Tree invariants on the GPU, checked on the tree buffer itself, apart from
any query: the leaves are the input boxes (outward-rounded for an FP32 tree),
every inner box is the exact union of its children's boxes in space and time
(the refit of the bottom-up pass), every node but the root is the child of
exactly one inner node, the link and skip records walk every node once in
depth-first pre-order, and the seed list holds exactly the sibling pairs whose
boxes overlap (closed extents in space, half-open tags in time).

Covered: uniform steps, where the boxes of each interval form one slab --
in object order, which one workgroup sorts in LDS per slab before the
top-down Karras pass and the chunked refit (slabs of 1, 2, 300 and 17 408
boxes, the largest one workgroup sorts, and 70 000 slabs of 3; 17 409
objects per interval take the device-wide sort and the bottom-up pass
instead); in the sorted layout as box arrays (no sort; the bottom-up pass
reads box j as leaf j) or as the tree's own leaf records (the bottom-up pass
over the records in place; up to 16 sorted runs merged per block);
per-object steps (one radix sort of all keys, then the bottom-up pass reads
the boxes through the sorted items); FP64 and FP32 trees; boxes with and
without Morton codes.

Tree buffer layout read here: a 256-byte header (error bits, seed count, seed
overflow), the node records (FP64: 64 bytes each, lo[3], hi[3] as doubles, then
t0, t1, link, esc as uint32; FP32: 32-byte boxes with float lo/hi and t0, t1,
then 8-byte (link, esc) records), kids[N - 1] (left, right) and the seeds.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1901_10475_amd as cd
from paper_1901_10475_amd import catalog
from tests.gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu
END = 0xFFFFFFFF


def _decode(tree, N, prec):
    raw = tree.mem.cpu().numpy().view(np.uint8)
    hdr = raw[:256].view(np.uint32)
    nn = 2 * N - 1
    if prec == cd.CD_FP64:
        rec = raw[256:256 + nn * 64].reshape(nn, 64)
        lo = rec[:, 0:24].copy().view(np.float64)
        hi = rec[:, 24:48].copy().view(np.float64)
        tags = rec[:, 48:64].copy().view(np.uint32)
        t0, t1, link, esc = tags[:, 0], tags[:, 1], tags[:, 2], tags[:, 3]
        kids_off = 256 + nn * 64
    else:
        box = raw[256:256 + nn * 32].reshape(nn, 32)
        lo = box[:, 0:12].copy().view(np.float32).astype(np.float64)
        hi = box[:, 12:24].copy().view(np.float32).astype(np.float64)
        tg = box[:, 24:32].copy().view(np.uint32)
        t0, t1 = tg[:, 0], tg[:, 1]
        lk = raw[256 + nn * 32:256 + nn * 40].copy().view(np.uint32).reshape(nn, 2)
        link, esc = lk[:, 0], lk[:, 1]
        kids_off = 256 + nn * 40
    kids = raw[kids_off:kids_off + (N - 1) * 8].copy().view(np.uint32).reshape(N - 1, 2)
    seeds_off = kids_off + max(N - 1, 1) * 8
    ns = int(hdr[1])
    ns = min(ns, N // 4 + 4096)
    seeds = raw[seeds_off:seeds_off + ns * 8].copy().view(np.uint32).reshape(ns, 2)
    if prec == cd.CD_FP64 and hdr[3]:
        # leaf records written in place by the box build: the leaves' skip
        # links are in the side array after the seeds (the records hold codes)
        side_off = seeds_off + (N // 4 + 4096) * 8
        esc = esc.copy()
        esc[N - 1:] = raw[side_off:side_off + 4 * N].copy().view(np.uint32)
    return dict(err=int(hdr[0]), overflow=int(hdr[2]), lo=lo, hi=hi, t0=t0, t1=t1, link=link,
                esc=esc, kids=kids.astype(np.int64), seeds=seeds)


def _round_out(lo, hi):
    f_lo, f_hi = lo.astype(np.float32), hi.astype(np.float32)
    f_lo = np.where(f_lo.astype(np.float64) > lo, np.nextafter(f_lo, np.float32(-np.inf)), f_lo)
    f_hi = np.where(f_hi.astype(np.float64) < hi, np.nextafter(f_hi, np.float32(np.inf)), f_hi)
    return f_lo.astype(np.float64), f_hi.astype(np.float64)


def check_tree(bp):
    N, prec = bp.count, bp.tree_precision
    torch.cuda.synchronize()
    t = _decode(bp.tree, N, prec)
    assert t["err"] == 0
    lo, hi, t0, t1, kids = t["lo"], t["hi"], t["t0"], t["t1"], t["kids"]
    # leaves: the input boxes, in some order
    b = bp.boxes
    blo = b.lo[:, :N].cpu().numpy().T.astype(np.float64)
    bhi = b.hi[:, :N].cpu().numpy().T.astype(np.float64)
    if prec == cd.CD_FP32 and b.precision == cd.CD_FP64:
        blo, bhi = _round_out(blo, bhi)
    bt0 = b.t0[:N].cpu().numpy().view(np.uint32)
    bt1 = b.t1[:N].cpu().numpy().view(np.uint32)
    bob = b.obj[:N].cpu().numpy().view(np.uint32)
    want = np.column_stack([blo, bhi, bt0, bt1, bob])
    L = slice(N - 1, 2 * N - 1)
    got = np.column_stack([lo[L], hi[L], t0[L], t1[L], t["link"][L]])
    assert np.array_equal(want[np.lexsort(want.T[::-1])], got[np.lexsort(got.T[::-1])])
    if N == 1:
        return
    # every node but the root is a child exactly once
    seen = np.bincount(kids.ravel(), minlength=2 * N - 1)
    assert seen[0] == 0 and np.all(seen[1:] == 1)
    # exact unions, bottom-up definition checked top-down on every inner node
    l, r = kids[:, 0], kids[:, 1]
    I = slice(0, N - 1)
    assert np.array_equal(lo[I], np.minimum(lo[l], lo[r]))
    assert np.array_equal(hi[I], np.maximum(hi[l], hi[r]))
    assert np.array_equal(t0[I], np.minimum(t0[l], t0[r]))
    assert np.array_equal(t1[I], np.maximum(t1[l], t1[r]))
    assert np.array_equal(t["link"][I], l.astype(np.uint32))
    # pre-order walk by link (inner) and esc (leaf), and esc skips the subtree
    order, cur = [], 0
    while cur != END and len(order) <= 2 * N:
        order.append(cur)
        cur = int(t["link"][cur]) if cur < N - 1 else int(t["esc"][cur])
    assert len(order) == 2 * N - 1 and len(set(order)) == 2 * N - 1
    pos = np.empty(2 * N - 1, np.int64)
    pos[np.array(order)] = np.arange(2 * N - 1)
    size = np.ones(2 * N - 1, np.int64)
    for v in reversed(order):
        if v < N - 1:
            size[v] = 1 + size[kids[v, 0]] + size[kids[v, 1]]
    nxt = pos + size
    esc = t["esc"].astype(np.int64)
    has = nxt < 2 * N - 1
    assert np.all(esc[~has] == END)
    assert np.array_equal(pos[esc[has]], nxt[has])
    # seeds: exactly the overlapping sibling pairs
    ov = ((t0[l] < t1[r]) & (t0[r] < t1[l])
          & np.all(lo[l] <= hi[r], axis=1) & np.all(lo[r] <= hi[l], axis=1))
    want_s = {(int(a), int(c)) for a, c in zip(l[ov], r[ov])}
    got_s = {(int(a), int(c)) for a, c in t["seeds"]}
    assert len(got_s) == len(t["seeds"])
    if t["overflow"]:   # a full seed list holds some of them (the query then walks)
        assert got_s <= want_s
    else:
        assert got_s == want_s
    return len(want_s)


def _uniform(n, K, dt, seed=0, box_precision=cd.CD_FP64, tree_precision=cd.CD_FP64,
             codes=True, layout=cd.CD_LAYOUT_SORTED, in_tree=True, build=True):
    """n LEO objects, K intervals of dt one-second ticks, threshold 1 km."""
    rng = np.random.default_rng(seed)
    el = catalog.leo_mix(rng, n)
    p = cd.params_struct(1.0, catalog.MU_EARTH, 1.0, K * dt - 1, dt)
    bp = cd.BroadPhase(n, p, box_precision=box_precision, tree_precision=tree_precision,
                       codes=codes, layout=layout, in_tree=in_tree)
    bp.el_soa = cd.soa(el)
    if build:
        bp.build(bp.el_soa)
    return bp


@pytest.mark.parametrize("layout,in_tree", [(cd.CD_LAYOUT_OBJECT, False),
                                            (cd.CD_LAYOUT_SORTED, False),
                                            (cd.CD_LAYOUT_SORTED, True)])
@pytest.mark.parametrize("n,K", [(1, 50), (2, 40), (300, 60), (17408, 3), (17409, 3),
                                 (3, 70000), (257, 17)])
def test_uniform_step_trees(n, K, layout, in_tree):
    """Object order: the slab build sorts each slab; sorted layout: the boxes
    arrive in their slabs' Morton order and no sort runs, as arrays (the refit
    writes the leaf records; 17 409 objects per slab exceed one workgroup's
    sort and fall back to object order) or as the tree's own leaf records (up
    to 16 sorted runs of 17 408 merged per block)."""
    need_gpu()
    say("tree invariants, uniform steps, n", n, "K", K, "layout", layout, "in tree", in_tree)
    bp = _uniform(n, K, 2, seed=n, layout=layout, in_tree=in_tree)
    assert bp.count == n * K
    want = layout if n <= cd.CD_SORTED_MAX_ARRAYS or in_tree else cd.CD_LAYOUT_OBJECT
    assert bp.boxes.desc.layout == want
    assert bp.in_tree == (in_tree and want == cd.CD_LAYOUT_SORTED)
    say("seeds", check_tree(bp))


@pytest.mark.parametrize("layout", [cd.CD_LAYOUT_OBJECT, cd.CD_LAYOUT_SORTED])
@pytest.mark.parametrize("box_prec,tree_prec,codes", [(cd.CD_FP64, cd.CD_FP32, True),
                                                      (cd.CD_FP32, cd.CD_FP32, True),
                                                      (cd.CD_FP64, cd.CD_FP64, False)])
def test_uniform_step_tree_precisions(box_prec, tree_prec, codes, layout):
    need_gpu()
    say("tree invariants, precisions", box_prec, tree_prec, "codes", codes, "layout", layout)
    bp = _uniform(500, 40, 30, seed=7, box_precision=box_prec, tree_precision=tree_prec,
                  codes=codes, layout=layout, in_tree=False)
    assert bp.boxes.desc.layout == (layout if codes else cd.CD_LAYOUT_OBJECT)
    check_tree(bp)


@pytest.mark.parametrize("n,K", [(300, 60), (1000, 17), (1, 9), (16848, 20)])
def test_sorted_layout_order(n, K):
    """Sorted layout: every slab holds each object once; inside each block of 8
    slabs the order (and the codes) is the same in every slab and the codes
    are non-decreasing; the boxes and the record list equal the object
    layout's."""
    need_gpu()
    say("sorted layout, n", n, "K", K)
    a = _uniform(n, K, 2, seed=n + 5, layout=cd.CD_LAYOUT_OBJECT, in_tree=False)
    b = _uniform(n, K, 2, seed=n + 5, layout=cd.CD_LAYOUT_SORTED, in_tree=False)
    # the same boxes written as the tree's leaf records, read before the tree
    # build turns their code words into skip links
    c = _uniform(n, K, 2, seed=n + 5, layout=cd.CD_LAYOUT_SORTED, in_tree=True, build=False)
    assert c.in_tree
    cd.cd_build_boxes(c.el_soa, None, c.params, c.boxes, c.ws_boxes)
    assert c.boxes.desc.code_valid == 1 and c.boxes.desc.layout == cd.CD_LAYOUT_SORTED
    # the two store forms run one loop (and multiply-adds are fused only as
    # written), so they hold the same bits
    same_bits = True
    for arr in ("lo", "hi"):
        x, y = getattr(b.boxes, arr)[:, :n * K], getattr(c.boxes, arr)
        rel = ((x - y).abs() / x.abs().clamp(min=6000.0)).max().item()
        assert rel <= 1e-15, (arr, rel)
        same_bits &= bool(torch.equal(x, y))
    assert same_bits
    for arr in ("t0", "t1", "obj", "code"):
        assert torch.equal(getattr(b.boxes, arr)[:n * K], getattr(c.boxes, arr))
    cd.cd_build_tree(c.boxes, c.tree_precision, c.tree, c.ws_tree)
    check_tree(c)
    assert b.boxes.desc.layout == cd.CD_LAYOUT_SORTED and b.boxes.desc.code_valid == 1
    N = n * K
    obj = b.boxes.obj[:N].cpu().numpy().view(np.uint32).reshape(K, n)
    code = b.boxes.code[:N].cpu().numpy().view(np.uint32).reshape(K, n)
    assert np.all(np.sort(obj, axis=1) == np.arange(n)[None, :])
    assert np.all(np.diff(code.astype(np.int64), axis=1) >= 0)
    for k in range(K):
        k0 = (k // 8) * 8
        assert np.array_equal(obj[k], obj[k0]) and np.array_equal(code[k], code[k0])
    # same boxes, object by object
    oa = a.boxes.obj[:N].cpu().numpy().view(np.uint32).reshape(K, n)
    assert np.all(oa == np.arange(n)[None, :])
    inv = np.argsort(obj, axis=1) + (np.arange(K) * n)[:, None]
    for arr in ("lo", "hi"):
        ga = getattr(a.boxes, arr)[:, :N].cpu().numpy()
        gb = getattr(b.boxes, arr)[:, :N].cpu().numpy()
        assert np.array_equal(ga, gb[:, inv.ravel()])
    for arr in ("t0", "t1"):
        ga = getattr(a.boxes, arr)[:N].cpu().numpy()
        gb = getattr(b.boxes, arr)[:N].cpu().numpy()
        assert np.array_equal(ga, gb[inv.ravel()])
    ra = a.query().cpu().numpy()
    rb = b.query().cpu().numpy()
    rc = c.query().cpu().numpy().view(np.uint32)
    assert np.array_equal(ra, rb)
    if same_bits:
        assert np.array_equal(ra, rc)
    # the records of the in-place leaves against the oracle on those boxes
    lo, hi, t0, t1, obj = c.boxes.to_host()
    assert np.array_equal(rc, oracle.pairs_bucketed(oracle.Boxes(lo, hi, t0, t1, obj)))


@pytest.mark.parametrize("n,K", [(17409, 9), (20000, 9), (36001, 9), (20000, 16), (36001, 13)])
def test_sorted_layout_from_merged_runs(n, K):
    """More objects than one workgroup sorts: each block's codes are sorted in
    runs and merged by rank.  Every slab holds each object once, in
    non-decreasing code order with equal codes by object index, the same
    order in every slab of a block; the boxes and the record list equal the
    object layout's, and the records equal the oracle's on the in-place
    leaves.  9 slabs (a block of 8 and one of 1) keep the sort's scratch in
    the first slab's records; 16 and 13 slabs (last blocks of 8 and 5) keep
    it in the code array's entries of each block's first five slabs."""
    need_gpu()
    say("sorted layout from merged runs, n", n, "K", K)
    a = _uniform(n, K, 2, seed=n + 7, layout=cd.CD_LAYOUT_OBJECT, in_tree=False)
    c = _uniform(n, K, 2, seed=n + 7, layout=cd.CD_LAYOUT_SORTED, in_tree=True)
    assert c.in_tree and c.boxes.desc.layout == cd.CD_LAYOUT_SORTED
    check_tree(c)
    N = n * K
    obj = c.boxes.obj.cpu().numpy().view(np.uint32).reshape(K, n)
    code = c.boxes.code.cpu().numpy().view(np.uint32).reshape(K, n)
    assert np.all(np.sort(obj, axis=1) == np.arange(n)[None, :])
    key = (code.astype(np.int64) << 32) | obj.astype(np.int64)
    assert np.all(np.diff(key, axis=1) > 0)
    for k in range(K):
        k0 = (k // 8) * 8
        assert np.array_equal(obj[k], obj[k0]) and np.array_equal(code[k], code[k0])
    lo, hi, t0, t1, ob = c.boxes.to_host()
    inv = np.argsort(obj, axis=1) + (np.arange(K) * n)[:, None]
    for arr, got in (("lo", lo), ("hi", hi)):
        ga = getattr(a.boxes, arr)[:, :N].cpu().numpy()
        assert np.array_equal(ga.T, got[inv.ravel()])
    rc = c.query().cpu().numpy().view(np.uint32)
    assert np.array_equal(a.query().cpu().numpy().view(np.uint32), rc)
    assert np.array_equal(rc, oracle.pairs_bucketed(oracle.Boxes(lo, hi, t0, t1, ob)))
    say("records", len(rc))


def test_sorted_layout_with_unsorted_codes_is_reported():
    """Boxes that claim the sorted layout but whose codes are out of order in
    a slab: the tree build flags it and the query reports CD_E_INVALID."""
    need_gpu()
    b = _uniform(300, 16, 2, seed=3, layout=cd.CD_LAYOUT_SORTED, in_tree=False)
    c = b.boxes.code
    lo, hi = int(c[5 * 300].item()), int(c[5 * 300 + 299].item())
    assert lo < hi
    c[5 * 300] = hi
    c[5 * 300 + 299] = lo
    cd.cd_build_tree(b.boxes, b.tree_precision, b.tree, b.ws_tree)
    with pytest.raises(cd.CDError) as ei:
        cd.cd_query_pairs(b.tree, b.out, b.capacity, b.ws_query)
    assert ei.value.status == cd.CD_E_INVALID
    # records in place: a packed code out of order is reported the same way;
    # a record outside its slab is reported by the refit
    r = _uniform(300, 16, 2, seed=3, layout=cd.CD_LAYOUT_SORTED, in_tree=True)
    want = r.query().cpu().numpy()
    cd.cd_build_tree(r.boxes, r.tree_precision, r.tree, r.ws_tree)   # again: same list
    assert np.array_equal(r.query().cpu().numpy(), want)
    c = r.boxes.code
    lo, hi = int(c[7 * 300].item()), int(c[7 * 300 + 299].item())
    c[7 * 300], c[7 * 300 + 299] = hi, lo
    cd.cd_build_tree(r.boxes, r.tree_precision, r.tree, r.ws_tree)
    with pytest.raises(cd.CDError) as ei:
        cd.cd_query_pairs(r.tree, r.out, r.capacity, r.ws_query)
    assert ei.value.status == cd.CD_E_INVALID
    r.boxes.code[7 * 300], r.boxes.code[7 * 300 + 299] = lo, hi
    t0 = int(r.boxes.t0[5 * 300 + 17].item())
    r.boxes.t0[5 * 300 + 17] = t0 + 2          # one tick past its slab of 2 ticks
    cd.cd_build_tree(r.boxes, r.tree_precision, r.tree, r.ws_tree)
    with pytest.raises(cd.CDError) as ei:
        cd.cd_query_pairs(r.tree, r.out, r.capacity, r.ws_query)
    assert ei.value.status == cd.CD_E_INVALID


@pytest.mark.parametrize("box_prec,tree_prec", [(cd.CD_FP64, cd.CD_FP64),
                                                (cd.CD_FP64, cd.CD_FP32),
                                                (cd.CD_FP32, cd.CD_FP32)])
@pytest.mark.parametrize("horizon,disp_km,slab_ticks", [(3000, 20.0, 0), (200000, 2000.0, 1),
                                                      (1 << 22, 20000.0, 1)])
def test_per_object_step_tree(box_prec, tree_prec, horizon, disp_km, slab_ticks):
    """The general path: one device-wide key sort, then the bottom-up pass
    reading each leaf's box through the sorted items.  Slab, 30-bit code and
    box index fit one 64-bit word in the first case (8-byte sort items); with
    one-tick slabs over 200 000 ticks (18 slab bits) the word keeps the
    code's top 27 bits; over 2^22 ticks (23 slab bits) fewer than 24 would
    remain, so the third sorts 16-byte (key, index) items."""
    need_gpu()
    say(f"tree invariants, per-object steps, boxes {box_prec} tree {tree_prec}, "
        f"horizon {horizon}, slab ticks {slab_ticks}")
    rng = np.random.default_rng(11)
    el = catalog.leo_mix(rng, 400)
    p = cd.params_struct(1.0, catalog.MU_EARTH, 1.0, horizon, 0)
    bp = cd.BroadPhase(400, p, dt_heuristic_km=disp_km, el_soa=cd.soa(el),
                       box_precision=box_prec, tree_precision=tree_prec,
                       slab_ticks=slab_ticks)
    bp.build(cd.soa(el))
    N = bp.count
    max_slab = horizon // bp.tree.desc.slab_ticks
    room = 64 - max_slab.bit_length() - (N - 1).bit_length()
    assert (room >= 30, room >= 24) == {3000: (True, True), 200000: (False, True),
                                        1 << 22: (False, False)}[horizon], (N, room)
    check_tree(bp)
