"""Helpers shared by the GPU parity tests (not collected by pytest)."""
import sys

import numpy as np


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def need_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a HIP device"


def run_catalog(sc, box_precision=0, tree_precision=0, dt_array=None, capacity=None,
                box_rule=0):
    """Boxes, tree and canonical pairs for a scenario on the GPU."""
    import torch
    import paper_1901_10475_amd as cd
    el = cd.soa(sc.elements)
    p = cd.params_struct(sc.tick_s, sc.mu, sc.threshold_km, sc.horizon_ticks,
                         sc.dt_ticks if np.ndim(sc.dt_ticks) == 0 else 0, box_rule=box_rule)
    dt = None
    if dt_array is not None:
        dt = torch.from_numpy(np.asarray(dt_array, np.uint32).view(np.int32)).cuda()
    bp = cd.BroadPhase(sc.n, p, dt, box_precision, tree_precision, capacity=capacity)
    pairs = bp.run(el)
    torch.cuda.synchronize()
    return bp, pairs.cpu().numpy().view(np.uint32).copy()


def gpu_to_object_major(obj, n, K):
    """Index map: oracle box (i, k) at i*K + k  ->  its time-major GPU machine (slab
    k at [k n, (k + 1) n), in whatever order the layout put the slab's
    objects; obj = the GPU machines' object ids)."""
    obj = np.asarray(obj, np.int64)
    slab = np.arange(n * K, dtype=np.int64) // n
    key = obj * K + slab
    g = np.empty(n * K, np.int64)
    g[key] = np.arange(n * K, dtype=np.int64)
    return g


def slab_positions(obj, n):
    """pos[k * n + i] = index of object i's box in slab k (time-major boxes
    in any per-slab order); obj may be a numpy array or a device tensor."""
    import torch
    if isinstance(obj, torch.Tensor):
        o = obj.long()
        N = o.numel()
        b = torch.arange(N, device=o.device)
        pos = torch.empty(N, dtype=torch.long, device=o.device)
        pos[(b // n) * n + o] = b
        return pos
    o = np.asarray(obj, np.int64)
    b = np.arange(len(o), dtype=np.int64)
    pos = np.empty(len(o), np.int64)
    pos[(b // n) * n + o] = b
    return pos


def assert_boxes_close(g_lo, g_hi, o_lo, o_hi, a_obj):
    """|gpu - cpu| <= 1e-9 * max(|cpu|, a) per coordinate (a = semi-major axis)."""
    scale = np.maximum(np.maximum(np.abs(o_lo), np.abs(o_hi)), a_obj[:, None])
    dlo = np.abs(g_lo - o_lo) / scale
    dhi = np.abs(g_hi - o_hi) / scale
    worst = max(dlo.max(initial=0.0), dhi.max(initial=0.0))
    assert worst <= 1e-9, f"box bounds differ by {worst:.3e} (relative)"
    return worst


def records_of_boxes(recs, obj, t0, t1, sample):
    """GPU records that involve sampled box s: object obj[s] on either side and
    t_lo inside the box's tag (an object's tags partition time)."""
    keep = np.zeros(len(recs), bool)
    for s in sample:
        o, a, b = obj[s], t0[s], t1[s]
        keep |= ((recs[:, 0] == o) | (recs[:, 1] == o)) & (recs[:, 2] >= a) & (recs[:, 2] < b)
    return recs[keep]


def device_boxes_to_oracle(boxes, idx=None, lo_hi=None):
    """Boxes of a device box set (``Boxes`` or the batch runner's arrays) as
    oracle.Boxes with float64 bounds: all of them, the index tensor idx, or
    the range lo_hi = (a, b)."""
    import oracle
    lo, hi, t0, t1, obj = boxes
    if lo_hi is not None:
        a, b = lo_hi
        sel = slice(a, b)
        take = lambda x: x[..., sel]
    elif idx is not None:
        take = lambda x: x.index_select(x.dim() - 1, idx)
    else:
        take = lambda x: x
    u = lambda t: take(t).cpu().numpy().view(np.uint32)
    f = lambda t: np.ascontiguousarray(take(t).T.double().cpu().numpy())
    return oracle.Boxes(f(lo), f(hi), u(t0), u(t1), u(obj))


def arrays_of(bp_boxes):
    """(lo [3,N], hi [3,N], t0, t1, obj) device tensors cut to the box count."""
    N = bp_boxes.count
    return (bp_boxes.lo[:, :N], bp_boxes.hi[:, :N], bp_boxes.t0[:N], bp_boxes.t1[:N],
            bp_boxes.obj[:N])


def window_index(arrays, ta, tb):
    """Device indices of the boxes whose tags meet the ticks [ta, tb)."""
    import torch
    _, _, t0, t1, _ = arrays
    return torch.nonzero((t0 < tb) & (t1 > ta)).flatten()
