"""Learned per-object step: training driver for the step network.

The paper lets every object keep its own time interval, so that an object far
from all others can take long intervals and be processed rarely (Sec.
Collision Detection with 4D AABB Trees; Procedure advanceTime), but gives no
rule for the step itself beyond doubling it while the object meets nobody.
The library's network (``cd_dt_mlp``, a 5 -> 64 -> 64 -> 1 ReLU regressor of
log2(step)) predicts each object's step from its orbital elements.  Every step
keeps the boxes conservative, so the network changes the cost of a query,
never its correctness.

Training targets come from step sweeps run through the library itself: for a
catalog, every object gets the speed-bound step for a displacement bound
s * disp_km, for each scale s of a sweep, and each sweep point is one full
query.  An object's cost at scale s is

    C_i(s) = K_i(s) + pair_weight * R_i(s) + node_weight * V_i(s)

with K_i its number of intervals (its boxes: build, sort and refit work), R_i
the number of candidate records naming it (work handed to the narrow phase,
where each candidate is refined by repeated halving of its interval) and V_i
the traversal's box tests with one of its boxes on a side (counted by the
library built with CD_COUNTERS; node_weight = 0 leaves the term out).
Counts of single objects are small and noisy, so the target is not the
arg-min of the measured C_i but of a cost model fitted to the whole sweep:
K_i(s) = K_i(1) / s, R_i(s) = r_i s^q and V_i(s) = v_i s^u, the exponents q
and u fitted to the catalog's totals (least squares in log-log) and r_i, v_i
the pooled rates sum_s R_i(s) / sum_s s^q and sum_s V_i(s) / sum_s s^u (the
maximum-likelihood rates of Poisson counts with those means).  Without the
test term the model's minimum is

    s_i* = (K_i(1) / (pair_weight q r_i))^(1 / (q + 1));

with it, s_i* is the minimum over a grid of 512 scales spaced evenly in
log s across the sweep's range.  s_i* is clamped to the sweep's range (its
largest scale when r_i = 0 and v_i = 0), and the target is log2 of the step
s_i* dt_i(1), in seconds.

The default node_weight is the measured cost of one executed traversal test
over that of one box (boxes, keys, sort, hierarchy and unions) on the path
the network serves -- FP32 boxes and tree with per-object steps, here the
16 848-object hour with learned steps and the eccentric-anomaly box: 1.89 ms
for 7.87 M boxes (240 ps each) against 1.01 ms for the traversal's 38.9 M
tests (26 ps each).  (On the uniform-step FP64 path a box is cheaper, 72 ps
against 45 ps per test; that ratio, 0.6, trains steps that make the learned
queries slower.)

Everything numeric runs in the library's kernels (features, forward, backward,
Adam, record counts, the broad phase); this module sequences the calls and
keeps the buffers.
"""
import ctypes
import math

import numpy as np
import torch

from . import (CD_FP32, CD_FP64, BroadPhase, _bytes, _check, _ptr, _stream, cd_counters_reset,
               cd_dt_heuristic, counters_build, elements_struct, lib)

CD_MLP_PARAMS = 4609
DEFAULT_SCALES = (0.25, 0.5, 1.0, 2.0, 4.0, 8.0, 16.0, 32.0, 64.0)
PAIR_WEIGHT = 32.0
NODE_WEIGHT = 0.1


# ---- marshalled C calls --------------------------------------------------------------

def _need(t, dtype, numel, what):
    if t is None:
        return
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous() and t.numel() >= numel):
        raise ValueError(f"{what}: need a contiguous {dtype} CUDA tensor of >= {numel} values")


def _need_w(w, dtype=torch.float32, what="weights"):
    if not (w.is_cuda and w.dtype == dtype and w.is_contiguous() and w.numel() == CD_MLP_PARAMS):
        raise ValueError(f"{what}: need a contiguous {dtype} CUDA tensor of {CD_MLP_PARAMS}")


def _need_x(x):
    if not (x.is_cuda and x.dtype == torch.float32 and x.dim() == 2 and x.shape[1] == 5
            and x.is_contiguous()):
        raise ValueError("x: need a contiguous float32 CUDA tensor [B, 5]")


def cd_mlp_features(el_soa, params):
    """[n, 5] float32 features of every object (computed in FP64)."""
    el = elements_struct(el_soa)
    x = torch.empty((max(el.n, 1), 5), dtype=torch.float32, device=el_soa.device)
    _check(lib().cd_mlp_features(ctypes.byref(el), ctypes.byref(params), _ptr(x), _stream()))
    return x[:el.n]


def cd_dt_mlp(el_soa, w_bf16, fallback_disp_km, params, dt_out, y_out=None):
    """BF16 inference into dt_out (int32 tensor [n]); y_out (float32 [n]) optional.
    w_bf16: int16 tensor [CD_MLP_PARAMS] of bfloat16 bit patterns, or None."""
    el = elements_struct(el_soa)
    _need(dt_out, torch.int32, el.n, "dt_out")
    _need(y_out, torch.float32, el.n, "y_out")
    if w_bf16 is not None:
        _need_w(w_bf16, torch.int16, "w_bf16")
    _check(lib().cd_dt_mlp(ctypes.byref(el), _ptr(w_bf16) if w_bf16 is not None else None,
                           float(fallback_disp_km), ctypes.byref(params), _ptr(dt_out),
                           _ptr(y_out) if y_out is not None else None, _stream()))


def cd_mlp_forward(w, x):
    _need_w(w)
    _need_x(x)
    B = int(x.shape[0])
    y = torch.empty(max(B, 1), dtype=torch.float32, device=x.device)
    _check(lib().cd_mlp_forward(_ptr(w), _ptr(x), B, _ptr(y), _stream()))
    return y[:B]


def cd_mlp_grad(w, x, target, ws=None):
    """(grad [CD_MLP_PARAMS] float32, loss [1] float32) of the mean squared error."""
    _need_w(w)
    _need_x(x)
    B = int(x.shape[0])
    _need(target, torch.float32, B, "target")
    if ws is None:
        ws = _bytes(lib().cd_mlp_grad_ws(B), x.device)
    g = torch.empty(CD_MLP_PARAMS, dtype=torch.float32, device=x.device)
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    _check(lib().cd_mlp_grad(_ptr(w), _ptr(x), _ptr(target), B, _ptr(g), _ptr(loss), _ptr(ws),
                             ws.numel(), _stream()))
    return g, loss


def cd_mlp_adam(w, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, w_bf16=None):
    for t, name in ((w, "w"), (m, "m"), (v, "v"), (g, "g")):
        _need_w(t, what=name)
    if w_bf16 is not None:
        _need_w(w_bf16, torch.int16, "w_bf16")
    _check(lib().cd_mlp_adam(_ptr(w), _ptr(m), _ptr(v), _ptr(g), int(step), float(lr),
                             float(beta1), float(beta2), float(eps),
                             _ptr(w_bf16) if w_bf16 is not None else None, _stream()))


def cd_pair_object_counts(pairs, n):
    """int32 tensor [n]: records naming each object (as i or j)."""
    if not (pairs.is_cuda and pairs.dtype == torch.int32 and pairs.dim() == 2
            and pairs.shape[1] == 4 and pairs.is_contiguous()):
        raise ValueError("pairs: need a contiguous int32 CUDA tensor [P, 4]")
    counts = torch.empty(max(int(n), 1), dtype=torch.int32, device=pairs.device)
    _check(lib().cd_pair_object_counts(_ptr(pairs), int(pairs.shape[0]), int(n), _ptr(counts),
                                       _stream()))
    return counts[:int(n)]


# ---- the trainer --------------------------------------------------------------------

def init_weights(seed):
    """He-uniform weights, zero biases (flat FP32 vector, host)."""
    rng = np.random.default_rng(seed)
    parts = [rng.uniform(-1, 1, 64 * 5) * math.sqrt(6.0 / 5), np.zeros(64),
             rng.uniform(-1, 1, 64 * 64) * math.sqrt(6.0 / 64), np.zeros(64),
             rng.uniform(-1, 1, 64) * math.sqrt(6.0 / 64), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)


class StepNet:
    """FP32 master weights and Adam moments on the device, with the BF16 copy
    that inference reads kept current by every Adam step."""

    def __init__(self, seed=0, device="cuda", weights=None):
        w = init_weights(seed) if weights is None else np.asarray(weights, np.float32)
        assert w.shape == (CD_MLP_PARAMS,)
        self.device = device
        self.w = torch.from_numpy(w.copy()).to(device)
        self.m = torch.zeros(CD_MLP_PARAMS, dtype=torch.float32, device=device)
        self.v = torch.zeros_like(self.m)
        self.w_bf16 = torch.empty(CD_MLP_PARAMS, dtype=torch.int16, device=device)
        self.step = 0
        self._export()

    def _export(self):
        # an Adam call with zero gradient and zero rate leaves w, m and v as
        # they are and writes the BF16 copy
        zero = torch.zeros_like(self.m)
        m, v = torch.zeros_like(self.m), torch.zeros_like(self.m)
        cd_mlp_adam(self.w, m, v, zero, 1, 0.0, w_bf16=self.w_bf16)

    def set_output_bias(self, b3):
        """Start from a constant prediction (e.g. the mean target)."""
        self.w[CD_MLP_PARAMS - 1] = float(b3)
        self._export()

    def train(self, x, target, steps, lr=3e-3, lr_end=None, log_every=0):
        """Full-batch Adam on the mean squared error; returns the loss history
        (one value per step, read back once at the end)."""
        x = x.contiguous()
        target = target.contiguous().float()
        ws = _bytes(lib().cd_mlp_grad_ws(int(x.shape[0])), x.device)
        losses = torch.empty(steps, dtype=torch.float32, device=x.device)
        lr_end = lr if lr_end is None else lr_end
        for k in range(steps):
            g, loss = cd_mlp_grad(self.w, x, target, ws)
            losses[k:k + 1].copy_(loss)
            self.step += 1
            rate = lr * (lr_end / lr) ** (k / max(steps - 1, 1))   # geometric decay
            cd_mlp_adam(self.w, self.m, self.v, g, self.step, rate, w_bf16=self.w_bf16)
            if log_every and (k % log_every == 0 or k == steps - 1):
                print(f"[step-net] step {k}: loss {losses[k].item():.5f}", flush=True)
        return losses.cpu().numpy()

    def predict(self, x):
        return cd_mlp_forward(self.w, x.contiguous())

    def dt(self, el_soa, params, fallback_disp_km=5.0, y_out=None):
        n = el_soa.shape[1]
        dt = torch.empty(max(n, 1), dtype=torch.int32, device=el_soa.device)
        cd_dt_mlp(el_soa, self.w_bf16, fallback_disp_km, params, dt, y_out)
        return dt[:n]


# ---- targets from step sweeps ----------------------------------------------------------

def intervals_of(dt, horizon_ticks):
    """K_i = max(1, ceil(T / dt_i)) as an int64 tensor."""
    T = int(horizon_ticks)
    d = dt.long()
    return torch.clamp((T + d - 1) // d, min=1) if T > 0 else torch.ones_like(d)


def _run(el_soa, params, dt, visits_too, box_precision, tree_precision):
    """One query with per-object steps dt: (pairs, per-object record counts,
    per-object test counts or None, boxes)."""
    n = el_soa.shape[1]
    bp = BroadPhase(n, params, dt_ticks=dt, box_precision=box_precision,
                    tree_precision=tree_precision)
    visits = None
    if visits_too:
        visits = torch.zeros(n, dtype=torch.int32, device=el_soa.device)
        with counters_build():
            cd_counters_reset(visits)
            try:
                pairs = bp.run(el_soa)
            finally:
                cd_counters_reset(None)   # unbind before the tensor goes
    else:
        pairs = bp.run(el_soa)
    return pairs, cd_pair_object_counts(pairs, n), visits, bp.count


def run_costs(el_soa, params, dt, pair_weight=PAIR_WEIGHT, node_weight=NODE_WEIGHT,
              box_precision=CD_FP32, tree_precision=CD_FP32):
    """One query with per-object steps dt: (per-object cost, records, boxes, pairs)."""
    pairs, counts, visits, boxes = _run(el_soa, params, dt, node_weight > 0, box_precision,
                                        tree_precision)
    K = intervals_of(dt, params.horizon_ticks)
    cost = K.double() + pair_weight * counts.double()
    if visits is not None:
        cost += node_weight * visits.double()
    return cost, counts, boxes, pairs


def _growth(scales, totals, lo, hi):
    """Exponent of a count's growth with the scale: least squares in log-log
    over the catalog totals, clamped to [lo, hi]."""
    if len(scales) < 2:
        return 1.0
    tot = np.maximum(np.asarray(totals, dtype=np.float64), 1.0)
    x = float(np.polyfit(np.log(scales), np.log(tot), 1)[0])
    return min(max(x, lo), hi)


def sweep_targets(el_soa, params, scales=DEFAULT_SCALES, disp_km=5.0, pair_weight=PAIR_WEIGHT,
                  node_weight=NODE_WEIGHT, box_precision=CD_FP32, tree_precision=CD_FP32):
    """(features [n,5], target log2 seconds [n], per-scale summary)."""
    n = el_soa.shape[1]
    scales = sorted(float(s) for s in scales)
    counts, visits = [], []
    summary = []
    dt1 = torch.empty(n, dtype=torch.int32, device=el_soa.device)
    cd_dt_heuristic(el_soa, params, disp_km, dt1)
    for s in scales:
        dt = torch.empty(n, dtype=torch.int32, device=el_soa.device)
        cd_dt_heuristic(el_soa, params, disp_km * s, dt)
        pairs, c, v, boxes = _run(el_soa, params, dt, node_weight > 0, box_precision,
                                  tree_precision)
        cost = intervals_of(dt, params.horizon_ticks).double() + pair_weight * c.double()
        if v is not None:
            cost += node_weight * v.double()
            visits.append(v.double())
        summary.append({"scale": s, "boxes": int(boxes), "records": int(pairs.shape[0]),
                        "tests": int(v.sum().item()) if v is not None else None,
                        "cost": float(cost.sum().item())})
        counts.append(c.double())
        del pairs
    q = _growth(scales, [r["records"] for r in summary], 0.25, 4.0)
    rate = torch.stack(counts).sum(dim=0) / sum(s ** q for s in scales)
    K1 = intervals_of(dt1, params.horizon_ticks).double()
    s_lo, s_hi = scales[0], scales[-1]
    if not visits:
        s_star = torch.where(
            rate > 0, (K1 / (pair_weight * q * rate.clamp(min=1e-30))) ** (1.0 / (q + 1.0)),
            torch.full_like(K1, s_hi)).clamp(s_lo, s_hi)
        u = None
    else:
        # V_i counts the tests of every box of object i; with fewer, longer
        # boxes it may fall or grow, so u may take either sign
        u = _growth(scales, [r["tests"] for r in summary], -4.0, 4.0)
        vrate = torch.stack(visits).sum(dim=0) / sum(s ** u for s in scales)
        grid = torch.logspace(math.log2(s_lo), math.log2(s_hi), 512, base=2.0,
                              dtype=torch.float64, device=K1.device)
        s_star = torch.empty_like(K1)
        for a in range(0, n, 8192):   # rows of objects x grid scales
            b = min(n, a + 8192)
            C = (K1[a:b, None] / grid + pair_weight * rate[a:b, None] * grid ** q
                 + node_weight * vrate[a:b, None] * grid ** u)
            s_star[a:b] = grid[torch.argmin(C, dim=1)]
    target = torch.log2(s_star * dt1.double() * params.tick_s).float()
    for r in summary:
        r["q"] = q
        r["u"] = u
    return cd_mlp_features(el_soa, params), target, summary
