"""GPU parity of the step network against the FP64 reference (oracle/mlp.py),
and what the trained network gains over the speed-bound step.

Tolerances (derived in the design notes):
  features      one FP32 rounding of the FP64 value (relative 2^-23);
  FP32 forward  |dy| <= 1e-5 max(1, |y|);
  FP32 gradient ||g - g_ref|| <= 1e-5 ||g_ref||, loss to 1e-5 relative;
  Adam          |dw| <= 1e-6 max(1, |w|), BF16 copy bit-exact from the FP32 w;
  BF16 forward  within 5e-3 max(1, |y|) of the BF16-rounded reference and
                within 2e-2 max(1, |y|) of the FP64 network;
  decode        the step equals the decode of the kernel's own y, taken in FP64
                on both sides.
"""
import time

import numpy as np
import pytest
import torch

import oracle
from oracle import mlp as ref
import paper_1901_10475_amd as cd
from paper_1901_10475_amd import catalog
from paper_1901_10475_amd import learned_dt as ld
from tests.gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu


def _theta(seed):
    """Reference parameters that FP32 represents exactly, non-zero biases."""
    rng = np.random.default_rng(seed)
    p = ref.unpack(ref.init_params(seed).copy())
    p["b1"][:] = rng.normal(0, 0.1, 64)
    p["b2"][:] = rng.normal(0, 0.1, 64)
    p["b3"][:] = 0.5
    return ref.pack(p).astype(np.float32).astype(np.float64)


def _bf16_bits(theta):
    b = np.asarray(ref.bf16(theta), np.float32).view(np.uint32) >> 16
    return torch.from_numpy(b.astype(np.uint16).view(np.int16)).cuda()


def _params(sc):
    return cd.params_struct(sc.tick_s, sc.mu, sc.threshold_km, sc.horizon_ticks, 0)


def test_features_match_reference():
    need_gpu()
    sc = catalog.projected_debris(seed=77, n=3001, parents=3, horizon_ticks=600_000, planted=4)
    say("features", sc.name, sc.n)
    x = ld.cd_mlp_features(cd.soa(sc.elements), _params(sc)).cpu().numpy()
    xr = ref.features(sc.elements[:, 0], sc.elements[:, 1], sc.elements[:, 2], sc.mu)
    np.testing.assert_allclose(x, xr, rtol=2.0 ** -23, atol=0)


@pytest.mark.parametrize("B", [1, 255, 1024, 3001])
def test_forward_and_gradient_match_reference(B):
    need_gpu()
    say("mlp grad B", B)
    theta = _theta(B)
    rng = np.random.default_rng(B + 1)
    X = rng.uniform(0, 1.2, (B, 5)).astype(np.float32)
    t = rng.normal(0, 1, B).astype(np.float32)
    w = torch.from_numpy(theta.astype(np.float32)).cuda()
    xg, tg = torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda()
    X64, t64 = X.astype(np.float64), t.astype(np.float64)

    y = ld.cd_mlp_forward(w, xg).cpu().numpy().astype(np.float64)
    yr, _ = ref.forward(theta, X64)
    assert np.all(np.abs(y - yr) <= 1e-5 * np.maximum(1.0, np.abs(yr)))

    g, loss = ld.cd_mlp_grad(w, xg, tg)
    g = g.cpu().numpy().astype(np.float64)
    gr = ref.grad(theta, X64, t64)
    rel = np.linalg.norm(g - gr) / np.linalg.norm(gr)
    say("  grad rel err", rel)
    assert rel <= 1e-5
    lr = ref.loss(theta, X64, t64)
    assert abs(loss.item() - lr) <= 1e-5 * lr
    # every parameter group is exercised
    pg, pr = ref.unpack(g), ref.unpack(gr)
    for name in ("W1", "b1", "W2", "b2", "w3", "b3"):
        assert np.linalg.norm(pg[name] - pr[name]) <= 1e-4 * np.linalg.norm(pr[name]) + 1e-12, name
    # fixed summation order: bitwise repeatable
    g2, loss2 = ld.cd_mlp_grad(w, xg, tg)
    assert np.array_equal(g2.cpu().numpy().view(np.uint32),
                          g.astype(np.float32).view(np.uint32))
    assert loss2.item() == loss.item()


def test_adam_matches_reference_and_exports_bf16():
    need_gpu()
    theta = _theta(5)
    rng = np.random.default_rng(6)
    w = torch.from_numpy(theta.astype(np.float32)).cuda()
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    wb = torch.empty(ld.CD_MLP_PARAMS, dtype=torch.int16, device="cuda")
    th, mo, vo = theta.copy(), np.zeros_like(theta), np.zeros_like(theta)
    for step in range(1, 4):
        g = rng.normal(0, 1e-2, theta.size).astype(np.float32)
        ld.cd_mlp_adam(w, m, v, torch.from_numpy(g).cuda(), step, 1e-3, w_bf16=wb)
        th, mo, vo = ref.adam(th, mo, vo, g.astype(np.float64), step, 1e-3)
    wg = w.cpu().numpy()
    assert np.all(np.abs(wg - th) <= 1e-6 * np.maximum(1.0, np.abs(th)))
    expect = (np.asarray(ref.bf16(wg), np.float32).view(np.uint32) >> 16).astype(np.uint16)
    assert np.array_equal(wb.cpu().numpy().view(np.uint16), expect)


def test_bf16_inference_matches_reference():
    need_gpu()
    sc = catalog.projected_debris(seed=78, n=4097, parents=4, horizon_ticks=3_600_000,
                                  planted=4)
    say("bf16 inference", sc.name, sc.n)
    theta = _theta(9)
    el = cd.soa(sc.elements)
    dt = torch.empty(sc.n, dtype=torch.int32, device="cuda")
    y = torch.empty(sc.n, dtype=torch.float32, device="cuda")
    ld.cd_dt_mlp(el, _bf16_bits(theta), 5.0, _params(sc), dt, y)
    y = y.cpu().numpy().astype(np.float64)
    dt = dt.cpu().numpy().view(np.uint32)
    X = ref.features(sc.elements[:, 0], sc.elements[:, 1], sc.elements[:, 2], sc.mu)
    ye = ref.forward_bf16(theta, X)
    y64, _ = ref.forward(theta, X)
    assert np.all(np.abs(y - ye) <= 5e-3 * np.maximum(1.0, np.abs(ye)))
    assert np.all(np.abs(y - y64) <= 2e-2 * np.maximum(1.0, np.abs(y64)))
    # the step is the decode of the kernel's y, both in FP64
    want = ref.decode(y, sc.tick_s, sc.horizon_ticks)
    v = np.exp2(y) / sc.tick_s
    edge = np.abs(v - np.round(v)) <= 1e-9 * np.maximum(v, 1.0)
    assert np.all((dt == want) | edge)
    assert len(np.unique(dt)) > 10


def test_dt_mlp_fallbacks_and_clamps():
    need_gpu()
    sc = catalog.projected_debris(seed=79, n=513, parents=1, horizon_ticks=600_000, planted=0)
    el, p = cd.soa(sc.elements), _params(sc)
    heur = torch.empty(sc.n, dtype=torch.int32, device="cuda")
    cd.cd_dt_heuristic(el, p, 5.0, heur)
    heur = heur.cpu().numpy()
    dt = torch.empty(sc.n, dtype=torch.int32, device="cuda")
    y = torch.empty(sc.n, dtype=torch.float32, device="cuda")
    # no weights: the speed-bound step, y = NaN
    ld.cd_dt_mlp(el, None, 5.0, p, dt, y)
    assert np.array_equal(dt.cpu().numpy(), heur) and np.all(np.isnan(y.cpu().numpy()))
    theta = _theta(10)
    pz = ref.unpack(theta.copy())
    pz["w3"][:] = 0.0
    for b3, expect in ((float("nan"), heur), (float("inf"), heur),
                       (40.0, np.full(sc.n, sc.horizon_ticks)), (-30.0, np.ones(sc.n))):
        pz["b3"][:] = b3
        ld.cd_dt_mlp(el, _bf16_bits(ref.pack(pz)), 5.0, p, dt, y)
        assert np.array_equal(dt.cpu().numpy(), expect), b3


def test_pair_object_counts():
    need_gpu()
    sc = catalog.scaled(catalog.small_leo(), n=400)
    el = cd.soa(sc.elements)
    p = cd.params_struct(sc.tick_s, sc.mu, sc.threshold_km, sc.horizon_ticks, sc.dt_ticks)
    bp = cd.BroadPhase(sc.n, p)
    pairs = bp.run(el)
    counts = ld.cd_pair_object_counts(pairs, sc.n).cpu().numpy()
    pr = pairs.cpu().numpy().view(np.uint32)
    expect = np.bincount(pr[:, 0], minlength=sc.n) + np.bincount(pr[:, 1], minlength=sc.n)
    assert len(pr) > 0 and np.array_equal(counts, expect)


def _recall(pairs, planted):
    pr = pairs.cpu().numpy().view(np.uint32)
    found = 0
    for i, j, tc in planted:
        sel = (pr[:, 0] == i) & (pr[:, 1] == j) & (pr[:, 2] <= tc) & (tc < pr[:, 3])
        found += bool(sel.any())
    return found / max(len(planted), 1)


def _timed(el, p, dt, reps=5):
    bp = cd.BroadPhase(el.shape[1], p, dt_ticks=dt, box_precision=cd.CD_FP32,
                       tree_precision=cd.CD_FP32)
    pairs = bp.run(el)
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pairs = bp.run(el)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return pairs, bp.count, 1e3 * float(np.median(ts))


def test_trained_network_gains_over_speed_bound_step():
    """Train on step sweeps of two catalogs; on a third (held out) the learned
    steps give a lower cost objective and fewer boxes than the speed-bound
    step at 5 km, with every planted conjunction still reported.  Against
    one tuned scalar the network does not win: the learned steps times the
    one scalar that is best on the training catalogs cost at most 5 % more
    than the uniform rescaling of the speed bound that is best on the
    training catalogs, on the held-out catalog (the cost counts boxes,
    candidate records and the traversal's box tests; the rescaling that is
    best on the held-out catalog itself is printed too)."""
    need_gpu()
    T, n = 600_000, 6000
    xs, ts = [], []
    for seed in (5101, 5102):
        sc = catalog.projected_debris(seed=seed, n=n, parents=3, horizon_ticks=T, planted=0)
        say("sweep", sc.name, seed)
        x, t, summary = ld.sweep_targets(cd.soa(sc.elements), _params(sc),
                                         scales=ld.DEFAULT_SCALES)
        say("  ", summary)
        xs.append(x)
        ts.append(t)
    X, Y = torch.cat(xs), torch.cat(ts)
    net = ld.StepNet(seed=0)
    net.set_output_bias(float(Y.mean().item()))
    losses = net.train(X, Y, steps=400, lr=3e-3, lr_end=3e-4)
    say("train loss", losses[0], "->", losses[-1], "target var", float(Y.var().item()))
    assert losses[-1] < losses[0]

    # one scalar tuned on the training catalogs, for the uniform rescaling of
    # the speed bound and for the learned steps alike
    train = [catalog.projected_debris(seed=seed, n=n, parents=3, horizon_ticks=T, planted=0)
             for seed in (5101, 5102)]
    def train_cost(steps_of):
        tot = 0.0
        for tc in train:
            tel, tp = cd.soa(tc.elements), _params(tc)
            tot += float(ld.run_costs(tel, tp, steps_of(tel, tp), 32.0)[0].sum().item())
        return tot
    def uniform(scale):
        def f(tel, tp):
            d = torch.empty(tel.shape[1], dtype=torch.int32, device="cuda")
            cd.cd_dt_heuristic(tel, tp, 5.0 * scale, d)
            return d
        return f
    def scaled_net(c):
        return lambda tel, tp: torch.clamp((net.dt(tel, tp).double() * c).round(), 1,
                                           max(T, 1)).to(torch.int32)
    s_train = min(ld.DEFAULT_SCALES, key=lambda x: train_cost(uniform(x)))
    c_train = min((0.5, 0.71, 1.0, 1.41, 2.0), key=lambda x: train_cost(scaled_net(x)))
    say("tuned on the training catalogs: uniform scale", s_train, "network scale", c_train)

    sc = catalog.projected_debris(seed=5103, n=n, parents=3, horizon_ticks=T, planted=8)
    el, p = cd.soa(sc.elements), _params(sc)
    dt_h = torch.empty(sc.n, dtype=torch.int32, device="cuda")
    cd.cd_dt_heuristic(el, p, 5.0, dt_h)
    dt_m = net.dt(el, p)
    runs = [("speed-bound", dt_h), ("learned", dt_m),
            ("learned tuned", scaled_net(c_train)(el, p))]
    for s in ld.DEFAULT_SCALES:   # uniform rescalings of the speed bound
        d = torch.empty(sc.n, dtype=torch.int32, device="cuda")
        cd.cd_dt_heuristic(el, p, 5.0 * s, d)
        runs.append((f"speed-bound x{s:g}", d))
    rows = {}
    for name, dt in runs:
        cost, counts, boxes, pairs = ld.run_costs(el, p, dt, 32.0)
        pairs, boxes, ms = _timed(el, p, dt)
        rows[name] = {"cost": float(cost.sum().item()), "boxes": int(boxes),
                      "records": int(pairs.shape[0]), "ms": ms,
                      "recall": _recall(pairs, sc.planted)}
        say(name, rows[name])
    assert rows["speed-bound"]["recall"] == 1.0 and rows["learned"]["recall"] == 1.0
    assert rows["learned"]["cost"] < rows["speed-bound"]["cost"]
    assert rows["learned"]["boxes"] < rows["speed-bound"]["boxes"]
    unif = {k: v for k, v in rows.items() if k.startswith("speed-bound x")}
    best = min(unif, key=lambda k: unif[k]["cost"])
    fair = unif[f"speed-bound x{s_train:g}"]
    say("uniform tuned on training", s_train, fair)
    say("uniform best on the held-out catalog", best, unif[best])
    say("learned", rows["learned"], "learned tuned", rows["learned tuned"])
    assert all(v["recall"] == 1.0 for v in rows.values())
    # the learned steps (with their training-tuned scalar) against the
    # training-tuned uniform rescaling: no gain, at most a small loss
    assert rows["learned tuned"]["cost"] <= 1.05 * fair["cost"]
