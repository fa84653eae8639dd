"""The query without caller workspace (cd_query_pairs_async_noalloc) against
the query with one (cd_query_pairs_async): the same record list, count and
status, record for record, on two calls in a row (the second with a smaller
tree, so the shared scratch holds the first call's leftovers), plus the size
limit, which is rejected before anything is enqueued."""
import ctypes

import numpy as np
import pytest
import torch

import paper_1901_10475_amd as cd
from paper_1901_10475_amd import catalog
from tests.gpu_util import need_gpu, say


def _query_both(sc, heur=None):
    el = cd.soa(sc.elements)
    p = cd.params_struct(sc.tick_s, sc.mu, sc.threshold_km, sc.horizon_ticks,
                         sc.dt_ticks if heur is None else 0)
    bp = cd.BroadPhase(sc.n, p, dt_heuristic_km=heur, el_soa=el)
    ref = bp.run(el).cpu().numpy()
    P = len(ref)
    cap = 2 * P + 17
    assert cd.lib().cd_query_pairs_ws(bp.count, cap) <= cd.lib().cd_noalloc_scratch_bytes()
    out = []
    for fn in ("ws", "noalloc"):
        rec = torch.full((cap, 4), -1, dtype=torch.int32, device="cuda")
        cnt = torch.full((1,), 12345, dtype=torch.int64, device="cuda")
        st = torch.full((1,), 7, dtype=torch.int32, device="cuda")
        if fn == "ws":
            ws = cd._bytes(cd.lib().cd_query_pairs_ws(bp.count, cap), "cuda")
            cd.cd_query_pairs_async(bp.tree, rec, cap, cnt, st, ws)
        else:
            cd.cd_query_pairs_async_noalloc(bp.tree, rec, cap, cnt, st)
        torch.cuda.synchronize()
        c = int(cnt.item())
        out.append((c, int(st.item()), rec[:c].cpu().numpy()))
    (c0, s0, r0), (c1, s1, r1) = out
    assert s0 == 0 and s1 == 0 and c0 == P and c1 == P
    assert np.array_equal(r0, ref) and np.array_equal(r1, ref)
    return bp, P


@pytest.mark.gpu
def test_noalloc_query_equals_workspace_query_twice():
    need_gpu()
    big = catalog.scaled(catalog.tracked_hour(seed=61, planted=8), n=4000, horizon_ticks=240_000)
    small = catalog.scaled(catalog.small_leo(seed=62, n=600, planted=6), horizon_ticks=60_000)
    say("noalloc query: first call", big.n, "objects")
    bp_big, P_big = _query_both(big)
    say("  records", P_big, "boxes", bp_big.count)
    say("noalloc query: second call, smaller", small.n, "objects")
    bp_small, P_small = _query_both(small)
    say("  records", P_small, "boxes", bp_small.count)
    assert bp_small.count < bp_big.count and P_big > 0 and P_small > 0
    # per-object steps (device-wide sort path) after both
    deb = catalog.projected_debris(seed=63, n=3000, parents=2, horizon_ticks=60_000, planted=4)
    say("noalloc query: per-object steps", deb.n)
    _query_both(deb, heur=5.0)


@pytest.mark.gpu
def test_noalloc_query_rejects_oversized_workspace():
    need_gpu()
    sc = catalog.scaled(catalog.small_leo(seed=64, n=300, planted=0), horizon_ticks=20_000)
    el = cd.soa(sc.elements)
    p = cd.params_struct(sc.tick_s, sc.mu, sc.threshold_km, sc.horizon_ticks, sc.dt_ticks)
    bp = cd.BroadPhase(sc.n, p)
    bp.run(el)
    lim = cd.lib().cd_noalloc_scratch_bytes()
    cap = lim // 16          # raw records alone exceed the scratch
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    rc = cd.lib().cd_query_pairs_async_noalloc(ctypes.byref(bp.tree.desc),
                                               ctypes.c_void_p(bp.out.data_ptr()), cap,
                                               ctypes.c_void_p(cnt.data_ptr()),
                                               ctypes.c_void_p(st.data_ptr()), None)
    assert rc == cd.CD_E_WORKSPACE
    assert "fixed scratch" in cd.lib().cd_last_error().decode()
