"""CD_DEBUG_SYNC=1: a call that enqueues work waits for it and reports at
once what would otherwise surface at the next synchronising call -- here the
tree build's error bits (codes out of order in a slab that claims the sorted
layout) from cd_build_tree itself, and an exceeded capacity from the
device-count query itself.  The variable is read once per process, so the
case runs in a child process of its own.
"""
import os
import subprocess
import sys

import pytest

from tests.gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r'''
import sys
sys.path.insert(0, sys.argv[1])
import numpy as np
import torch
import paper_1901_10475_amd as cd
from tests.test_gpu_tree import _uniform


def status(f):
    try:
        f()
    except cd.CDError as e:
        return e.status
    return 0


from paper_1901_10475_amd import catalog

sc = catalog.scaled(catalog.small_leo(seed=77, n=400, planted=8), horizon_ticks=120_000)
el = cd.soa(sc.elements)
p = cd.params_struct(sc.tick_s, sc.mu, sc.threshold_km, sc.horizon_ticks, sc.dt_ticks)
bp = cd.BroadPhase(sc.n, p)
want = bp.run(el).cpu().numpy()
print("records", len(want), flush=True)
# every call on a good tree passes
print("build_ok", status(lambda: bp.build(el)), flush=True)
P = len(want)
out = torch.empty((P, 4), dtype=torch.int32, device="cuda")
ws = cd._bytes(cd.lib().cd_query_pairs_ws(bp.count, P), "cuda")
cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
st = torch.zeros(1, dtype=torch.int32, device="cuda")
print("async_ok", status(lambda: cd.cd_query_pairs_async(bp.tree, out, P, cnt, st, ws)),
      flush=True)
print("async_equal", int(np.array_equal(out.cpu().numpy(), want)), flush=True)
# one record short: the query call itself reports the capacity
print("async_short", status(lambda: cd.cd_query_pairs_async(bp.tree, out[:P - 1], P - 1, cnt,
                                                             st, ws)), flush=True)
# codes out of order in a slab that claims the sorted layout: the build call
# itself reports the tree
b = _uniform(300, 16, 2, seed=3, layout=cd.CD_LAYOUT_SORTED, in_tree=False)
c = b.boxes.code
lo, hi = int(c[5 * 300].item()), int(c[5 * 300 + 299].item())
c[5 * 300], c[5 * 300 + 299] = hi, lo
print("build_bad", status(lambda: cd.cd_build_tree(b.boxes, b.tree_precision, b.tree,
                                                    b.ws_tree)), flush=True)
'''


def test_debug_sync_reports_at_the_call():
    need_gpu()
    say("CD_DEBUG_SYNC child process")
    env = dict(os.environ, CD_DEBUG_SYNC="1")
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT], env=env, capture_output=True,
                       text=True, timeout=300)
    say(r.stdout.strip().replace("\n", "; "))
    assert r.returncode == 0, r.stderr[-2000:]
    got = dict(line.split() for line in r.stdout.strip().splitlines())
    import paper_1901_10475_amd as cd
    assert int(got["records"]) > 1
    assert int(got["build_ok"]) == cd.CD_OK
    assert int(got["async_ok"]) == cd.CD_OK
    assert got["async_equal"] == "1"
    assert int(got["async_short"]) == cd.CD_E_CAPACITY
    assert int(got["build_bad"]) == cd.CD_E_INVALID
