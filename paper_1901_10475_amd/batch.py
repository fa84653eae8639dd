"""Many independent scenarios in one graph launch.

The paper notes that sub-problems of the collision search are independent
(Sec. Decomposition of the AABB Tree State Space), which makes batching them
natural.  ``BatchRunner`` runs the whole path (boxes, tree, canonical pairs)
for every scenario of a batch and records it once into a hipGraph
(``cd_graph_*``); a replay is one launch for the whole batch, with no host
synchronisation inside it.

The scenarios are dealt to ``branches`` streams (largest first, each to the
branch with the fewest boxes so far); inside the graph the branches run side
by side, each one's scenarios in order, so the small scenarios' short,
latency-bound launches overlap instead of queueing behind each other.  The
scenarios of a branch share one set of box, tree and workspace buffers sized
for its largest (``shared_buffers=False`` gives every scenario its own boxes
and tree instead, so that they outlive the replay); each scenario keeps its
own output list, record count and status word on the device.  FP64 boxes
of an FP64 tree are written as the tree's own leaf records in the sorted
layout (``Boxes.in_tree``), so every scenario's tree is built bottom-up in
place; other precisions use box arrays.  Output
capacities come from one eager pass (``calibrate``); a replay whose status
reports exceeded capacity is repeated eagerly for that scenario by
``results``.  Launch shapes can differ per
scenario (``tunings``): they are read while the graph is recorded.  A
scenario's replays launch the node-pair levels its eager query needed plus
two (``cd_last_query_levels``) instead of the default 96; a replay whose
inputs need more finishes with the per-leaf walk.
"""
import ctypes
import math

import numpy as np
import torch

from . import (CD_E_CAPACITY, CD_FP64, CD_LAYOUT_SORTED, CD_OK, CD_SORTED_MAX_RECORDS, Boxes, Graph,
               _bytes, _check, _ptr, _stream, cd_boxes, cd_build_boxes, cd_get_tuning,
               cd_last_query_levels, cd_query_pairs, cd_query_pairs_async, cd_set_tuning,
               cd_tree, lib, params_struct, soa)


class _Boxes:
    """Descriptor over shared box arrays for one scenario's count."""

    def __init__(self, arrays, count, precision):
        self.desc = cd_boxes()
        self.desc.count = int(count)
        self.desc.precision = precision
        lo, hi, t0, t1, obj, code = arrays
        for d in range(3):
            self.desc.lo[d] = lo[d].data_ptr()
            self.desc.hi[d] = hi[d].data_ptr()
        self.desc.t0 = t0.data_ptr()
        self.desc.t1 = t1.data_ptr()
        self.desc.obj = obj.data_ptr()
        self.desc.code = code.data_ptr()
        self.desc.code_valid = 0
        self.desc.layout = CD_LAYOUT_SORTED


class _Tree:
    def __init__(self, mem, count, precision):
        self.mem = mem
        self.desc = cd_tree()
        self.desc.mem = mem.data_ptr()
        self.desc.bytes = lib().cd_tree_bytes(int(count), precision)


class BatchRunner:
    def __init__(self, scenarios, box_precision=CD_FP64, tree_precision=CD_FP64,
                 margin=1.25, min_capacity=4096, device="cuda", shared_buffers=True,
                 branches=4):
        self.sc = list(scenarios)
        self.box_precision, self.tree_precision = box_precision, tree_precision
        self.margin, self.min_capacity = margin, min_capacity
        self.device = device
        self.el = [soa(s.elements, device) for s in self.sc]
        self.params = []
        self.counts = []
        for s in self.sc:
            if not s.uniform_dt:
                raise ValueError("batched scenarios take a uniform step")
            p = params_struct(s.tick_s, s.mu, s.threshold_km, s.horizon_ticks, s.dt_ticks)
            self.params.append(p)
            K = 1 if s.horizon_ticks == 0 else -(-s.horizon_ticks // int(s.dt_ticks))
            self.counts.append(s.n * K)
        Nmax = max(self.counts)
        ft = torch.float64 if box_precision == CD_FP64 else torch.float32

        # records in the tree where the layout allows (all FP64, n within the
        # sorted layout's limit), box arrays otherwise
        self.in_tree = [box_precision == CD_FP64 and tree_precision == CD_FP64
                        and s.n <= CD_SORTED_MAX_RECORDS for s in self.sc]

        def box_arrays(N):
            return (torch.empty((3, N), dtype=ft, device=device),
                    torch.empty((3, N), dtype=ft, device=device),
                    torch.empty(N, dtype=torch.int32, device=device),
                    torch.empty(N, dtype=torch.int32, device=device),
                    torch.empty(N, dtype=torch.int32, device=device),
                    torch.empty(N, dtype=torch.int32, device=device))

        # branches: largest scenario first, each to the branch with the
        # fewest boxes so far
        S = len(self.sc)
        B = max(1, min(int(branches), S))
        load = [0] * B
        self.branch_of = [0] * S
        for k in sorted(range(S), key=lambda k: -self.counts[k]):
            b = min(range(B), key=lambda b: load[b])
            self.branch_of[k] = b
            load[b] += self.counts[k]
        members = [[k for k in range(S) if self.branch_of[k] == b] for b in range(B)]
        self.members = members

        need_arrays = not all(self.in_tree)
        if shared_buffers:
            self.arrays, self.codes, self.tree_mems = [None] * S, [None] * S, [None] * S
            for b in range(B):
                Nb = max(self.counts[k] for k in members[b])
                arrays = (box_arrays(Nb) if any(not self.in_tree[k] for k in members[b])
                          else None)
                codes = torch.empty(Nb, dtype=torch.int32, device=device)
                tree_mem = _bytes(lib().cd_tree_bytes(Nb, tree_precision), device)
                for k in members[b]:
                    self.arrays[k], self.codes[k], self.tree_mems[k] = arrays, codes, tree_mem
        else:
            self.arrays = [None if t else box_arrays(N) for N, t in zip(self.counts, self.in_tree)]
            self.codes = [torch.empty(N, dtype=torch.int32, device=device) for N in self.counts]
            self.tree_mems = [_bytes(lib().cd_tree_bytes(N, tree_precision), device)
                              for N in self.counts]
        # workspaces per branch
        self.ws_boxes_b = [_bytes(max(lib().cd_build_boxes_ws(self.sc[k].n) for k in members[b]),
                                  device) for b in range(B)]
        self.ws_tree_b = [_bytes(lib().cd_build_tree_ws(max(self.counts[k] for k in members[b])),
                                 device) for b in range(B)]
        self.trees = [_Tree(m, N, tree_precision) for m, N in zip(self.tree_mems, self.counts)]
        self.boxes = [Boxes.in_tree(tr, N, device, code=c) if t else _Boxes(a, N, box_precision)
                      for tr, N, t, a, c in zip(self.trees, self.counts, self.in_tree, self.arrays,
                                                self.codes)]
        self.count_dev = torch.zeros(S, dtype=torch.int64, device=device)
        self.status_dev = torch.zeros(S, dtype=torch.int32, device=device)
        self.capacity = [0] * S
        self.out = [None] * S
        self.ws_query = None
        self.graph = None
        self.stream = torch.cuda.Stream(device=device)
        self.branch_streams = [torch.cuda.Stream(device=device) for _ in range(B)]
        self.tunings = [None] * S
        # node-pair levels each scenario's eager query needed (+2): the
        # replays launch that many instead of the default
        self.levels = [0] * S

    def box_arrays(self, k):
        """(lo [3,N], hi [3,N], t0, t1, obj) of scenario k's boxes as last built
        (with shared buffers, only the scenario built last still holds them)."""
        N = self.counts[k]
        if self.in_tree[k]:
            b = self.boxes[k]
            return b.lo[:, :N], b.hi[:, :N], b.t0[:N], b.t1[:N], b.obj[:N]
        lo, hi, t0, t1, obj, _ = self.arrays[k]
        return lo[:, :N], hi[:, :N], t0[:N], t1[:N], obj[:N]

    # -- one scenario, eager ------------------------------------------------------
    def _build(self, k):
        b = self.boxes[k]
        br = self.branch_of[k]
        b.desc.layout = CD_LAYOUT_SORTED   # where n allows; the layout written is kept
        cd_build_boxes(self.el[k], None, self.params[k], b, self.ws_boxes_b[br])
        ws_tree = self.ws_tree_b[br]
        _check(lib().cd_build_tree(ctypes.byref(b.desc), self.tree_precision, 0,
                                   ctypes.byref(self.trees[k].desc), _ptr(ws_tree),
                                   ws_tree.numel(), _stream()))

    def run_eager(self, k):
        """Pairs of scenario k by the synchronising query (int32 [P, 4])."""
        self._build(k)
        cap = max(self.capacity[k], self.min_capacity)
        while True:
            out = torch.empty((cap, 4), dtype=torch.int32, device=self.device)
            ws = _bytes(lib().cd_query_pairs_ws(self.counts[k], cap), self.device)
            rc, cnt = cd_query_pairs(self.trees[k], out, cap, ws)
            if rc == CD_OK:
                return out[:cnt]
            cap = int(cnt * self.margin) + 1024

    def query_built(self, k):
        """Pairs of scenario k's tree as last built (synchronising query)."""
        cap = max(self.capacity[k], self.min_capacity)
        while True:
            out = torch.empty((cap, 4), dtype=torch.int32, device=self.device)
            ws = _bytes(lib().cd_query_pairs_ws(self.counts[k], cap), self.device)
            rc, cnt = cd_query_pairs(self.trees[k], out, cap, ws)
            if rc == CD_OK:
                return out[:cnt]
            cap = int(cnt * self.margin) + 1024

    def autotune(self, path=None, reps=2, log=None):
        """Launch shapes per scenario from the autotuner (autotune.tuned),
        keyed by box-count bucket: one scenario per bucket is built and its
        query tuned (or the cached choice taken); every scenario of the bucket
        gets it.  Returns {bucket key: (tuning, cached)}."""
        from . import autotune
        prec = self.tree_precision
        chosen = {}
        with torch.cuda.stream(self.stream):
            for k in range(len(self.sc)):
                key = autotune.cache_key(prec, self.counts[k], "fixed")
                if key not in chosen:
                    self._build(k)
                    chosen[key] = autotune.tuned(lambda: self.query_built(k), prec,
                                                 self.counts[k], "fixed", path=path, reps=reps,
                                                 log=log)
                self.tunings[k] = chosen[key][0]
        self.stream.synchronize()
        return chosen

    def calibrate(self):
        """One eager pass: sets every scenario's output capacity and the
        node-pair levels its replays launch."""
        with torch.cuda.stream(self.stream):
            for k in range(len(self.sc)):
                self._apply_tuning(k)
                P = int(self.run_eager(k).shape[0])
                self.capacity[k] = max(self.min_capacity, int(math.ceil(P * self.margin)))
                lv = cd_last_query_levels()
                self.levels[k] = min(400, lv + 2) if lv > 0 else 0
        self.stream.synchronize()
        self._alloc_outputs()

    def _alloc_outputs(self):
        self.out = [torch.empty((c, 4), dtype=torch.int32, device=self.device)
                    for c in self.capacity]
        self.ws_query = [
            _bytes(lib().cd_query_pairs_ws(max(self.counts[k] for k in m),
                                           max(self.capacity[k] for k in m)), self.device)
            for m in self.members]

    def _apply_tuning(self, k):
        t = dict(self.tunings[k]) if self.tunings[k] else {}
        if self.levels[k]:
            t["max_levels"] = self.levels[k]
        cd_set_tuning(t or None)

    # -- the batch as one graph -------------------------------------------------------
    def enqueue_branch(self, b):
        """Enqueue branch b's scenarios (boxes, tree, device-count query each)
        on the current stream."""
        saved = cd_get_tuning()
        try:
            for k in self.members[b]:
                self._apply_tuning(k)
                self._build(k)
                cd_query_pairs_async(self.trees[k], self.out[k], self.capacity[k],
                                     self.count_dev[k:k + 1], self.status_dev[k:k + 1],
                                     self.ws_query[b])
        finally:
            cd_set_tuning(saved)

    def enqueue(self):
        """Enqueue the whole batch from the current stream: the branches fork
        from it on their own streams and join it again at the end."""
        main = torch.cuda.current_stream()
        fork = torch.cuda.Event()
        fork.record(main)
        joins = []
        for b, st in enumerate(self.branch_streams):
            st.wait_event(fork)
            with torch.cuda.stream(st):
                self.enqueue_branch(b)
            ev = torch.cuda.Event()
            ev.record(st)
            joins.append(ev)
        for ev in joins:
            main.wait_event(ev)

    def capture(self):
        if self.ws_query is None:
            self.calibrate()
        elif any(o.shape[0] < c for o, c in zip(self.out, self.capacity)):
            self._alloc_outputs()
        self.close()
        g = Graph()
        self.stream.synchronize()
        with torch.cuda.stream(self.stream):
            g.begin()
            try:
                self.enqueue()
            finally:
                g.end()
        self.graph = g

    def replay(self):
        with torch.cuda.stream(self.stream):
            self.graph.launch()

    def results(self):
        """Wait for the last replay; per-scenario pair tensors (int32 [P, 4]).
        A scenario whose capacity was exceeded is rerun eagerly (and its
        capacity raised for the next capture)."""
        self.stream.synchronize()
        cnt = self.count_dev.cpu().numpy()
        st = self.status_dev.cpu().numpy()
        res = []
        for k in range(len(self.sc)):
            if st[k] & 2:
                raise RuntimeError(f"scenario {k}: tree inconsistent (status {st[k]})")
            if st[k] & 1:
                self.capacity[k] = int(cnt[k] * self.margin) + 1024
                with torch.cuda.stream(self.stream):
                    res.append(self.run_eager(k))
                self.stream.synchronize()
            else:
                res.append(self.out[k][:int(cnt[k])])
        return res

    def close(self):
        if self.graph is not None:
            self.graph.close()
            self.graph = None

    def boxes_total(self):
        return int(sum(self.counts))

    def brute_force_tests(self):
        """Box pairs of different objects whose tags overlap (uniform step:
        K * C(n, 2) per scenario)."""
        tot = 0
        for s, N in zip(self.sc, self.counts):
            K = N // s.n
            tot += K * s.n * (s.n - 1) // 2
        return tot
