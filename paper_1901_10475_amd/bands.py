"""A catalog run as altitude-band sub-problems: the edge partition of the
potential-collision graph (cd_band_partition), one broad phase per band, the
bands' records mapped back to catalog ids (cd_remap_records), filtered by the
band test (cd_band_filter) and merged into one canonical list
(cd_canonical_records).  The result equals the band-filtered records of the
whole catalog; the bands are independent, so on several GPUs each would run
on its own.  Everything here is argument marshalling; every step runs in the
library's kernels.
"""
import time

import torch

from . import (BroadPhase, cd_band_filter, cd_band_partition, cd_canonical_records,
               cd_gather_elements, cd_remap_records)


class BandRunner:
    def __init__(self, el_soa, params, nbands, **bp_kwargs):
        """el_soa: [6, n] float64 CUDA elements; bp_kwargs go to each band's
        BroadPhase (steps, precisions)."""
        self.params, self.nbands = params, int(nbands)
        self.n = int(el_soa.shape[1])
        self.edges, offsets, members = cd_band_partition(el_soa, params, nbands)
        off = offsets.cpu().tolist()
        self.ids = [members[off[k]:off[k + 1]] for k in range(self.nbands)]
        self.bp = []
        for ids in self.ids:
            if ids.numel() < 2:
                self.bp.append(None)
                continue
            el_k = cd_gather_elements(el_soa, ids)
            kw = dict(bp_kwargs)
            if "dt_heuristic_km" in kw or "dt_mlp" in kw:
                kw["el_soa"] = el_k
            self.bp.append(BroadPhase(int(ids.numel()), params, **kw))

    def sizes(self):
        """(objects, boxes) per band."""
        return [(int(ids.numel()), bp.count if bp is not None else 0)
                for ids, bp in zip(self.ids, self.bp)]

    def run(self, el_soa, band_ms=None):
        """The canonical band-filtered records of the catalog.  band_ms (a list)
        receives each band's wall time when given (synchronising per band)."""
        parts = []
        for ids, bp in zip(self.ids, self.bp):
            t0 = time.perf_counter()
            if bp is not None:
                parts.append((ids, bp.run(cd_gather_elements(el_soa, ids))))
            if band_ms is not None:
                torch.cuda.synchronize()
                band_ms.append((time.perf_counter() - t0) * 1000.0)
        total = sum(int(r.shape[0]) for _, r in parts)
        merged = torch.empty((max(total, 1), 4), dtype=torch.int32, device=el_soa.device)
        at = 0
        for ids, r in parts:
            m = int(r.shape[0])
            if m:
                cd_remap_records(r, ids, out=merged[at:at + m])
            at += m
        kept = cd_band_filter(el_soa, self.params, merged[:total])
        return cd_canonical_records(kept, self.params.horizon_ticks, self.n)
