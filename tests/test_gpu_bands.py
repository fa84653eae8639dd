"""Altitude-band partition on the GPU against the oracle, and the band
sub-problems' merged records against the whole catalog's filtered records."""
import numpy as np
import pytest
import torch

import oracle
import paper_1901_10475_amd as cd
from paper_1901_10475_amd import catalog
from paper_1901_10475_amd.bands import BandRunner
from tests.gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu


def _mixed(seed, n, T, dt, thr):
    rng = np.random.default_rng(seed)
    el = catalog.tracked_population(rng, n)
    k = n // 10
    el[:k, 0] = rng.uniform(15000.0, 26000.0, k)
    el[:k, 1] = rng.uniform(0.5, 0.7, k)
    pl = catalog.plant_conjunctions(rng, el, 6, T, dt, thr)
    return catalog.Scenario(f"mixed{n}", el, dt, T, thr, planted=pl)


@pytest.mark.parametrize("p,n", [(1, 2000), (3, 2000), (16, 2000), (100, 2000), (64, 30)])
def test_partition_matches_oracle(p, n):
    need_gpu()
    sc = _mixed(41, n, 1000, 1000, 40.0)
    say("band partition p", p)
    el = cd.soa(sc.elements)
    params = cd.params_struct(sc.tick_s, sc.mu, sc.threshold_km, sc.horizon_ticks, sc.dt_ticks)
    edges, offsets, members = cd.cd_band_partition(el, params, p)
    want_edges, want_bands = oracle.band_partition(sc.elements, sc.threshold_km, p)
    assert np.array_equal(edges.cpu().numpy(), want_edges)
    off = offsets.cpu().numpy()
    mem = members.cpu().numpy().view(np.uint32)
    assert off[-1] == len(mem) == sum(len(b) for b in want_bands)
    for k in range(p):
        assert np.array_equal(mem[off[k]:off[k + 1]], want_bands[k])


def test_band_filter_matches_oracle():
    need_gpu()
    sc = _mixed(42, 600, 60_000, 5_000, 40.0)
    say("band filter")
    el = cd.soa(sc.elements)
    params = cd.params_struct(sc.tick_s, sc.mu, sc.threshold_km, sc.horizon_ticks, sc.dt_ticks)
    pairs = cd.BroadPhase(sc.n, params).run(el).clone()
    got = cd.cd_band_filter(el, params, pairs).cpu().numpy().view(np.uint32)
    rec = pairs.cpu().numpy().view(np.uint32)
    want = oracle.band_filter(sc.elements, rec, sc.threshold_km)
    say("records", len(rec), "kept", len(got))
    assert len(want) > 0 and np.array_equal(got, want)


@pytest.mark.parametrize("p,heur", [(1, None), (3, None), (8, None), (8, 20.0)])
def test_band_problems_merge_to_the_filtered_catalog(p, heur):
    need_gpu()
    sc = _mixed(43, 1500, 120_000, 5_000, 40.0)
    say("band runner p", p, "heur", heur)
    el = cd.soa(sc.elements)
    params = cd.params_struct(sc.tick_s, sc.mu, sc.threshold_km, sc.horizon_ticks,
                              sc.dt_ticks if heur is None else 0)
    kw = {} if heur is None else {"dt_heuristic_km": heur}
    full_bp = cd.BroadPhase(sc.n, params, el_soa=el, **kw)
    full = cd.cd_band_filter(el, params, full_bp.run(el).clone())
    runner = BandRunner(el, params, p, **kw)
    merged = runner.run(el)
    torch.cuda.synchronize()
    a = full.cpu().numpy().view(np.uint32)
    b = merged.cpu().numpy().view(np.uint32)
    say("filtered records", len(a), "band sizes", runner.sizes())
    assert len(a) > 0 and np.array_equal(a, b)
    for i, j, tc in sc.planted:
        hit = b[(b[:, 0] == i) & (b[:, 1] == j)]
        assert np.any((hit[:, 2] <= tc) & (tc < hit[:, 3]))


def test_gather_remap_canonical():
    need_gpu()
    rng = np.random.default_rng(44)
    el_np = catalog.leo_mix(rng, 50)
    el = cd.soa(el_np)
    ids = torch.tensor([7, 3, 49, 0], dtype=torch.int32, device="cuda")
    g = cd.cd_gather_elements(el, ids).cpu().numpy()
    assert np.array_equal(g, el_np[[7, 3, 49, 0]].T)
    rec = torch.tensor([[0, 1, 5, 9], [2, 3, 0, 4], [1, 2, 3, 3]], dtype=torch.int32,
                       device="cuda")
    out = cd.cd_remap_records(rec, ids).cpu().numpy()
    assert out.tolist() == [[3, 7, 5, 9], [0, 49, 0, 4], [3, 49, 3, 3]]
    dup = torch.tensor([[5, 6, 2, 3], [1, 2, 9, 10], [5, 6, 2, 3], [1, 2, 0, 4]],
                       dtype=torch.int32, device="cuda")
    c = cd.cd_canonical_records(dup, 20, 10).cpu().numpy()
    assert c.tolist() == [[1, 2, 0, 4], [1, 2, 9, 10], [5, 6, 2, 3]]


@pytest.mark.parametrize("count", [0, 1, 2, 3, 1000, 4095, 4096, 4097, 20000, 65536, 65537,
                                   100000, 262144, 262145, 400000])
def test_canonical_records_small_medium_and_radix_paths(count):
    """Up to 4096 records take the one-workgroup LDS sort, up to 262144
    the LDS tiles merged pairwise, more the radix path: all give numpy's
    sorted unique rows."""
    need_gpu()
    rng = np.random.default_rng(45 + count)
    rec = np.stack([rng.integers(0, 300, count), rng.integers(0, 300, count),
                    rng.integers(0, 3000, count), rng.integers(0, 3001, count)],
                   axis=1).astype(np.uint32)
    if count > 10:
        rec[count // 2:count // 2 + 7] = rec[:7]     # exact repeats
        rec[-3:, :3] = rec[0, :3]                    # same (i, j, t_lo), other t_hi
    t = torch.from_numpy(rec.view(np.int32)).cuda()
    got = cd.cd_canonical_records(t, 3001, 300).cpu().numpy().view(np.uint32)
    want = np.unique(rec, axis=0)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("count", [3000, 100000, 300000])
def test_canonical_records_end_times_past_the_horizon(count):
    """Only t_lo and the ids are bounded by the sort-key sizes: t_hi may take
    any 32-bit value (a caller's box may end past the horizon) on every path."""
    need_gpu()
    rng = np.random.default_rng(77 + count)
    rec = np.stack([rng.integers(0, 300, count), rng.integers(0, 300, count),
                    rng.integers(0, 3001, count),
                    rng.integers(0, (1 << 32) - 1, count, dtype=np.uint64)],
                   axis=1).astype(np.uint32)
    rec[-5:, :3] = rec[0, :3]                        # same (i, j, t_lo), other t_hi
    rec[-5:, 3] = [3001, 1 << 12, 1 << 20, (1 << 31) + 5, (1 << 32) - 2]
    t = torch.from_numpy(rec.view(np.int32)).cuda()
    got = cd.cd_canonical_records(t, 3000, 300).cpu().numpy().view(np.uint32)
    assert np.array_equal(got, np.unique(rec, axis=0))
