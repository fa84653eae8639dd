// k_refit.hip -- the atomic bottom-up refit of the tree's inner boxes.
//
// Each inner box (space and time) is set to the exact union of its two
// children by a bottom-up pass in which the second of the two threads reaching
// a node computes it; the pass also records every pair of sibling nodes whose
// boxes overlap, the seeds of the node-pair traversal.
#include "cd_internal.h"

namespace cd {

static inline unsigned nblk(uint64_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

// ---- bottom-up refit ---------------------------------------------------------------------
//
// Every inner box is the exact union of its children.  The classic scheme (one
// thread per leaf climbs; at each node the first arrival stops and the second
// writes the union) needs, on MI355X, agent-scope release/acquire whenever the
// two threads sit in different workgroups: the eight XCDs have separate L2
// caches, so each such atomic writes back and invalidates L2.  Here every
// meeting happens inside one workgroup instead.  Leaves are cut into blocks of
// refit_block(k) = 1024 * 16^k consecutive leaves, level by level; a node
// belongs to the lowest level whose blocks hold its whole range.
//   level 0: one workgroup per 1024-leaf chunk, one leaf per thread.  Parents,
//      children, arrival counters, computed inner boxes and the hand-offs to
//      upper levels are staged in LDS (79.6 KiB, two workgroups per CU); a
//      sibling leaf is read back from its record, written before the barrier
//      and still in L2.  Computed inner records are written out in one
//      coalesced pass at the end.
//   level k >= 1: one workgroup per level-k block climbs, in global memory with
//      workgroup-scope counters, from the nodes queued for it by lower levels.
// A climb that meets a parent of a higher level queues the node for that level
// and block.  Kernel boundaries order each level's writes before the next.

template <int TP>
__global__ __launch_bounds__(kRefitChunk) void k_refit_chunks(
    uint32_t N, const uint32_t *__restrict__ parent,
    const uint2 *__restrict__ kids, LinkSink links, const uint8_t *clev,
    void *tree, RefitLists L, SeedSink seeds, unsigned int *err)
{
    __shared__ LBox innb[kRefitChunk];
    __shared__ uint2 kid[kRefitChunk];
    __shared__ uint32_t par_leaf[kRefitChunk], par_in[kRefitChunk];
    __shared__ unsigned int cnt[kRefitChunk];
    __shared__ uint2 sbuf[kSeedStage];
    __shared__ unsigned int sn, sbase;
    // nodes handed to levels 1..kPushLevels, staged per level: all of this
    // chunk's go to one list per level, reserved with one atomic at the end
    __shared__ uint32_t pstage[kPushLevels][kPushStage];
    __shared__ unsigned int pcnt[kPushLevels], pbase[kPushLevels];
    const SeedStage stage{sbuf, &sn};
    const uint32_t t = threadIdx.x;
    if (t == 0)
        sn = 0;
    if (t < (uint32_t)kPushLevels)
        pcnt[t] = 0;
    const uint32_t c = xcd_block(blockIdx.x, gridDim.x);
    const uint32_t c0 = c * (uint32_t)kRefitChunk;
    const uint32_t m = N - c0 < (uint32_t)kRefitChunk ? N - c0 : (uint32_t)kRefitChunk;
    double lo[3], hi[3];
    uint32_t t0 = 0, t1 = 0;
    bool bad = false;
    if (t < m) {
        // leaf records already written in sorted order by the slab build
        uint32_t leaf = N - 1 + c0 + t;
        NodeIO<TP>::get_box(tree, N, leaf, lo, hi, t0, t1);
        par_leaf[t] = parent[leaf];
    }
    if (c0 + t + 1 < N) {  // inner node c0 + t exists
        kid[t] = kids[c0 + t];
        par_in[t] = parent[c0 + t];
    }
    // The skip links of the records this lane writes at the end, loaded now
    // so that the final pass waits on no global load: FP64, the last quarter
    // of records t / 4 + j * kRefitChunk / 4; FP32, the link record of node
    // c0 + t.
    uint32_t esc_w[4] = {0, 0, 0, 0};
    if (TP == CD_FP64) {
        if ((t & 3u) == 3u)
            for (int j = 0; j < 4; ++j) {
                uint32_t p = c0 + (t >> 2) + (uint32_t)(kRefitChunk / 4) * (uint32_t)j;
                if (p + 1 < N)
                    esc_w[j] = links.esc_of(p);
            }
    } else if (c0 + t + 1 < N) {
        esc_w[0] = links.esc_of(c0 + t);
    }
    cnt[t] = 0;
    __syncthreads();
    if (t < m) {
        uint32_t node = N - 1 + c0 + t;
        uint32_t pv = par_leaf[t];
        for (int guard = 0; guard < 160; ++guard) {
            if (pv == kEnd)
                break;
            uint32_t p = pv & kNodeMask;
            if (pv & kCross) {
                uint32_t lev = clev[p];
                if (lev >= 1 && lev <= (uint32_t)kPushLevels) {
                    unsigned int k = atomicAdd(&pcnt[lev - 1], 1u);
                    if (k < (unsigned)kPushStage) {
                        pstage[lev - 1][k] = node;
                        break;
                    }
                }
                bad |= !L.push(lev, c0, node);   // a full stage or a higher level
                break;
            }
            uint32_t slot = p - c0;
            if (p < c0 || slot >= m) {
                bad = true;
                break;
            }
            uint2 lr = kid[slot];
            uint32_t sib = lr.x == node ? lr.y : lr.x;
            // a leaf sibling of this chunk: its record was written before the
            // barrier and never changes here, so its load need not wait for
            // the arrival order and overlaps the atomic
            bool sib_leaf = sib >= N - 1 && sib - (N - 1) - c0 < m;
            double olo[3], ohi[3];
            uint32_t ot0 = 0, ot1 = 0;
            if (sib_leaf)
                NodeIO<TP>::get_box(tree, N, sib, olo, ohi, ot0, ot1);
            unsigned int old = __hip_atomic_fetch_add(&cnt[slot], 1u, __ATOMIC_ACQ_REL,
                                                      __HIP_MEMORY_SCOPE_WORKGROUP);
            if (old == 0)
                break;
            if (lr.x != node && lr.y != node) {
                bad = true;
                break;
            }
            if (sib_leaf) {
                // loaded above
            } else if (sib < N - 1 && sib - c0 < m) {
                const LBox &o = innb[sib - c0];
                for (int d = 0; d < 3; ++d) {
                    olo[d] = o.lo[d];
                    ohi[d] = o.hi[d];
                }
                ot0 = o.t0;
                ot1 = o.t1;
            } else {
                bad = true;
                break;
            }
            if (time_overlap(t0, t1, ot0, ot1) && space_overlap(lo, hi, olo, ohi))
                stage.push(seeds, lr.x, lr.y);
            unite(lo, hi, t0, t1, olo, ohi, ot0, ot1);
            for (int d = 0; d < 3; ++d) {
                innb[slot].lo[d] = lo[d];
                innb[slot].hi[d] = hi[d];
            }
            innb[slot].t0 = t0;
            innb[slot].t1 = t1;
            node = p;
            pv = par_in[slot];
        }
    }
    __syncthreads();
    // Space for the staged seeds (lane 0) and for level t's staged hand-offs
    // (lane t) is reserved now; the atomics' round trips overlap the record
    // pass below.
    uint32_t res = 0;
    if (t == 0) {
        uint32_t ms = sn < (unsigned)kSeedStage ? sn : (unsigned)kSeedStage;
        res = ms ? seeds.reserve(ms) : 0u;
    } else if (t <= (uint32_t)kPushLevels) {
        uint32_t c = pcnt[t - 1] < (unsigned)kPushStage ? pcnt[t - 1] : (unsigned)kPushStage;
        if (c)
            res = atomicAdd(&L.count[L.base[t] + (uint32_t)((uint64_t)c0 >> refit_shift(t))], c);
    }
    // inner nodes completed here (both children arrived) go out in one pass
    if (TP == CD_FP64) {
        // Four lanes per 64-byte record, 16 bytes each: every store
        // instruction of a wave writes 16 consecutive records (1 KB of whole
        // lines), so the stores can bypass the caches (non-temporal) without
        // partial-line writes.
        typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            uint32_t x = t + (uint32_t)kRefitChunk * (uint32_t)j;
            uint32_t r = x >> 2, q = x & 3u;
            uint32_t p = c0 + r;
            if (p + 1 < N && cnt[r] == 2) {
                const LBox &o = innb[r];
                u64x2 v;
                if (q == 0) {
                    v.x = __builtin_bit_cast(unsigned long long, o.lo[0]);
                    v.y = __builtin_bit_cast(unsigned long long, o.lo[1]);
                } else if (q == 1) {
                    v.x = __builtin_bit_cast(unsigned long long, o.lo[2]);
                    v.y = __builtin_bit_cast(unsigned long long, o.hi[0]);
                } else if (q == 2) {
                    v.x = __builtin_bit_cast(unsigned long long, o.hi[1]);
                    v.y = __builtin_bit_cast(unsigned long long, o.hi[2]);
                } else {
                    v.x = (unsigned long long)o.t0 | ((unsigned long long)o.t1 << 32);
                    v.y = (unsigned long long)kid[r].x | ((unsigned long long)esc_w[j] << 32);
                }
                __builtin_nontemporal_store(v, (u64x2 *)((Node64 *)tree + p) + q);
            }
        }
    } else {
        // FP32: two lanes per 32-byte box record, then one lane per 8-byte
        // link record; the unions of float-valued boxes are exact in float
        typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
        typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
        for (uint32_t x = t; x < 2u * (uint32_t)kRefitChunk; x += (uint32_t)kRefitChunk) {
            uint32_t r = x >> 1, q = x & 1u;
            uint32_t p = c0 + r;
            if (p + 1 < N && cnt[r] == 2) {
                const LBox &o = innb[r];
                u32x4 v;
                if (q == 0) {
                    v.x = __float_as_uint(__double2float_rd(o.lo[0]));
                    v.y = __float_as_uint(__double2float_rd(o.lo[1]));
                    v.z = __float_as_uint(__double2float_rd(o.lo[2]));
                    v.w = __float_as_uint(__double2float_ru(o.hi[0]));
                } else {
                    v.x = __float_as_uint(__double2float_ru(o.hi[1]));
                    v.y = __float_as_uint(__double2float_ru(o.hi[2]));
                    v.z = o.t0;
                    v.w = o.t1;
                }
                __builtin_nontemporal_store(v, (u32x4 *)((Box32 *)tree + p) + q);
            }
        }
        uint32_t p = c0 + t;
        if (p + 1 < N && cnt[t] == 2) {
            u32x2 l = {kid[t].x, esc_w[0]};
            Link *lrec = (Link *)((Box32 *)tree + (2 * (size_t)N - 1));
            __builtin_nontemporal_store(l, (u32x2 *)(lrec + p));
        }
    }
    if (t == 0)
        sbase = res;
    else if (t <= (uint32_t)kPushLevels)
        pbase[t - 1] = res;
    __syncthreads();
    {
        uint32_t ms = sn < (unsigned)kSeedStage ? sn : (unsigned)kSeedStage;
        for (uint32_t k = t; k < ms; k += blockDim.x)
            if (sbase + k < seeds.cap)
                seeds.items[sbase + k] = sbuf[k];
    }
    for (int lv = 0; lv < kPushLevels; ++lv) {
        uint32_t c = pcnt[lv] < (unsigned)kPushStage ? pcnt[lv] : (unsigned)kPushStage;
        uint32_t slot = L.base[lv + 1] + (uint32_t)((uint64_t)c0 >> refit_shift((uint32_t)lv + 1));
        for (uint32_t k = t; k < c; k += blockDim.x) {
            uint32_t at = pbase[lv] + k;
            if (at < (unsigned)kRefitListCap)
                L.items[(size_t)slot * kRefitListCap + at] = pstage[lv][k];
            else
                bad = true;
        }
    }
    if (bad)
        atomicOr(err, 2u);
}

// Phase k >= 1: one workgroup per level-k block climbs from the nodes queued
// for it, in global memory with workgroup-scope arrival counters, through the
// nodes of level k; a parent of a higher level gets the node queued instead.
// What a level climb needs to know about the parent pv points to, before
// its arrival atomic: the pointer itself, the parent's level, children, skip
// link and own parent pointer (kEnd or an id out of range: pointer only).
struct PMeta {
    uint32_t pv, lev, esc, ppv;
    uint2 kids;
};
__device__ inline PMeta parent_meta(uint32_t N, uint32_t pv, const uint32_t *parent,
                                    const uint2 *kids, const LinkSink &links,
                                    const uint8_t *clev)
{
    PMeta m;
    m.pv = pv;
    m.lev = 0;
    m.esc = kEnd;
    m.ppv = kEnd;
    m.kids = make_uint2(kEnd, kEnd);
    uint32_t p = pv & kNodeMask;
    if (pv != kEnd && p < N - 1) {
        m.lev = clev[p];
        m.kids = kids[p];
        m.esc = links.esc_of(p);
        m.ppv = parent[p];
    }
    return m;
}

template <int TP>
__global__ __launch_bounds__(kRefitLevelThreads) void k_refit_level(
    uint32_t N, uint32_t lev, const uint32_t *__restrict__ parent, const uint2 *__restrict__ kids,
    LinkSink links, const uint8_t *clev, void *tree, unsigned int *arrive,
    RefitLists L, SeedSink seeds, unsigned int *err)
{
    __shared__ uint2 sbuf[kSeedStage];
    __shared__ unsigned int sn, sbase;
    const SeedStage stage{sbuf, &sn};
    if (threadIdx.x == 0)
        sn = 0;
    __syncthreads();
    uint32_t blk = blockIdx.x;
    uint32_t n = L.count[L.base[lev] + blk];
    n = n < (uint32_t)kRefitListCap ? n : (uint32_t)kRefitListCap;
    const uint32_t *list = L.items + (size_t)(L.base[lev] + blk) * kRefitListCap;
    uint64_t first_leaf = (uint64_t)blk << refit_shift(lev);
    bool ok = true;
    for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) {
        uint32_t node = list[j];
        if (node >= 2 * N - 1) {
            ok = false;
            continue;
        }
        double lo[3], hi[3];
        uint32_t t0, t1;
        NodeIO<TP>::get_box(tree, N, node, lo, hi, t0, t1);
        // Everything about a parent that does not depend on the arrival order
        // (its level, children, skip link and own parent) is loaded one step
        // ahead, alongside the previous step's sibling box, so a step waits on
        // the arrival atomic and the sibling's box only.
        PMeta cur = parent_meta(N, parent[node], parent, kids, links, clev);
        for (int guard = 0;; ++guard) {
            if (cur.pv == kEnd)
                break;
            uint32_t p = cur.pv & kNodeMask;
            if (p >= N - 1 || guard > 160) {
                ok = false;
                break;
            }
            if (cur.lev > lev) {
                ok &= L.push(cur.lev, first_leaf, node);
                break;
            }
            unsigned int old = __hip_atomic_fetch_add(&arrive[p], 1u, __ATOMIC_ACQ_REL,
                                                      __HIP_MEMORY_SCOPE_WORKGROUP);
            if (old == 0)
                break;
            PMeta nxt = parent_meta(N, cur.ppv, parent, kids, links, clev);
            uint2 lr = cur.kids;
            if (lr.x != node && lr.y != node) {
                ok = false;
                break;
            }
            uint32_t sib = lr.x == node ? lr.y : lr.x;
            double olo[3], ohi[3];
            uint32_t ot0, ot1;
            NodeIO<TP>::get_box(tree, N, sib, olo, ohi, ot0, ot1);
            if (time_overlap(t0, t1, ot0, ot1) && space_overlap(lo, hi, olo, ohi))
                stage.push(seeds, lr.x, lr.y);
            unite(lo, hi, t0, t1, olo, ohi, ot0, ot1);
            NodeIO<TP>::put(tree, N, p, lo, hi, t0, t1, lr.x, cur.esc);
            node = p;
            cur = nxt;
        }
    }
    stage.flush(seeds, &sbase);
    if (!ok)
        atomicOr(err, 2u);
}

uint32_t refit_levels(uint32_t N)
{
    uint32_t lev = 0;
    while (N > 1 && ((uint64_t)(N - 1) >> refit_shift(lev)) != 0)
        ++lev;
    return lev;
}

size_t refit_list_slots(uint32_t N, uint32_t *base)
{
    uint32_t L = refit_levels(N);
    size_t slots = 0;
    for (uint32_t k = 0; k <= L + 1 && k < kRefitMaxLevels; ++k) {
        if (base)
            base[k] = (uint32_t)slots;
        if (k >= 1)
            slots += ((uint64_t)N + (1ull << refit_shift(k)) - 1) >> refit_shift(k);
    }
    return slots;
}

hipError_t launch_refit(int tree_precision, uint32_t N, const uint32_t *parent,
                        const uint2 *kids,
                        const LinkSink &links, const uint8_t *clev, unsigned int *arrive,
                        uint32_t *list_items, uint32_t *list_count, void *tree,
                        const SeedSink &seeds, unsigned int *err, hipStream_t s)
{
    if (N == 0)
        return hipSuccess;
    RefitLists L{};
    size_t slots = refit_list_slots(N, L.base);
    L.items = list_items;
    L.count = list_count;
    uint32_t levels = refit_levels(N);
    hipError_t e = hipSuccess;
    if (levels > 0) {
        e = launch_fill_u32(list_count, 0u, slots, s);
        if (e == hipSuccess)
            e = launch_fill_u32(arrive, 0u, N - 1, s);
        if (e != hipSuccess)
            return e;
    }
    uint32_t nchunks = nblk(N, kRefitChunk);
    if (tree_precision == CD_FP64)
        k_refit_chunks<CD_FP64><<<nchunks, kRefitChunk, 0, s>>>(N, parent, kids, links, clev,
                                                                 tree, L, seeds, err);
    else
        k_refit_chunks<CD_FP32><<<nchunks, kRefitChunk, 0, s>>>(N, parent, kids, links, clev,
                                                                 tree, L, seeds, err);
    e = hipGetLastError();
    for (uint32_t k = 1; k <= levels && e == hipSuccess; ++k) {
        uint32_t nb = (uint32_t)(((uint64_t)N + (1ull << refit_shift(k)) - 1) >> refit_shift(k));
        if (tree_precision == CD_FP64)
            k_refit_level<CD_FP64><<<nb, kRefitLevelThreads, 0, s>>>(
                N, k, parent, kids, links, clev, tree, arrive, L, seeds, err);
        else
            k_refit_level<CD_FP32><<<nb, kRefitLevelThreads, 0, s>>>(
                N, k, parent, kids, links, clev, tree, arrive, L, seeds, err);
        e = hipGetLastError();
    }
    return e;
}

} // namespace cd
