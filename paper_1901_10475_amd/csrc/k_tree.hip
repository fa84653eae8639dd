// k_tree.hip -- Morton keys, Karras hierarchy and the atomic bottom-up refit.
//
// The tree is the AABB tree of Sec. 3.2 (leaves hold object boxes, every inner
// box contains the boxes below it) built in bulk over 4D boxes: the time
// dimension enters through the key, whose high bits are the box's time slab
// (t0 / slab_ticks) and whose low 30 bits are the Morton code of its centre.
// Sorting by this key puts each time slab in one contiguous subtree; the
// hierarchy (Karras 2012) is built over the sorted keys with one thread per
// inner node, and each inner box (space and time) is set to the exact union of
// its two children by a bottom-up pass in which the second of the two threads
// reaching a node computes it.
#include "cd_internal.h"

namespace cd {

static inline unsigned nblk(uint64_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

// ---- scene bounds of the box centres -------------------------------------------------

// The frame only shapes the tree (codes outside it are clamped), so a strided
// sample of about 2^18 boxes is enough.
template <int PREC>
__global__ __launch_bounds__(256) void k_bounds(BoxView b, uint32_t N, uint32_t stride,
                                                unsigned long long *bounds)
{
    __shared__ unsigned long long red[6][4];
    unsigned long long mn[3] = {~0ull, ~0ull, ~0ull}, mx[3] = {0ull, 0ull, 0ull};
    for (uint64_t k = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * stride; k < N;
         k += (uint64_t)gridDim.x * blockDim.x * stride) {
        double lo[3], hi[3];
        load_box<PREC>(b, k, lo, hi);
        for (int d = 0; d < 3; ++d) {
            unsigned long long c = ordered_bits(0.5 * (lo[d] + hi[d]));
            mn[d] = c < mn[d] ? c : mn[d];
            mx[d] = c > mx[d] ? c : mx[d];
        }
    }
    for (int d = 0; d < 3; ++d) {
        for (int o = 32; o >= 1; o >>= 1) {
            unsigned long long a = __shfl_xor(mn[d], o, 64), c = __shfl_xor(mx[d], o, 64);
            mn[d] = a < mn[d] ? a : mn[d];
            mx[d] = c > mx[d] ? c : mx[d];
        }
    }
    int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int d = 0; d < 3; ++d) {
            red[d][w] = mn[d];
            red[3 + d][w] = mx[d];
        }
    __syncthreads();
    if (threadIdx.x < 3) {
        int d = threadIdx.x;
        unsigned long long a = red[d][0], c = red[3 + d][0];
        for (int ww = 1; ww < 4; ++ww) {
            a = red[d][ww] < a ? red[d][ww] : a;
            c = red[3 + d][ww] > c ? red[3 + d][ww] : c;
        }
        atomicMin(&bounds[d], a);
        atomicMax(&bounds[3 + d], c);
    }
}

hipError_t launch_bounds(const BoxView &b, int precision, uint32_t N, unsigned long long *bounds,
                         hipStream_t s)
{
    hipError_t e = launch_fill_u64(bounds, ~0ull, 3, s);
    if (e == hipSuccess)
        e = launch_fill_u64(bounds + 3, 0ull, 3, s);
    if (e != hipSuccess || N == 0)
        return e;
    uint32_t stride = N > (1u << 18) ? N >> 18 : 1u;
    unsigned g = nblk((N + stride - 1) / stride, 256);
    g = g > 1024 ? 1024 : g;
    if (precision == CD_FP64)
        k_bounds<CD_FP64><<<g, 256, 0, s>>>(b, N, stride, bounds);
    else
        k_bounds<CD_FP32><<<g, 256, 0, s>>>(b, N, stride, bounds);
    return hipGetLastError();
}

// ---- keys ------------------------------------------------------------------------------

// morton[k] (slab-local sort input) and kv[k] = {slab << 32 | morton, k}
// (device-wide sort input).  err bit 1: a box's slab disagrees with the slab
// hint or exceeds max_slab.
template <int PREC>
__global__ void k_keys(BoxView b, uint32_t N, uint32_t slab_ticks, uint32_t max_slab,
                       uint32_t slab_size, const unsigned long long *bounds, uint32_t *morton,
                       KV *kv, unsigned int *err)
{
    uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N)
        return;
    double mn[3], inv[3];
    for (int d = 0; d < 3; ++d) {   // the frame is read only when codes are formed here
        mn[d] = inv[d] = 0.0;
        if (!b.code) {
            mn[d] = from_ordered_bits(bounds[d]);
            double ext = from_ordered_bits(bounds[3 + d]) - mn[d];
            inv[d] = ext > 0.0 ? 1.0 / ext : 0.0;
        }
    }
    uint32_t m;
    if (b.code) {
        m = b.code[k];
    } else {
        double lo[3], hi[3];
        load_box<PREC>(b, k, lo, hi);
        m = morton30(0.5 * (lo[0] + hi[0]), 0.5 * (lo[1] + hi[1]), 0.5 * (lo[2] + hi[2]), mn,
                     inv);
    }
    uint32_t slab = b.t0[k] / slab_ticks;
    if (slab > max_slab) {
        atomicOr(err, 1u);
        slab = max_slab;
    }
    if (slab_size && slab != k / slab_size)
        atomicOr(err, 1u);
    if (morton)
        morton[k] = m;
    if (kv) {
        KV x;
        x.key = ((uint64_t)slab << 32) | m;
        x.val = k;
        x.pad = 0;
        kv[k] = x;
    }
}

hipError_t launch_keys(const BoxView &b, int precision, uint32_t N, uint32_t slab_ticks,
                       uint32_t max_slab, uint32_t slab_size, const unsigned long long *bounds,
                       uint32_t *morton, KV *kv, unsigned int *err, hipStream_t s)
{
    if (N == 0)
        return hipSuccess;
    if (precision == CD_FP64)
        k_keys<CD_FP64><<<nblk(N, 256), 256, 0, s>>>(b, N, slab_ticks, max_slab, slab_size,
                                                     bounds, morton, kv, err);
    else
        k_keys<CD_FP32><<<nblk(N, 256), 256, 0, s>>>(b, N, slab_ticks, max_slab, slab_size,
                                                     bounds, morton, kv, err);
    return hipGetLastError();
}

__global__ void k_unpack_kv(const KV *kv, uint32_t N, uint64_t *keys, uint32_t *idx)
{
    uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N)
        return;
    KV x = kv[k];
    keys[k] = x.key;
    idx[k] = x.val;
}

hipError_t launch_unpack_kv(const KV *kv, uint32_t N, uint64_t *keys, uint32_t *idx,
                            hipStream_t s)
{
    if (N == 0)
        return hipSuccess;
    k_unpack_kv<<<nblk(N, 256), 256, 0, s>>>(kv, N, keys, idx);
    return hipGetLastError();
}

// ---- Karras hierarchy + skip links ------------------------------------------------------
//
// Thread i builds inner node i.  Outputs: kids[i] = {left, right};
// links[id] = {left child (inner) or 0 (leaf), skip link} for every node id;
// clev[i] = refit level of node i (the smallest k whose level-k blocks of
// refit_block(k) leaves contain its whole leaf range); parent[child] = i, with
// kCross set when clev[i] > 0.

__global__ void k_karras(const uint64_t *__restrict__ keys, uint32_t N, uint2 *kids, Link *links,
                         uint32_t *parent, uint8_t *clev, bool leaf_links)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i + 1 >= N)
        return;
    KeyArray K{keys};
    KarrasNode nd = karras_node(K, N, i);
    uint32_t lev = 0;
    while ((uint64_t)(nd.first >> refit_shift(lev)) != (uint64_t)(nd.last >> refit_shift(lev)))
        ++lev;
    clev[i] = (uint8_t)lev;
    uint32_t pv = i | (lev > 0 ? kCross : 0u);
    parent[nd.left] = pv;
    parent[nd.right] = pv;
    if (i == 0)
        parent[0] = kEnd;
    kids[i] = make_uint2(nd.left, nd.right);
    Link li;
    li.link = nd.left;
    li.esc = karras_escape(K, N, nd.last);
    links[i] = li;
    if (!leaf_links)
        return;
    Link lf;
    lf.link = 0;
    lf.esc = karras_escape(K, N, i);
    links[N - 1 + i] = lf;
    if (i == N - 2) {
        Link ll;
        ll.link = 0;
        ll.esc = kEnd;
        links[2 * N - 2] = ll;
    }
}

// Same nodes as k_karras for time-major slabs: one workgroup per slab holds
// the slab's sorted 32-bit codes in LDS and computes every inner node whose
// index lies in the slab (node i's searches always compare key i, a key of the
// slab, so the slab-bits-only view of other slabs is exact).  The binary
// searches then wait on LDS instead of L2.  Leaf skip links come from the
// slab build.
__global__ __launch_bounds__(kSegThreads) void k_karras_slabs(const uint64_t *__restrict__ keys,
                                                              uint32_t N, uint32_t slab_size,
                                                              uint2 *kids, Link *links,
                                                              uint32_t *parent, uint8_t *clev)
{
    __shared__ uint32_t sk[kSegCap];
    uint64_t slab = blockIdx.x;
    uint64_t base = slab * slab_size;
    uint32_t m = (uint32_t)(base + slab_size <= N ? slab_size : N - base);
    for (uint32_t k = threadIdx.x; k < m; k += blockDim.x)
        sk[k] = (uint32_t)keys[base + k];
    __syncthreads();
    const SlabKeys K{sk, base, slab_size, slab << 32};
    for (uint32_t k = threadIdx.x; k < m; k += blockDim.x) {
        uint32_t i = (uint32_t)(base + k);
        if (i + 1 >= N)
            break;
        KarrasNode nd = karras_node(K, N, i);
        uint32_t lev = 0;
        while ((uint64_t)(nd.first >> refit_shift(lev)) != (uint64_t)(nd.last >> refit_shift(lev)))
            ++lev;
        clev[i] = (uint8_t)lev;
        uint32_t pv = i | (lev > 0 ? kCross : 0u);
        parent[nd.left] = pv;
        parent[nd.right] = pv;
        if (i == 0)
            parent[0] = kEnd;
        kids[i] = make_uint2(nd.left, nd.right);
        Link li;
        li.link = nd.left;
        li.esc = karras_escape(K, N, nd.last);
        links[i] = li;
    }
}

__global__ void k_single_leaf(Link *links, uint32_t *parent)
{
    Link l;
    l.link = 0;
    l.esc = kEnd;
    links[0] = l;
    parent[0] = kEnd;
}

hipError_t launch_karras(const uint64_t *keys, uint32_t N, uint2 *kids, Link *links,
                         uint32_t *parent, uint8_t *clev, bool leaf_links, hipStream_t s)
{
    if (N == 0)
        return hipSuccess;
    if (N == 1) {
        k_single_leaf<<<1, 1, 0, s>>>(links, parent);
        return hipGetLastError();
    }
    k_karras<<<nblk(N - 1, 256), 256, 0, s>>>(keys, N, kids, links, parent, clev, leaf_links);
    return hipGetLastError();
}

hipError_t launch_karras_slabs(const uint64_t *keys, uint32_t N, uint32_t slab_size, uint2 *kids,
                               Link *links, uint32_t *parent, uint8_t *clev, hipStream_t s)
{
    if (N <= 1 || slab_size == 0 || (int64_t)slab_size > kSegCap)
        return hipErrorInvalidValue;
    uint32_t nslabs = (uint32_t)((N + slab_size - 1) / slab_size);
    k_karras_slabs<<<nslabs, kSegThreads, 0, s>>>(keys, N, slab_size, kids, links, parent, clev);
    return hipGetLastError();
}

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
//      children, arrival counters and computed inner boxes are staged in LDS
//      (77 KB, two workgroups per CU); a sibling leaf is read back from its
//      record, written before the barrier and still in L2.  Computed inner
//      records are written out in one coalesced pass at the end.
//   level k >= 1: one workgroup per level-k block climbs, in global memory with
//      workgroup-scope counters, from the nodes queued for it by lower levels.
// A climb that meets a parent of a higher level queues the node for that level
// and block.  Kernel boundaries order each level's writes before the next.

// Per-workgroup seed staging: lanes append to LDS; a full stage or the end of
// the kernel flushes it with one global atomic.
struct SeedStage {
    uint2 *buf;            // LDS, kSeedStage entries
    unsigned int *n;       // LDS counter
    __device__ void push(const SeedSink &sink, uint32_t a, uint32_t b) const
    {
        unsigned int k = atomicAdd(n, 1u);
        if (k < (unsigned)kSeedStage) {
            buf[k] = make_uint2(a, b);
        } else {  // stage full: this one goes straight out
            uint2 one = make_uint2(a, b);
            sink.put_many(&one, 1, sink.reserve(1));
        }
    }
    // all threads of the block call this after the last push
    __device__ void flush(const SeedSink &sink, unsigned int *base_lds) const
    {
        __syncthreads();
        uint32_t m = *n < (unsigned)kSeedStage ? *n : (unsigned)kSeedStage;
        if (threadIdx.x == 0)
            *base_lds = m ? sink.reserve(m) : 0u;
        __syncthreads();
        for (uint32_t k = threadIdx.x; k < m; k += blockDim.x)
            if (*base_lds + k < sink.cap)
                sink.items[*base_lds + k] = buf[k];
    }
};

template <int BP, int TP>
__global__ __launch_bounds__(kRefitChunk) void k_refit_chunks(
    BoxView b, uint32_t N, const uint32_t *__restrict__ idx, const uint32_t *__restrict__ parent,
    const uint2 *__restrict__ kids, const Link *__restrict__ links, const uint8_t *clev,
    void *tree, RefitLists L, SeedSink seeds, unsigned int *err)
{
    __shared__ LBox innb[kRefitChunk];
    __shared__ uint2 kid[kRefitChunk];
    __shared__ uint32_t par_leaf[kRefitChunk], par_in[kRefitChunk];
    __shared__ unsigned int cnt[kRefitChunk];
    __shared__ uint2 sbuf[kSeedStage];
    __shared__ unsigned int sn, sbase;
    const SeedStage stage{sbuf, &sn};
    const uint32_t t = threadIdx.x;
    if (t == 0)
        sn = 0;
    const uint32_t c = xcd_block(blockIdx.x, gridDim.x);
    const uint32_t c0 = c * (uint32_t)kRefitChunk;
    const uint32_t m = N - c0 < (uint32_t)kRefitChunk ? N - c0 : (uint32_t)kRefitChunk;
    double lo[3], hi[3];
    uint32_t t0 = 0, t1 = 0;
    bool bad = false;
    if (t < m && idx) {
        uint32_t i = c0 + t;
        uint32_t src = idx[i];
        if (src >= N) {
            bad = true;
            src = 0;
        }
        load_box<BP>(b, src, lo, hi);
        if (TP == CD_FP32 && BP == CD_FP64) {
            // the unions must see the rounded leaves, as the traversal does
            for (int d = 0; d < 3; ++d) {
                lo[d] = __double2float_rd(lo[d]);
                hi[d] = __double2float_ru(hi[d]);
            }
        }
        t0 = b.t0[src];
        t1 = b.t1[src];
        uint32_t leaf = N - 1 + i;
        NodeIO<TP>::put(tree, N, leaf, lo, hi, t0, t1, b.obj[src], links[leaf].esc);
        par_leaf[t] = parent[leaf];
    } else if (t < m) {
        // leaf records already written in sorted order by the slab build
        uint32_t leaf = N - 1 + c0 + t;
        NodeIO<TP>::get_box(tree, N, leaf, lo, hi, t0, t1);
        par_leaf[t] = parent[leaf];
    }
    if (c0 + t + 1 < N) {  // inner node c0 + t exists
        kid[t] = kids[c0 + t];
        par_in[t] = parent[c0 + t];
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
                bad |= !L.push(clev[p], c0, node);
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
    // inner nodes completed here (both children arrived) go out in one pass
    if (c0 + t + 1 < N && cnt[t] == 2) {
        uint32_t p = c0 + t;
        NodeIO<TP>::put(tree, N, p, innb[t].lo, innb[t].hi, innb[t].t0, innb[t].t1, kid[t].x,
                        links[p].esc);
    }
    stage.flush(seeds, &sbase);
    if (bad)
        atomicOr(err, 2u);
}

// Phase k >= 1: one workgroup per level-k block climbs from the nodes queued
// for it, in global memory with workgroup-scope arrival counters, through the
// nodes of level k; a parent of a higher level gets the node queued instead.
template <int TP>
__global__ __launch_bounds__(kRefitLevelThreads) void k_refit_level(
    uint32_t N, uint32_t lev, const uint32_t *__restrict__ parent, const uint2 *__restrict__ kids,
    const Link *__restrict__ links, const uint8_t *clev, void *tree, unsigned int *arrive,
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
        uint32_t pv = parent[node];
        for (int guard = 0;; ++guard) {
            if (pv == kEnd)
                break;
            uint32_t p = pv & kNodeMask;
            if (p >= N - 1 || guard > 160) {
                ok = false;
                break;
            }
            // everything about p that does not depend on the arrival order is
            // loaded at once; only the sibling's box waits for the acquire
            uint32_t pl = clev[p];
            uint2 lr = kids[p];
            uint32_t pesc = links[p].esc;
            uint32_t ppv = parent[p];
            if (pl > lev) {
                ok &= L.push(pl, first_leaf, node);
                break;
            }
            unsigned int old = __hip_atomic_fetch_add(&arrive[p], 1u, __ATOMIC_ACQ_REL,
                                                      __HIP_MEMORY_SCOPE_WORKGROUP);
            if (old == 0)
                break;
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
            NodeIO<TP>::put(tree, N, p, lo, hi, t0, t1, lr.x, pesc);
            node = p;
            pv = ppv;
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

hipError_t launch_refit(const BoxView &b, int box_precision, int tree_precision, uint32_t N,
                        const uint32_t *idx, const uint32_t *parent, const uint2 *kids,
                        const Link *links, const uint8_t *clev, unsigned int *arrive,
                        uint32_t *list_items, uint32_t *list_count, void *tree,
                        const SeedSink &seeds, unsigned int *err, hipStream_t s)
{
    if (N == 0)
        return hipSuccess;
    RefitLists L;
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
    if (box_precision == CD_FP64 && tree_precision == CD_FP64)
        k_refit_chunks<CD_FP64, CD_FP64><<<nchunks, kRefitChunk, 0, s>>>(
            b, N, idx, parent, kids, links, clev, tree, L, seeds, err);
    else if (box_precision == CD_FP64)
        k_refit_chunks<CD_FP64, CD_FP32><<<nchunks, kRefitChunk, 0, s>>>(
            b, N, idx, parent, kids, links, clev, tree, L, seeds, err);
    else
        k_refit_chunks<CD_FP32, CD_FP32><<<nchunks, kRefitChunk, 0, s>>>(
            b, N, idx, parent, kids, links, clev, tree, L, seeds, err);
    e = hipGetLastError();
    for (uint32_t k = 1; k <= levels && e == hipSuccess; ++k) {
        uint32_t nb = (uint32_t)(((uint64_t)N + (1ull << refit_shift(k)) - 1) >> refit_shift(k));
        if (tree_precision == CD_FP64)
            k_refit_level<CD_FP64><<<nb, kRefitLevelThreads, 0, s>>>(N, k, parent, kids, links, clev,
                                                              tree, arrive, L, seeds, err);
        else
            k_refit_level<CD_FP32><<<nb, kRefitLevelThreads, 0, s>>>(N, k, parent, kids, links, clev,
                                                              tree, arrive, L, seeds, err);
        e = hipGetLastError();
    }
    return e;
}

} // namespace cd
