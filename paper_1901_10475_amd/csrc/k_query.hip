// k_query.hip -- the n-to-n self-traversal and the canonical pair list.
//
// One lane per leaf (query box), leaves taken in sorted key order so that the
// lanes of a wave hold neighbouring boxes and walk nearly the same nodes.  A
// query visits only the part of the tree to the right of its own leaf: it
// starts at its leaf's skip link (the next node in pre-order after the leaf)
// and follows, without a stack, the left-child link into overlapping inner
// nodes and the skip link past everything else.  Every unordered pair of
// leaves is therefore tested once, from the left one.  The node test is the
// 4D overlap of Def. 4D Occupancy Region: half-open integer time tags and
// closed spatial extents; leaves of the same object are skipped, as queryObject
// excludes the queried object (Sec. 4.4).
//
// Because keys are time-major, everything right of a node whose earliest tag
// starts at t0 begins no earlier than slab(t0) * slab_ticks, so a query stops as
// soon as t0_min(node) >= t1(query) + slab_ticks - 1.
//
// Records are appended through one atomic per wave per step: the lanes with a
// hit are counted with a ballot, the lowest one reserves the range, and each
// lane writes at its prefix position.
#include "cd_internal.h"

namespace cd {

static inline unsigned nblk(uint64_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

#ifdef CD_COUNTERS
// Executed-work counters of the traversal (the diagnostic build only), in the
// order of cd_counters: box-box tests, tests of two leaves, tests of a leaf
// and an inner node, tests of two overlapping leaves of different objects
// (each one appended record), node pairs expanded, per-leaf walk steps.  Per
// object: tests with a leaf box of that object on one side (g_visits, when
// the caller bound an array).
__device__ unsigned long long g_ctr[kCounterWords];
__device__ uint32_t *g_visits;
__device__ uint32_t g_nobj;

// Wave sum, one atomic per wave; every lane of the wave must call it.
__device__ inline void ctr_wave_add(int k, uint32_t v)
{
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0 && v)
        atomicAdd(&g_ctr[k], (unsigned long long)v);
}

__device__ inline void ctr_visit(uint32_t obj)
{
    uint32_t *vis = g_visits;
    if (vis && obj < g_nobj)
        atomicAdd(&vis[obj], 1u);
}
#endif

template <int TP>
struct Q;

template <>
struct Q<CD_FP64> {
    using F = double;
    __device__ static void load(const void *tree, uint32_t N, uint32_t id, F lo[3], F hi[3],
                                uint32_t &t0, uint32_t &t1, uint32_t &link, uint32_t &esc)
    {
        const Node64 *n = (const Node64 *)tree + id;
        double4 a = *(const double4 *)&n->lo[0];   // lo0 lo1 lo2 hi0
        double2 c = *(const double2 *)&n->hi[1];   // hi1 hi2
        uint4 u = *(const uint4 *)&n->t0;          // t0 t1 link esc
        lo[0] = a.x;
        lo[1] = a.y;
        lo[2] = a.z;
        hi[0] = a.w;
        hi[1] = c.x;
        hi[2] = c.y;
        t0 = u.x;
        t1 = u.y;
        link = u.z;
        esc = u.w;
    }
    // the box and tags alone (the links share the record's last 16 bytes)
    __device__ static void load_box(const void *tree, uint32_t N, uint32_t id, F lo[3],
                                    F hi[3], uint32_t &t0, uint32_t &t1)
    {
        uint32_t link, esc;
        load(tree, N, id, lo, hi, t0, t1, link, esc);
    }
};

template <>
struct Q<CD_FP32> {
    using F = float;
    __device__ static void load(const void *tree, uint32_t N, uint32_t id, F lo[3], F hi[3],
                                uint32_t &t0, uint32_t &t1, uint32_t &link, uint32_t &esc)
    {
        const Box32 *b = (const Box32 *)tree + id;
        float4 a = *(const float4 *)&b->lo[0];     // lo0 lo1 lo2 hi0
        uint4 c = *(const uint4 *)&b->hi[1];       // hi1 hi2 t0 t1
        uint2 l = *((const uint2 *)((const Box32 *)tree + (2 * (size_t)N - 1)) + id);
        lo[0] = a.x;
        lo[1] = a.y;
        lo[2] = a.z;
        hi[0] = a.w;
        hi[1] = __uint_as_float(c.x);
        hi[2] = __uint_as_float(c.y);
        t0 = c.z;
        t1 = c.w;
        link = l.x;
        esc = l.y;
    }
    // the box and tags alone: the link array is a second cache line
    __device__ static void load_box(const void *tree, uint32_t N, uint32_t id, F lo[3],
                                    F hi[3], uint32_t &t0, uint32_t &t1)
    {
        const Box32 *b = (const Box32 *)tree + id;
        float4 a = *(const float4 *)&b->lo[0];
        uint4 c = *(const uint4 *)&b->hi[1];
        lo[0] = a.x;
        lo[1] = a.y;
        lo[2] = a.z;
        hi[0] = a.w;
        hi[1] = __uint_as_float(c.x);
        hi[2] = __uint_as_float(c.y);
        t0 = c.z;
        t1 = c.w;
    }
};

// An FP64 tree built bottom-up keeps its leaf skip links in a side array
// (*side_on set by the build).
template <int TP>
__global__ __launch_bounds__(256) void k_traverse(const void *__restrict__ tree, uint32_t N,
                                                  uint32_t slab_ticks, Rec *__restrict__ out,
                                                  unsigned long long capacity,
                                                  unsigned long long *counter,
                                                  unsigned int *err, const unsigned int *run_if,
                                                  const unsigned int *side_on,
                                                  const uint32_t *__restrict__ side)
{
    using F = typename Q<TP>::F;
    if (run_if && *run_if == 0)
        return;
    const bool use_side = TP == CD_FP64 && side_on && *side_on;
    uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
    uint32_t i = blk * blockDim.x + threadIdx.x;
    if (i >= N)
        return;
    F qlo[3], qhi[3];
    uint32_t qt0, qt1, qobj, node;
    Q<TP>::load(tree, N, N - 1 + i, qlo, qhi, qt0, qt1, qobj, node);
    if (use_side)
        node = side[i];
    const uint64_t stop = (uint64_t)qt1 + slab_ticks - 1;
    const uint32_t limit = 2 * N + 2;
    const uint64_t lt = (threadIdx.x & 63) ? (~0ull >> (64 - (threadIdx.x & 63))) : 0ull;
    uint32_t steps = 0;
#ifdef CD_COUNTERS
    uint32_t c_tests = 0, c_ll = 0, c_hits = 0;
#endif
    while (node != kEnd) {
        if (++steps > limit || node >= 2 * N - 1) {
            atomicOr(err, 4u);
            break;
        }
        F lo[3], hi[3];
        uint32_t t0, t1, link, esc;
        Q<TP>::load(tree, N, node, lo, hi, t0, t1, link, esc);
        if ((uint64_t)t0 >= stop)
            break;
        bool ov = time_overlap(qt0, qt1, t0, t1) && space_overlap(qlo, qhi, lo, hi);
        bool leaf = node >= N - 1;
#ifdef CD_COUNTERS
        ++c_tests;
        c_ll += leaf ? 1u : 0u;
        c_hits += (ov && leaf && link != qobj) ? 1u : 0u;
        ctr_visit(qobj);
        if (leaf)
            ctr_visit(link);
#endif
        if (use_side && leaf)
            esc = side[node - (N - 1)];
        bool hit = ov && leaf && link != qobj;
        uint64_t m = __ballot(hit);
        if (m) {
            int leader = __ffsll((unsigned long long)m) - 1;
            unsigned long long base = 0;
            if ((int)(threadIdx.x & 63) == leader)
                base = atomicAdd(counter, (unsigned long long)__popcll(m));
            base = __shfl(base, leader, 64);
            if (hit) {
                unsigned long long pos = base + (unsigned long long)__popcll(m & lt);
                if (pos < capacity) {
                    Rec r;
                    r.i = qobj < link ? qobj : link;
                    r.j = qobj < link ? link : qobj;
                    r.tlo = qt0 > t0 ? qt0 : t0;
                    r.thi = qt1 < t1 ? qt1 : t1;
                    out[pos] = r;
                }
            }
        }
        node = (ov && !leaf) ? link : esc;
    }
#ifdef CD_COUNTERS
    if (c_tests) {
        atomicAdd(&g_ctr[0], (unsigned long long)c_tests);
        atomicAdd(&g_ctr[1], (unsigned long long)c_ll);
        atomicAdd(&g_ctr[2], (unsigned long long)(c_tests - c_ll));
        atomicAdd(&g_ctr[3], (unsigned long long)c_hits);
        atomicAdd(&g_ctr[5], (unsigned long long)c_tests);
    }
#endif
}

hipError_t launch_traverse(const void *tree, int precision, uint32_t N, uint32_t slab_ticks,
                           Rec *out, unsigned long long capacity, unsigned long long *counter,
                           unsigned int *err, const unsigned int *run_if, uint32_t threads,
                           const unsigned int *side_on, const uint32_t *side, hipStream_t s)
{
    if (N <= 1)
        return hipSuccess;
    unsigned g = nblk(N, threads);
    if (precision == CD_FP64)
        k_traverse<CD_FP64><<<g, threads, 0, s>>>(tree, N, slab_ticks, out, capacity, counter,
                                                  err, run_if, side_on, side);
    else
        k_traverse<CD_FP32><<<g, threads, 0, s>>>(tree, N, slab_ticks, out, capacity, counter,
                                                  err, run_if, nullptr, nullptr);
    return hipGetLastError();
}

// ---- node-pair self-traversal ------------------------------------------------------------------
//
// The refit records every pair of sibling nodes whose 4D boxes overlap.  Every
// overlapping pair of leaves lies under exactly one such pair (the children of
// its lowest common ancestor), and expanding an overlapping node pair into the
// overlapping pairs of their children reaches each of those leaf pairs exactly
// once.  One launch per level: a lane takes one queued pair, loads the
// children's boxes, tests the (up to) four child pairs, emits leaf pairs as
// records and queues the rest; both appends are aggregated per wave with a
// ballot and one atomic.

// Side s of a pair: a leaf stays itself, an inner node is replaced by its two
// children (kids of the tree).  Loads the boxes of the resulting nodes, and
// the leaves' object ids unless LINKS is false (FP32: the ids sit in the
// link array, a second cache line, and are then read only for leaf pairs
// whose boxes overlap).
template <int TP, bool LINKS = true>
__device__ inline bool load_side(const void *tree, const uint2 *kids, uint32_t N, uint32_t x,
                                 uint32_t ids[2], typename Q<TP>::F lo[2][3],
                                 typename Q<TP>::F hi[2][3], uint32_t t0[2], uint32_t t1[2],
                                 uint32_t lk[2], uint32_t &cnt)
{
    const uint32_t nodes = 2 * N - 1;
    uint32_t e;
    if (x >= nodes)
        return false;
    if (x >= N - 1) {
        ids[0] = x;
        if (LINKS || TP == CD_FP64) {
            Q<TP>::load(tree, N, x, lo[0], hi[0], t0[0], t1[0], lk[0], e);
        } else {
            Q<TP>::load_box(tree, N, x, lo[0], hi[0], t0[0], t1[0]);
            lk[0] = 0;
        }
        cnt = 1;
        return true;
    }
    uint2 kk = kids[x];
    if (kk.x >= nodes || kk.y >= nodes)
        return false;
    ids[0] = kk.x;
    ids[1] = kk.y;
    if (TP == CD_FP64) {   // the links share the record's cache line
        Q<TP>::load(tree, N, kk.x, lo[0], hi[0], t0[0], t1[0], lk[0], e);
        Q<TP>::load(tree, N, kk.y, lo[1], hi[1], t0[1], t1[1], lk[1], e);
        cnt = 2;
        return true;
    }
    // FP32: an inner child's link (a second cache line) is never used, its
    // children come from kids, so only a leaf child pays for the object id
    lk[0] = lk[1] = 0;
    if (LINKS && kk.x >= N - 1)
        Q<TP>::load(tree, N, kk.x, lo[0], hi[0], t0[0], t1[0], lk[0], e);
    else
        Q<TP>::load_box(tree, N, kk.x, lo[0], hi[0], t0[0], t1[0]);
    if (LINKS && kk.y >= N - 1)
        Q<TP>::load(tree, N, kk.y, lo[1], hi[1], t0[1], t1[1], lk[1], e);
    else
        Q<TP>::load_box(tree, N, kk.y, lo[1], hi[1], t0[1], t1[1]);
    cnt = 2;
    return true;
}

// One level over the n pairs of `in`, by every workgroup of the grid in turn
// (block-uniform loop: the block scan needs every thread).  COH: the queue
// entries are written and read as device-scope atomics, each coherent across
// the XCDs' separate L2 caches by itself, for a reader in the same launch.
template <int TP, bool COH = false>
__device__ inline void expand_level(const void *__restrict__ tree, const uint2 *__restrict__ kids,
                                    uint32_t N, const uint2 *__restrict__ in, uint32_t n,
                                    uint2 *__restrict__ outq, unsigned int *n_out,
                                    uint32_t out_cap, Rec *__restrict__ out,
                                    unsigned long long capacity, unsigned long long *counter,
                                    unsigned int *flags, uint32_t *wsum, unsigned int &qbase,
                                    unsigned long long &rbase)
{
    using F = typename Q<TP>::F;
#ifdef CD_COUNTERS
    constexpr bool kLinks = true;   // the node-visit counts need every leaf's object
#else
    constexpr bool kLinks = TP == CD_FP64;   // FP32: object ids only for overlapping leaf pairs
#endif
    for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
        uint32_t k = base + threadIdx.x;
        bool active = k < n;
        uint32_t ids[2][2], cnt[2] = {0, 0};
        F lo[2][2][3], hi[2][2][3];
        uint32_t t0[2][2], t1[2][2], lk[2][2];
        if (active) {
            uint2 pr;
            if (COH) {
                unsigned long long v =
                    __hip_atomic_load(reinterpret_cast<const unsigned long long *>(in + k),
                                      __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                pr = make_uint2((uint32_t)v, (uint32_t)(v >> 32));
            } else {
                pr = in[k];
            }
            bool ok = load_side<TP, kLinks>(tree, kids, N, pr.x, ids[0], lo[0], hi[0], t0[0],
                                            t1[0], lk[0], cnt[0]) &&
                      load_side<TP, kLinks>(tree, kids, N, pr.y, ids[1], lo[1], hi[1], t0[1],
                                            t1[1], lk[1], cnt[1]);
            if (!ok) {
                atomicOr(flags, 2u);
                active = false;
            }
        }
        uint32_t push_mask = 0, hit_mask = 0;
        for (int ia = 0; ia < 2; ++ia)
            for (int ic = 0; ic < 2; ++ic) {
                bool ov = active && ia < (int)cnt[0] && ic < (int)cnt[1] &&
                          time_overlap(t0[0][ia], t1[0][ia], t0[1][ic], t1[1][ic]) &&
                          space_overlap(lo[0][ia], hi[0][ia], lo[1][ic], hi[1][ic]);
                bool leaves = ov && ids[0][ia] >= N - 1 && ids[1][ic] >= N - 1;
                int bit = ia * 2 + ic;
                if (!kLinks && leaves) {
                    const uint2 *links = (const uint2 *)((const Box32 *)tree + (2 * (size_t)N - 1));
                    lk[0][ia] = links[ids[0][ia]].x;
                    lk[1][ic] = links[ids[1][ic]].x;
                }
                if (leaves && lk[0][ia] != lk[1][ic])
                    hit_mask |= 1u << bit;
                if (ov && !leaves)
                    push_mask |= 1u << bit;
            }
#ifdef CD_COUNTERS
        {
            uint32_t c_tests = 0, c_ll = 0, c_li = 0;
            for (int ia = 0; ia < 2; ++ia)
                for (int ic = 0; ic < 2; ++ic) {
                    if (!(active && ia < (int)cnt[0] && ic < (int)cnt[1]))
                        continue;
                    const bool la = ids[0][ia] >= N - 1, lc = ids[1][ic] >= N - 1;
                    ++c_tests;
                    c_ll += (la && lc) ? 1u : 0u;
                    c_li += (la != lc) ? 1u : 0u;
                    if (la)
                        ctr_visit(lk[0][ia]);
                    if (lc)
                        ctr_visit(lk[1][ic]);
                }
            ctr_wave_add(0, c_tests);
            ctr_wave_add(1, c_ll);
            ctr_wave_add(2, c_li);
            ctr_wave_add(3, (uint32_t)__popc(hit_mask));
            ctr_wave_add(4, active ? 1u : 0u);
        }
#endif
        // one scan packs both counts: pushes in the low 16 bits, hits above
        uint32_t mine = (uint32_t)__popc(push_mask) | ((uint32_t)__popc(hit_mask) << 16);
        uint32_t total;
        uint32_t pre = block_exclusive_scan(mine, wsum, &total);
        if (threadIdx.x == 0) {
            qbase = (total & 0xFFFFu) ? atomicAdd(n_out, total & 0xFFFFu) : 0u;
            rbase = (total >> 16) ? atomicAdd(counter, (unsigned long long)(total >> 16)) : 0ull;
        }
        __syncthreads();
        uint32_t q = qbase + (pre & 0xFFFFu);
        unsigned long long r = rbase + (pre >> 16);
        for (int bit = 0; bit < 4; ++bit) {
            int ia = bit >> 1, ic = bit & 1;
            if (push_mask & (1u << bit)) {
                if (q < out_cap)
                {
                    if (COH)
                        __hip_atomic_store(reinterpret_cast<unsigned long long *>(outq + q),
                                           (unsigned long long)ids[0][ia] |
                                               ((unsigned long long)ids[1][ic] << 32),
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    else
                        outq[q] = make_uint2(ids[0][ia], ids[1][ic]);
                }
                else
                    atomicOr(flags, 1u);
                ++q;
            }
            if (hit_mask & (1u << bit)) {
                if (r < capacity) {
                    uint32_t oa = lk[0][ia], oc = lk[1][ic];
                    Rec rec;
                    rec.i = oa < oc ? oa : oc;
                    rec.j = oa < oc ? oc : oa;
                    rec.tlo = t0[0][ia] > t0[1][ic] ? t0[0][ia] : t0[1][ic];
                    rec.thi = t1[0][ia] < t1[1][ic] ? t1[0][ia] : t1[1][ic];
                    out[r] = rec;
                }
                ++r;
            }
        }
        __syncthreads();
    }
}

template <int TP>
__global__ __launch_bounds__(1024) void k_expand(const void *__restrict__ tree,
                                                const uint2 *__restrict__ kids, uint32_t N,
                                                const uint2 *__restrict__ in,
                                                const unsigned int *n_in, uint32_t in_cap,
                                                uint2 *__restrict__ outq, unsigned int *n_out,
                                                uint32_t out_cap, Rec *__restrict__ out,
                                                unsigned long long capacity,
                                                unsigned long long *counter, unsigned int *flags,
                                                int gated)
{
    __shared__ uint32_t wsum[64];
    __shared__ unsigned int qbase;
    __shared__ unsigned long long rbase;
    // gated: a set flag (queue overflow, bad node, the traversal handed to the
    // per-leaf walk, or an earlier level found its queue empty) ends the
    // node-pair levels
    if (gated && *flags)
        return;
    uint32_t n = *n_in;
    n = n < in_cap ? n : in_cap;
    if (n == 0) {
        // every pair has been expanded: flag 8 tells the host (and the gate)
        if (blockIdx.x == 0 && threadIdx.x == 0)
            atomicOr(flags, 8u);
        return;
    }
    expand_level<TP>(tree, kids, N, in, n, outq, n_out, out_cap, out, capacity, counter, flags,
                     wsum, qbase, rbase);
}

hipError_t launch_expand(const void *tree, const uint2 *kids, int precision, uint32_t N,
                         const uint2 *in, const unsigned int *n_in, uint32_t in_cap, uint2 *outq,
                         unsigned int *n_out, uint32_t out_cap, Rec *out,
                         unsigned long long capacity, unsigned long long *counter,
                         unsigned int *flags, int gated, uint32_t blocks, uint32_t threads,
                         hipStream_t s)
{
    if (N <= 1)
        return hipSuccess;
    if (precision == CD_FP64)
        k_expand<CD_FP64><<<blocks, threads, 0, s>>>(tree, kids, N, in, n_in, in_cap, outq, n_out,
                                                     out_cap, out, capacity, counter, flags,
                                                     gated);
    else
        k_expand<CD_FP32><<<blocks, threads, 0, s>>>(tree, kids, N, in, n_in, in_cap, outq, n_out,
                                                     out_cap, out, capacity, counter, flags,
                                                     gated);
    return hipGetLastError();
}

// ---- every level in one launch ----------------------------------------------------------------
//
// The same levels, run by one grid that the device holds at once: the
// workgroups take a level's pairs in turn, then wait for each other at a
// counter, so the next level reads a complete queue and count.  What one
// level hands to the next -- queue entries, counts, flags -- is written and
// read as device-scope atomics, each coherent by itself across the XCDs'
// separate L2 caches, and every wave waits for its own writes to complete
// before its workgroup arrives; no fence has to write back or invalidate the
// L2s (measured: with a release/acquire arrival per workgroup the traversal
// of the 16 848-object hour took 0.91 ms, with this one 0.79 ms; one launch
// per level takes 0.53 ms, so this form is not the default).
// The grid is sized on the host to the resident capacity, so every workgroup
// being waited for is running.  The wait ends in any case: a workgroup that
// sees an overflow or bad-node flag, or waits past kGridWaitTicks of the
// 100 MHz real-time clock, sets the handover flag and leaves; the query then
// runs the per-leaf walk from a cleared count, and every other workgroup sees
// the flag at its next wait.  A level with an empty input ends the kernel in
// every workgroup alike (the count is complete when it is read).
constexpr long long kGridWaitTicks = 200000000ll;   // 2 s

__device__ inline unsigned int load_dev(const unsigned int *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int TP>
__global__ __launch_bounds__(1024) void k_expand_all(const void *__restrict__ tree,
                                                    const uint2 *__restrict__ kids, uint32_t N,
                                                    const uint2 *seeds, const unsigned int *nseeds,
                                                    uint32_t seed_cap, uint2 *qa, uint2 *qb,
                                                    unsigned int *qcount, uint32_t qcap,
                                                    uint32_t max_levels, Rec *__restrict__ out,
                                                    unsigned long long capacity,
                                                    unsigned long long *counter,
                                                    unsigned int *flags, unsigned int *bar)
{
    __shared__ uint32_t wsum[64];
    __shared__ unsigned int qbase, go;
    __shared__ unsigned long long rbase;
    if (load_dev(flags) & 7u)   // handed over before the launch: the same in every workgroup
        return;
    const uint2 *in = seeds;
    const unsigned int *n_in = nseeds;
    uint32_t in_cap = seed_cap;
    for (uint32_t lev = 0; lev < max_levels; ++lev) {
        uint32_t n = load_dev(n_in);
        n = n < in_cap ? n : in_cap;
        if (n == 0) {
            if (blockIdx.x == 0 && threadIdx.x == 0)
                atomicOr(flags, 8u);
            return;
        }
        uint2 *outq = (lev & 1) ? qb : qa;
        expand_level<TP, true>(tree, kids, N, in, n, outq, qcount + lev + 1, qcap, out,
                               capacity, counter, flags, wsum, qbase, rbase);
        // every wave's queue stores and count updates have completed (each
        // is coherent by itself) before its workgroup arrives
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0) {
            __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned int target = (lev + 1) * gridDim.x;
            const long long start = wall_clock64();
            unsigned int ok = 1;
            while (load_dev(bar) < target) {
                if ((load_dev(flags) & 7u) || wall_clock64() - start > kGridWaitTicks) {
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            if (!ok)
                atomicOr(flags, 4u);
            go = ok;
        }
        __syncthreads();
        if (!go)
            return;
        in = outq;
        n_in = qcount + lev + 1;
        in_cap = qcap;
    }
    // levels exhausted with pairs left: the walk finishes the query
    if (blockIdx.x == 0 && threadIdx.x == 0 && load_dev(n_in) != 0)
        atomicOr(flags, 4u);
}

// Workgroups of k_expand_all<TP> (1 024 lanes) the device holds at once.
static uint32_t resident_expand_all(int precision)
{
    static uint32_t cached[2] = {0, 0};
    const int t = precision == CD_FP64 ? 0 : 1;
    if (cached[t])
        return cached[t];
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    hipError_t e = precision == CD_FP64
                       ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                             &per_cu, reinterpret_cast<const void *>(&k_expand_all<CD_FP64>),
                             1024, 0)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                             &per_cu, reinterpret_cast<const void *>(&k_expand_all<CD_FP32>),
                             1024, 0);
    if (e != hipSuccess || per_cu <= 0 || cus <= 0)
        return 0;
    cached[t] = (uint32_t)(per_cu * cus);
    return cached[t];
}

hipError_t launch_expand_all(const void *tree, const uint2 *kids, int precision, uint32_t N,
                             const uint2 *seeds, const unsigned int *nseeds, uint32_t seed_cap,
                             uint2 *qa, uint2 *qb, unsigned int *qcount, uint32_t qcap,
                             uint32_t max_levels, Rec *out, unsigned long long capacity,
                             unsigned long long *counter, unsigned int *flags, unsigned int *bar,
                             uint32_t blocks, hipStream_t s)
{
    if (N <= 1)
        return hipSuccess;
    uint32_t res = resident_expand_all(precision);
    if (res == 0)
        return hipErrorInvalidDeviceFunction;
    uint32_t g = blocks < res ? blocks : res;
    g = g ? g : 1;
    if (precision == CD_FP64)
        k_expand_all<CD_FP64><<<g, 1024, 0, s>>>(tree, kids, N, seeds, nseeds, seed_cap, qa, qb,
                                                  qcount, qcap, max_levels, out, capacity,
                                                  counter, flags, bar);
    else
        k_expand_all<CD_FP32><<<g, 1024, 0, s>>>(tree, kids, N, seeds, nseeds, seed_cap, qa, qb,
                                                  qcount, qcap, max_levels, out, capacity,
                                                  counter, flags, bar);
    return hipGetLastError();
}

// ---- device-side control of the query (no host reads) -----------------------------------------

// Before the node-pair levels: a build error or lost seeds hand the whole
// traversal to the per-leaf walk.
__global__ void k_query_begin(const TreeHeader *hdr, unsigned int *qflags)
{
    if (hdr->err || hdr->seed_overflow)
        atomicOr(qflags, 4u);
}

// After the last level: the per-leaf walk runs (from a cleared counter) if
// an overflow, bad-node or handover flag is set (bits 1, 2, 4; bit 8 only
// marks a drained queue) or the last queue is not empty.
__global__ void k_query_decide(const unsigned int *last_count, const unsigned int *qflags,
                               unsigned long long *counter, unsigned int *walk)
{
    unsigned int w = ((*qflags & 7u) != 0 || *last_count != 0) ? 1u : 0u;
    if (w)
        *counter = 0ull;
    *walk = w;
}

// Slots [min(count, cap), cap) get a record that sorts after every real one
// and is the same in every slot, so the sort and the repeat removal can run
// over a fixed number of slots.
__global__ void k_pad_records(Rec *raw, const unsigned long long *counter, uint32_t cap)
{
    uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long c = *counter;
    if (r >= cap || (unsigned long long)r < c)
        return;
    Rec pad;
    pad.i = pad.j = pad.tlo = pad.thi = 0xFFFFFFFFu;
    raw[r] = pad;
}

// Result words: count (records written, or records found when they exceed the
// capacity) and status bits (1 capacity exceeded, 2 tree inconsistent).
__global__ void k_query_finish(const unsigned long long *counter, const unsigned int *tree_err,
                               const uint32_t *uniq, uint32_t cap, unsigned long long *count_out,
                               unsigned int *status_out)
{
    unsigned long long c = *counter;
    unsigned int st = 0;
    if (c > cap)
        st |= 1u;
    if (*tree_err)
        st |= 2u;
    unsigned long long n = 0;
    if (c > cap)
        n = c;
    else if (c > 0)
        n = (unsigned long long)*uniq - (c < cap ? 1ull : 0ull);
    *count_out = n;
    *status_out = st;
}

// The record count and the tree's error word side by side, for one read.
__global__ void k_query_status(const unsigned long long *counter, const unsigned int *tree_err,
                               unsigned int *out)
{
    unsigned long long c = *counter;
    out[0] = (unsigned int)c;
    out[1] = (unsigned int)(c >> 32);
    out[2] = *tree_err;
}

hipError_t launch_query_status(const unsigned long long *counter, const unsigned int *tree_err,
                               unsigned int *out, hipStream_t s)
{
    k_query_status<<<1, 1, 0, s>>>(counter, tree_err, out);
    return hipGetLastError();
}

hipError_t launch_query_begin(const TreeHeader *hdr, unsigned int *qflags, hipStream_t s)
{
    k_query_begin<<<1, 1, 0, s>>>(hdr, qflags);
    return hipGetLastError();
}

hipError_t launch_query_decide(const unsigned int *last_count, const unsigned int *qflags,
                               unsigned long long *counter, unsigned int *walk, hipStream_t s)
{
    k_query_decide<<<1, 1, 0, s>>>(last_count, qflags, counter, walk);
    return hipGetLastError();
}

hipError_t launch_pad_records(Rec *raw, const unsigned long long *counter, uint32_t cap,
                              hipStream_t s)
{
    if (cap == 0)
        return hipSuccess;
    k_pad_records<<<nblk(cap, 256), 256, 0, s>>>(raw, counter, cap);
    return hipGetLastError();
}

hipError_t launch_query_finish(const unsigned long long *counter, const unsigned int *tree_err,
                               const uint32_t *uniq, uint32_t cap, unsigned long long *count_out,
                               unsigned int *status_out, hipStream_t s)
{
    k_query_finish<<<1, 1, 0, s>>>(counter, tree_err, uniq, cap, count_out, status_out);
    return hipGetLastError();
}

// Small lists (count <= kSmallCanon) in one workgroup: a stable LSD radix
// sort on the full (i, j, t_lo, t_hi) order, then repeat flags, one block
// scan and the scatter.  The order and the count equal the radix path's; one
// launch instead of a pass triple per digit.
__device__ inline bool rec_less(const Rec &a, const Rec &b)
{
    if (a.i != b.i)
        return a.i < b.i;
    if (a.j != b.j)
        return a.j < b.j;
    if (a.tlo != b.tlo)
        return a.tlo < b.tlo;
    return a.thi < b.thi;
}

__device__ inline bool rec_eq(const Rec &a, const Rec &b)
{
    return a.i == b.i && a.j == b.j && a.tlo == b.tlo && a.thi == b.thi;
}

constexpr int kRecPer = kSmallCanon / 1024;   // records per lane of a 1 024-lane workgroup

struct RecSortLds {
    Rec xch[kSmallCanon];
    uint32_t cnt[16 * 257];   // per (wave, digit), rows of 257 words
    uint32_t wsum[33];
    unsigned int fmax[4];     // largest value of each field
};

__device__ inline uint32_t rec_field(const Rec &r, uint32_t f)
{
    return f == 0 ? r.thi : f == 1 ? r.tlo : f == 2 ? r.j : r.i;
}

// Stable LSD radix sort of the m <= kSmallCanon records a 1 024-lane
// workgroup holds kRecPer per lane (item q of lane `lane` in wave w at place
// w * 64 * kRecPer + q * 64 + lane).  Fields from the least significant
// (t_hi) to the most (i), 8-bit digits, each field only over the bits its
// largest value in this list uses.  A digit's rank: the lanes holding it
// found by ballots, a per-(wave, digit) counter, a digit-major scan of the
// counters.  On return the sorted records are S.xch[0 .. m).
__device__ inline void lds_radix_rec(Rec (&x)[kRecPer], uint32_t m, RecSortLds &S)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t p0 = (uint32_t)w * 64 * kRecPer + lane;
    const uint64_t lt = lanemask_lt();
    if (threadIdx.x < 4)
        S.fmax[threadIdx.x] = 0;
    __syncthreads();
    {
        uint32_t mx[4] = {0, 0, 0, 0};
#pragma unroll
        for (int q = 0; q < kRecPer; ++q)
            if (p0 + q * 64 < m)
                for (uint32_t f = 0; f < 4; ++f)
                    mx[f] = max(mx[f], rec_field(x[q], f));
        for (uint32_t f = 0; f < 4; ++f) {
            for (int o = 32; o >= 1; o >>= 1)
                mx[f] = max(mx[f], (uint32_t)__shfl_xor(mx[f], o, 64));
            if (lane == 0)
                atomicMax(&S.fmax[f], mx[f]);
        }
    }
    __syncthreads();
    bool moved = false;   // S.xch holds the current order
    for (uint32_t f = 0; f < 4; ++f) {
        const uint32_t fm = S.fmax[f];
        for (uint32_t shift = 0; shift < 32 && (fm >> shift) != 0; shift += 8) {
            for (int k = threadIdx.x; k < 16 * 257; k += blockDim.x)
                S.cnt[k] = 0;
            __syncthreads();
            uint32_t rk[kRecPer], dg[kRecPer];
#pragma unroll
            for (int q = 0; q < kRecPer; ++q) {
                const bool valid = p0 + q * 64 < m;
                const uint32_t d = valid ? (rec_field(x[q], f) >> shift) & 0xFFu : 0u;
                const uint64_t peers = match_digit(d, __ballot(valid));
                const uint32_t c = valid ? S.cnt[w * 257 + d] : 0u;
                const uint32_t mine = (uint32_t)__popcll(peers & lt);
                if (valid && mine == 0)
                    S.cnt[w * 257 + d] = c + (uint32_t)__popcll(peers);
                rk[q] = c + mine;
                dg[q] = d;
            }
            __syncthreads();
            {   // exclusive scan of the 4 096 counters in (digit, wave) order
                uint32_t v[4], sum = 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const uint32_t o = threadIdx.x * 4 + k;
                    v[k] = S.cnt[(o % 16) * 257 + o / 16];
                    sum += v[k];
                }
                uint32_t total;
                uint32_t run = block_exclusive_scan(sum, S.wsum, &total);
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const uint32_t o = threadIdx.x * 4 + k;
                    S.cnt[(o % 16) * 257 + o / 16] = run;
                    run += v[k];
                }
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < kRecPer; ++q)
                if (p0 + q * 64 < m)
                    S.xch[S.cnt[w * 257 + dg[q]] + rk[q]] = x[q];
            __syncthreads();
#pragma unroll
            for (int q = 0; q < kRecPer; ++q)
                if (p0 + q * 64 < m)
                    x[q] = S.xch[p0 + q * 64];
            moved = true;
            __syncthreads();
        }
    }
    if (!moved) {   // a single distinct record (or none): already in order
#pragma unroll
        for (int q = 0; q < kRecPer; ++q)
            if (p0 + q * 64 < m)
                S.xch[p0 + q * 64] = x[q];
        __syncthreads();
    }
}

// Records [0, count) of `in` into the lanes, kRecPer per lane.
__device__ inline void load_lanes(Rec (&x)[kRecPer], const Rec *__restrict__ in, uint32_t count)
{
    const uint32_t p0 = (threadIdx.x >> 6) * 64 * kRecPer + (threadIdx.x & 63);
#pragma unroll
    for (int q = 0; q < kRecPer; ++q)
        if (p0 + q * 64 < count)
            x[q] = in[p0 + q * 64];
}

// The canonical list of count <= kSmallCanon records; returns the number
// written (every thread).
__device__ inline uint32_t small_canon(const Rec *__restrict__ in, uint32_t count,
                                       Rec *__restrict__ out, RecSortLds &S)
{
    Rec x[kRecPer];
    load_lanes(x, in, count);
    lds_radix_rec(x, count, S);
    // repeats dropped: each thread owns up to kRecPer consecutive records
    const Rec *r = S.xch;
    uint32_t k0 = threadIdx.x * kRecPer;
    uint32_t f[kRecPer], mine = 0;
    for (int q = 0; q < kRecPer; ++q) {
        uint32_t k = k0 + q;
        f[q] = (k < count && (k == 0 || !rec_eq(r[k], r[k - 1]))) ? 1u : 0u;
        mine += f[q];
    }
    uint32_t all;
    uint32_t pos = block_exclusive_scan(mine, S.wsum, &all);
    for (int q = 0; q < kRecPer; ++q)
        if (f[q])
            out[pos++] = r[k0 + q];
    return all;
}

__global__ __launch_bounds__(1024) void k_small_canon(const Rec *__restrict__ in,
                                                      uint32_t count, Rec *__restrict__ out,
                                                      uint32_t *total)
{
    __shared__ RecSortLds S;
    const uint32_t all = small_canon(in, count, out, S);
    if (threadIdx.x == 0)
        *total = all;
}

// The same, enqueued before the host knows the count: it runs only when the
// node-pair levels drained their queue (flag 8, no other flag), the tree has
// no error bits and the record count fits both the small path and the
// capacity; *done = records written + 1 then, else it stays 0.
__global__ __launch_bounds__(1024) void k_small_canon_gated(const Rec *__restrict__ in,
                                                            const unsigned long long *counter,
                                                            const unsigned int *qflags,
                                                            const unsigned int *tree_err,
                                                            uint32_t limit, Rec *__restrict__ out,
                                                            unsigned int *done)
{
    __shared__ RecSortLds S;
    const unsigned long long c = *counter;
    if (*qflags != 8u || *tree_err != 0u || c > (unsigned long long)limit)
        return;
    const uint32_t all = c ? small_canon(in, (uint32_t)c, out, S) : 0u;
    if (threadIdx.x == 0)
        *done = all + 1;
}

// Medium lists: each workgroup sorts one kSmallCanon-record tile in LDS ...
__global__ __launch_bounds__(1024) void k_tile_sort(const Rec *__restrict__ in, uint32_t bound,
                                                    Rec *__restrict__ out, DevCount g)
{
    __shared__ RecSortLds S;
    uint32_t count;
    if (!g.get(bound, count))
        return;
    uint32_t base = blockIdx.x * (uint32_t)kSmallCanon;
    if (base >= count)
        return;
    uint32_t m = count - base < (uint32_t)kSmallCanon ? count - base : (uint32_t)kSmallCanon;
    Rec x[kRecPer];
    load_lanes(x, in + base, m);
    lds_radix_rec(x, m, S);
    for (uint32_t k = threadIdx.x; k < m; k += blockDim.x)
        out[base + k] = S.xch[k];
}

// ... then sorted runs of `width` records are merged pairwise: output k finds
// by binary search how many of its predecessors come from the left run (the
// stable merge path: on equal records the left run goes first).
__global__ __launch_bounds__(256) void k_merge_runs(const Rec *__restrict__ in, uint32_t bound,
                                                    uint32_t width, Rec *__restrict__ out,
                                                    DevCount g)
{
    uint32_t count;
    if (!g.get(bound, count))
        return;
    uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count)
        return;
    uint64_t q0 = (uint64_t)(k / (2ull * width)) * 2ull * width;
    uint32_t la = (uint32_t)(count - q0 < width ? count - q0 : width);
    uint64_t b0 = q0 + la;
    uint32_t lb = (uint32_t)(count - b0 < width ? count - b0 : width);
    if (b0 >= count)
        lb = 0;
    const Rec *A = in + q0, *B = in + b0;
    uint32_t kk = (uint32_t)(k - q0);   // rank inside the merged pair
    uint32_t lo = kk > lb ? kk - lb : 0u, hi = kk < la ? kk : la;
    // smallest i in [lo, hi] with not (A[i] <= B[kk - i - 1])
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (!rec_less(B[kk - mid - 1], A[mid]))
            lo = mid + 1;
        else
            hi = mid;
    }
    uint32_t i = lo, j = kk - lo;
    bool take_a = i < la && (j >= lb || !rec_less(B[j], A[i]));
    out[k] = take_a ? A[i] : B[j];
}

hipError_t launch_small_canon(const Rec *in, uint32_t count, Rec *out, uint32_t *total,
                              hipStream_t s)
{
    if (count == 0 || count > (uint32_t)kSmallCanon)
        return hipErrorInvalidValue;
    k_small_canon<<<1, 1024, 0, s>>>(in, count, out, total);
    return hipGetLastError();
}

hipError_t launch_small_canon_gated(const Rec *in, const unsigned long long *counter,
                                    const unsigned int *qflags, const unsigned int *tree_err,
                                    uint32_t capacity, Rec *out, unsigned int *done,
                                    hipStream_t s)
{
    const uint32_t limit = capacity < (uint32_t)kSmallCanon ? capacity : (uint32_t)kSmallCanon;
    k_small_canon_gated<<<1, 1024, 0, s>>>(in, counter, qflags, tree_err, limit, out, done);
    return hipGetLastError();
}

hipError_t launch_medium_canon(Rec *a, Rec *b, uint32_t count, uint32_t *flags, uint32_t *pos,
                               void *scan_ws, Rec *out, hipStream_t s, const DevCount &g,
                               unsigned int *total, uint32_t bias)
{
    if (count <= (uint32_t)kSmallCanon || count > (uint32_t)kMediumCanon ||
        (g.counter && (!total || g.hi != count || !g.qflags || !g.tree_err)))
        return hipErrorInvalidValue;
    uint32_t tiles = (count + kSmallCanon - 1) / kSmallCanon;
    k_tile_sort<<<tiles, 1024, 0, s>>>(a, count, b, g);
    hipError_t e = hipGetLastError();
    Rec *src = b, *dst = a;
    // passes for the bound; with a smaller device count the last ones copy
    for (uint32_t w = kSmallCanon; e == hipSuccess && w < count; w *= 2) {
        k_merge_runs<<<nblk(count, 256), 256, 0, s>>>(src, count, w, dst, g);
        e = hipGetLastError();
        Rec *t = src;
        src = dst;
        dst = t;
    }
    if (e != hipSuccess)
        return e;
    return launch_unique(src, count, flags, pos, scan_ws, out, s, g, total, bias);
}

// ---- canonical list: sorted records, repeats dropped -----------------------------------------

__global__ void k_unique_flags(const Rec *in, uint32_t bound, uint32_t *flags, DevCount g)
{
    uint32_t count;
    if (!g.get(bound, count))
        return;
    uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= bound)
        return;
    if (r >= count) {   // past a device count: nothing to keep
        flags[r] = 0u;
        return;
    }
    bool f = true;
    if (r > 0) {
        Rec a = in[r - 1], b = in[r];
        f = a.i != b.i || a.j != b.j || a.tlo != b.tlo || a.thi != b.thi;
    }
    flags[r] = f ? 1u : 0u;
}

__global__ void k_unique_scatter(const Rec *in, uint32_t bound, const uint32_t *flags,
                                 const uint32_t *pos, Rec *out, uint32_t *total, uint32_t bias,
                                 DevCount g)
{
    uint32_t count;
    if (!g.get(bound, count))
        return;
    uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= count)
        return;
    if (flags[r])
        out[pos[r]] = in[r];
    if (r == count - 1)
        *total = pos[r] + flags[r] + bias;
}

hipError_t launch_unique(const Rec *in, uint32_t count, uint32_t *flags, uint32_t *pos,
                         void *scan_ws, Rec *out, hipStream_t s, const DevCount &g,
                         unsigned int *total, uint32_t bias)
{
    // total is written to pos[count] (pos holds count + 1 entries), or with a
    // device count to *total
    if (count == 0)
        return launch_fill_u32(pos, 0u, 1, s);
    k_unique_flags<<<nblk(count, 256), 256, 0, s>>>(in, count, flags, g);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = scan_exclusive_u32(flags, pos, count, scan_ws, s);
    if (e != hipSuccess)
        return e;
    k_unique_scatter<<<nblk(count, 256), 256, 0, s>>>(in, count, flags, pos, out,
                                                      g.counter ? total : pos + count, bias, g);
    return hipGetLastError();
}

#ifdef CD_COUNTERS
hipError_t counters_reset(uint32_t *visits, uint32_t nobj, hipStream_t s)
{
    static const unsigned long long zero[kCounterWords] = {};
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess)
        e = hipMemcpyToSymbol(HIP_SYMBOL(g_ctr), zero, sizeof zero, 0, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpyToSymbol(HIP_SYMBOL(g_visits), &visits, sizeof visits, 0,
                              hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpyToSymbol(HIP_SYMBOL(g_nobj), &nobj, sizeof nobj, 0, hipMemcpyHostToDevice);
    return e;
}

hipError_t counters_read(unsigned long long *out, hipStream_t s)
{
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess)
        e = hipMemcpyFromSymbol(out, HIP_SYMBOL(g_ctr), kCounterWords * sizeof(unsigned long long),
                                0, hipMemcpyDeviceToHost);
    return e;
}
#endif

} // namespace cd
