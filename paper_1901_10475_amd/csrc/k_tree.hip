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
// sample of about 2^20 boxes is enough.
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
    uint32_t stride = N > (1u << 20) ? N >> 20 : 1u;
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
    for (int d = 0; d < 3; ++d) {
        mn[d] = from_ordered_bits(bounds[d]);
        double ext = from_ordered_bits(bounds[3 + d]) - mn[d];
        inv[d] = ext > 0.0 ? 1.0 / ext : 0.0;
    }
    double lo[3], hi[3];
    load_box<PREC>(b, k, lo, hi);
    uint32_t m = morton30(0.5 * (lo[0] + hi[0]), 0.5 * (lo[1] + hi[1]), 0.5 * (lo[2] + hi[2]),
                          mn, inv);
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
// Thread i builds inner node i.  Outputs, all compact: links[id] = {left child
// (inner) or 0 (leaf), skip link} for every node id, and parent[child] = i with
// bit 31 set when node i's leaf range crosses a refit chunk boundary (the
// first refit phase stops below such nodes).

constexpr uint32_t kCrossBit = 0x80000000u;

__global__ void k_karras(const uint64_t *__restrict__ keys, uint32_t N, Link *links,
                         uint32_t *parent)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i + 1 >= N)
        return;
    KarrasNode nd = karras_node(keys, N, i);
    bool cross = (nd.first / kRefitLeaves) != (nd.last / kRefitLeaves);
    uint32_t pv = i | (cross ? kCrossBit : 0u);
    parent[nd.left] = pv;
    parent[nd.right] = pv;
    if (i == 0)
        parent[0] = kEnd;
    Link li;
    li.link = nd.left;
    li.esc = karras_escape(keys, N, nd.last);
    links[i] = li;
    Link lf;
    lf.link = 0;
    lf.esc = karras_escape(keys, N, i);
    links[N - 1 + i] = lf;
    if (i == N - 2) {
        Link ll;
        ll.link = 0;
        ll.esc = kEnd;
        links[2 * N - 2] = ll;
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

hipError_t launch_karras(const uint64_t *keys, uint32_t N, Link *links, uint32_t *parent,
                         hipStream_t s)
{
    if (N == 0)
        return hipSuccess;
    if (N == 1) {
        k_single_leaf<<<1, 1, 0, s>>>(links, parent);
        return hipGetLastError();
    }
    k_karras<<<nblk(N - 1, 256), 256, 0, s>>>(keys, N, links, parent);
    return hipGetLastError();
}

// ---- bottom-up refit ---------------------------------------------------------------------
//
// Every inner box is the exact union of its children.  MI355X's eight XCDs keep
// separate L2 caches, and agent-scope release/acquire (needed when two threads
// of different workgroups meet at a node) writes back and invalidates L2; done
// at every node it costs two orders of magnitude.  The refit therefore runs in
// two phases:
//   1. one workgroup per chunk of kRefitLeaves consecutive leaves writes the
//      leaf records and climbs; arrival counters live in LDS and ordering is
//      workgroup-scope.  The first thread to reach a node stops, the second
//      writes the union.  A climb also stops below a node whose leaf range
//      crosses a chunk boundary and records where it stopped.
//   2. one workgroup climbs from those stopping points through the remaining
//      top of the tree (at most depth x chunks nodes), again workgroup-scope.
// Kernel boundaries order phase 1's writes before phase 2's reads.

template <int TP>
struct NodeIO;

template <>
struct NodeIO<CD_FP64> {
    __device__ static void put(void *tree, uint32_t N, uint32_t id, const double lo[3],
                               const double hi[3], uint32_t t0, uint32_t t1, uint32_t link,
                               uint32_t esc)
    {
        Node64 n;
        for (int d = 0; d < 3; ++d) {
            n.lo[d] = lo[d];
            n.hi[d] = hi[d];
        }
        n.t0 = t0;
        n.t1 = t1;
        n.link = link;
        n.esc = esc;
        ((Node64 *)tree)[id] = n;
    }
    __device__ static void get_box(const void *tree, uint32_t N, uint32_t id, double lo[3],
                                   double hi[3], uint32_t &t0, uint32_t &t1)
    {
        const Node64 *n = (const Node64 *)tree + id;
        for (int d = 0; d < 3; ++d) {
            lo[d] = n->lo[d];
            hi[d] = n->hi[d];
        }
        t0 = n->t0;
        t1 = n->t1;
    }
};

template <>
struct NodeIO<CD_FP32> {
    // outward rounding; inner unions of floats are exact in float
    __device__ static void put(void *tree, uint32_t N, uint32_t id, const double lo[3],
                               const double hi[3], uint32_t t0, uint32_t t1, uint32_t link,
                               uint32_t esc)
    {
        Box32 b;
        for (int d = 0; d < 3; ++d) {
            b.lo[d] = __double2float_rd(lo[d]);
            b.hi[d] = __double2float_ru(hi[d]);
        }
        b.t0 = t0;
        b.t1 = t1;
        ((Box32 *)tree)[id] = b;
        Link l;
        l.link = link;
        l.esc = esc;
        ((Link *)((Box32 *)tree + (2 * (size_t)N - 1)))[id] = l;
    }
    __device__ static void get_box(const void *tree, uint32_t N, uint32_t id, double lo[3],
                                   double hi[3], uint32_t &t0, uint32_t &t1)
    {
        const Box32 *n = (const Box32 *)tree + id;
        for (int d = 0; d < 3; ++d) {
            lo[d] = n->lo[d];
            hi[d] = n->hi[d];
        }
        t0 = n->t0;
        t1 = n->t1;
    }
};

// Union of the box in (lo, hi, t0, t1) with the box of node `other`; writes
// node p.  Returns false on an inconsistent link.
template <int TP>
__device__ inline bool unite_into(void *tree, const Link *links, uint32_t N, uint32_t node,
                                  uint32_t p, double lo[3], double hi[3], uint32_t &t0,
                                  uint32_t &t1)
{
    Link lp = links[p];
    uint32_t l = lp.link;
    if (l >= 2 * N - 1)
        return false;
    uint32_t r = links[l].esc;
    uint32_t other = (l == node) ? r : l;
    if (other >= 2 * N - 1 || (l != node && r != node))
        return false;
    double olo[3], ohi[3];
    uint32_t ot0, ot1;
    NodeIO<TP>::get_box(tree, N, other, olo, ohi, ot0, ot1);
    for (int d = 0; d < 3; ++d) {
        lo[d] = fmin(lo[d], olo[d]);
        hi[d] = fmax(hi[d], ohi[d]);
    }
    t0 = t0 < ot0 ? t0 : ot0;
    t1 = t1 > ot1 ? t1 : ot1;
    NodeIO<TP>::put(tree, N, p, lo, hi, t0, t1, l, lp.esc);
    return true;
}

template <int BP, int TP>
__global__ __launch_bounds__(kRefitThreads) void k_refit_chunks(
    BoxView b, uint32_t N, const uint32_t *__restrict__ idx, const uint32_t *__restrict__ parent,
    const Link *__restrict__ links, void *tree, uint32_t *starts, uint32_t starts_cap,
    unsigned int *nstarts, unsigned int *err)
{
    __shared__ unsigned int cnt[kRefitLeaves];
    uint32_t c0 = blockIdx.x * (uint32_t)kRefitLeaves;
    uint32_t c1 = c0 + kRefitLeaves < N ? c0 + kRefitLeaves : N;
    for (uint32_t k = threadIdx.x; k < (uint32_t)kRefitLeaves; k += kRefitThreads)
        cnt[k] = 0;
    __syncthreads();
    for (uint32_t i = c0 + threadIdx.x; i < c1; i += kRefitThreads) {
        uint32_t src = idx[i];
        if (src >= N) {
            atomicOr(err, 2u);
            continue;
        }
        double lo[3], hi[3];
        load_box<BP>(b, src, lo, hi);
        if (TP == CD_FP32 && BP == CD_FP64) {
            // the union below must see the rounded leaf, as the traversal does
            for (int d = 0; d < 3; ++d) {
                lo[d] = __double2float_rd(lo[d]);
                hi[d] = __double2float_ru(hi[d]);
            }
        }
        uint32_t t0 = b.t0[src], t1 = b.t1[src];
        uint32_t node = N - 1 + i;
        NodeIO<TP>::put(tree, N, node, lo, hi, t0, t1, b.obj[src], links[node].esc);
        for (int guard = 0; guard < 160; ++guard) {
            uint32_t pv = parent[node];
            if (pv == kEnd)
                break;
            uint32_t p = pv & ~kCrossBit;
            if (p >= N - 1) {
                atomicOr(err, 2u);
                break;
            }
            if (pv & kCrossBit) {
                unsigned int at = atomicAdd(nstarts, 1u);
                if (at < starts_cap)
                    starts[at] = node;
                else
                    atomicOr(err, 8u);
                break;
            }
            if (p < c0 || p >= c1) {
                atomicOr(err, 2u);
                break;
            }
            unsigned int old = __hip_atomic_fetch_add(&cnt[p - c0], 1u, __ATOMIC_ACQ_REL,
                                                      __HIP_MEMORY_SCOPE_WORKGROUP);
            if (old == 0)
                break;
            if (!unite_into<TP>(tree, links, N, node, p, lo, hi, t0, t1)) {
                atomicOr(err, 2u);
                break;
            }
            node = p;
        }
    }
}

template <int TP>
__global__ __launch_bounds__(kRefitThreads) void k_refit_top(
    uint32_t N, const uint32_t *__restrict__ parent, const Link *__restrict__ links, void *tree,
    unsigned int *arrive, const uint32_t *starts, const unsigned int *nstarts, uint32_t starts_cap,
    unsigned int *err)
{
    uint32_t ns = *nstarts;
    ns = ns < starts_cap ? ns : starts_cap;
    for (uint32_t s = threadIdx.x; s < ns; s += kRefitThreads) {
        uint32_t node = starts[s];
        if (node >= 2 * N - 1) {
            atomicOr(err, 2u);
            continue;
        }
        double lo[3], hi[3];
        uint32_t t0, t1;
        NodeIO<TP>::get_box(tree, N, node, lo, hi, t0, t1);
        for (int guard = 0; guard < 160; ++guard) {
            uint32_t pv = parent[node];
            if (pv == kEnd)
                break;
            uint32_t p = pv & ~kCrossBit;
            if (p >= N - 1) {
                atomicOr(err, 2u);
                break;
            }
            unsigned int old = __hip_atomic_fetch_add(&arrive[p], 1u, __ATOMIC_ACQ_REL,
                                                      __HIP_MEMORY_SCOPE_WORKGROUP);
            if (old == 0)
                break;
            if (!unite_into<TP>(tree, links, N, node, p, lo, hi, t0, t1)) {
                atomicOr(err, 2u);
                break;
            }
            node = p;
        }
    }
}

size_t refit_starts_cap(uint32_t N)
{
    size_t chunks = ((size_t)N + kRefitLeaves - 1) / kRefitLeaves;
    return 2 * 160 * chunks + 64;
}

hipError_t launch_refit(const BoxView &b, int box_precision, int tree_precision, uint32_t N,
                        const uint32_t *idx, const uint32_t *parent, const Link *links,
                        unsigned int *arrive, uint32_t *starts, unsigned int *nstarts,
                        void *tree, unsigned int *err, hipStream_t s)
{
    if (N == 0)
        return hipSuccess;
    hipError_t e = launch_fill_u32(arrive, 0u, N > 1 ? N - 1 : 1, s);
    if (e == hipSuccess)
        e = launch_fill_u32(nstarts, 0u, 1, s);
    if (e != hipSuccess)
        return e;
    uint32_t cap = (uint32_t)refit_starts_cap(N);
    unsigned g = nblk(N, kRefitLeaves);
    if (box_precision == CD_FP64 && tree_precision == CD_FP64)
        k_refit_chunks<CD_FP64, CD_FP64><<<g, kRefitThreads, 0, s>>>(b, N, idx, parent, links,
                                                                      tree, starts, cap, nstarts,
                                                                      err);
    else if (box_precision == CD_FP64)
        k_refit_chunks<CD_FP64, CD_FP32><<<g, kRefitThreads, 0, s>>>(b, N, idx, parent, links,
                                                                      tree, starts, cap, nstarts,
                                                                      err);
    else
        k_refit_chunks<CD_FP32, CD_FP32><<<g, kRefitThreads, 0, s>>>(b, N, idx, parent, links,
                                                                      tree, starts, cap, nstarts,
                                                                      err);
    e = hipGetLastError();
    if (e != hipSuccess || N <= (uint32_t)kRefitLeaves)
        return e;
    if (tree_precision == CD_FP64)
        k_refit_top<CD_FP64><<<1, kRefitThreads, 0, s>>>(N, parent, links, tree, arrive, starts,
                                                         nstarts, cap, err);
    else
        k_refit_top<CD_FP32><<<1, kRefitThreads, 0, s>>>(N, parent, links, tree, arrive, starts,
                                                         nstarts, cap, err);
    return hipGetLastError();
}

} // namespace cd
