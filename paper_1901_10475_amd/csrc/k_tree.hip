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

template <int PREC>
__device__ inline void load_box(const BoxView &b, uint32_t k, double lo[3], double hi[3])
{
    for (int d = 0; d < 3; ++d) {
        if (PREC == CD_FP64) {
            lo[d] = ((const double *)b.lo[d])[k];
            hi[d] = ((const double *)b.hi[d])[k];
        } else {
            lo[d] = ((const float *)b.lo[d])[k];
            hi[d] = ((const float *)b.hi[d])[k];
        }
    }
}

// ---- scene bounds of the box centres -------------------------------------------------

template <int PREC>
__global__ __launch_bounds__(256) void k_bounds(BoxView b, uint32_t N, unsigned long long *bounds)
{
    __shared__ unsigned long long red[6][4];
    unsigned long long mn[3] = {~0ull, ~0ull, ~0ull}, mx[3] = {0ull, 0ull, 0ull};
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < N; k += gridDim.x * blockDim.x) {
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
    unsigned g = nblk(N, 256);
    g = g > 2048 ? 2048 : g;
    if (precision == CD_FP64)
        k_bounds<CD_FP64><<<g, 256, 0, s>>>(b, N, bounds);
    else
        k_bounds<CD_FP32><<<g, 256, 0, s>>>(b, N, bounds);
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

// ---- Karras hierarchy + escape links ------------------------------------------------------

__device__ inline void set_link(void *tree, int precision, uint32_t N, uint32_t id,
                                uint32_t link, uint32_t esc, bool write_link)
{
    if (precision == CD_FP64) {
        Node64 *n = (Node64 *)tree;
        if (write_link)
            n[id].link = link;
        n[id].esc = esc;
    } else {
        Link *L = (Link *)((Box32 *)tree + (2 * (size_t)N - 1));
        if (write_link)
            L[id].link = link;
        L[id].esc = esc;
    }
}

__global__ void k_karras(const uint64_t *__restrict__ keys, uint32_t N, int precision,
                         void *tree, uint32_t *parent)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i + 1 >= N)
        return;
    KarrasNode nd = karras_node(keys, N, i);
    parent[nd.left] = i;
    parent[nd.right] = i;
    if (i == 0)
        parent[0] = kEnd;
    // inner node i: left child and the skip link past its subtree
    set_link(tree, precision, N, i, nd.left, karras_escape(keys, N, nd.last), true);
    // leaf i's skip link; the last leaf has none
    set_link(tree, precision, N, N - 1 + i, 0, karras_escape(keys, N, i), false);
    if (i == N - 2)
        set_link(tree, precision, N, 2 * N - 2, 0, kEnd, false);
}

__global__ void k_single_leaf(void *tree, int precision, uint32_t *parent)
{
    set_link(tree, precision, 1, 0, 0, kEnd, false);
    parent[0] = kEnd;
}

hipError_t launch_karras(const uint64_t *keys, uint32_t N, int precision, void *tree,
                         uint32_t *parent, hipStream_t s)
{
    if (N == 0)
        return hipSuccess;
    if (N == 1) {
        k_single_leaf<<<1, 1, 0, s>>>(tree, precision, parent);
        return hipGetLastError();
    }
    k_karras<<<nblk(N - 1, 256), 256, 0, s>>>(keys, N, precision, tree, parent);
    return hipGetLastError();
}

// ---- bottom-up refit ---------------------------------------------------------------------
//
// Thread i writes leaf i (box idx[i], rounded outward when the tree is FP32 and
// the boxes FP64) and climbs.  At each parent it bumps an arrival counter with
// agent-scope acquire-release ordering: the first thread stops, the second
// (which then sees its sibling's box) writes the union.  The 8 XCDs of MI355X
// keep separate L2 caches, so the agent scope is what makes a box written on
// one XCD visible to a thread on another.

template <int TP>
struct NodeIO;

template <>
struct NodeIO<CD_FP64> {
    __device__ static void put_box(void *tree, uint32_t N, uint32_t id, const double lo[3],
                                   const double hi[3], uint32_t t0, uint32_t t1)
    {
        Node64 *n = (Node64 *)tree + id;
        for (int d = 0; d < 3; ++d) {
            n->lo[d] = lo[d];
            n->hi[d] = hi[d];
        }
        n->t0 = t0;
        n->t1 = t1;
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
    __device__ static uint32_t link(const void *tree, uint32_t N, uint32_t id)
    {
        return ((const Node64 *)tree)[id].link;
    }
    __device__ static uint32_t esc(const void *tree, uint32_t N, uint32_t id)
    {
        return ((const Node64 *)tree)[id].esc;
    }
    __device__ static void set_obj(void *tree, uint32_t N, uint32_t id, uint32_t obj)
    {
        ((Node64 *)tree)[id].link = obj;
    }
};

template <>
struct NodeIO<CD_FP32> {
    __device__ static Link *links(const void *tree, uint32_t N)
    {
        return (Link *)((Box32 *)tree + (2 * (size_t)N - 1));
    }
    // inner unions of outward-rounded floats are exact in float
    __device__ static void put_box(void *tree, uint32_t N, uint32_t id, const double lo[3],
                                   const double hi[3], uint32_t t0, uint32_t t1)
    {
        Box32 *n = (Box32 *)tree + id;
        for (int d = 0; d < 3; ++d) {
            n->lo[d] = __double2float_rd(lo[d]);
            n->hi[d] = __double2float_ru(hi[d]);
        }
        n->t0 = t0;
        n->t1 = t1;
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
    __device__ static uint32_t link(const void *tree, uint32_t N, uint32_t id)
    {
        return links(tree, N)[id].link;
    }
    __device__ static uint32_t esc(const void *tree, uint32_t N, uint32_t id)
    {
        return links(tree, N)[id].esc;
    }
    __device__ static void set_obj(void *tree, uint32_t N, uint32_t id, uint32_t obj)
    {
        links(tree, N)[id].link = obj;
    }
};

template <int BP, int TP>
__global__ void k_refit(BoxView b, uint32_t N, const uint32_t *__restrict__ idx,
                        const uint32_t *__restrict__ parent, unsigned int *arrive, void *tree,
                        unsigned int *err)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N)
        return;
    uint32_t src = idx[i];
    if (src >= N) {
        atomicOr(err, 2u);
        return;
    }
    double lo[3], hi[3];
    load_box<BP>(b, src, lo, hi);
    uint32_t node = N - 1 + i;
    NodeIO<TP>::put_box(tree, N, node, lo, hi, b.t0[src], b.t1[src]);
    NodeIO<TP>::set_obj(tree, N, node, b.obj[src]);
    // depth of a Karras tree is bounded by key bits + index bits
    for (int guard = 0; guard < 160; ++guard) {
        uint32_t p = parent[node];
        if (p == kEnd)
            return;
        if (p >= N - 1) {
            atomicOr(err, 2u);
            return;
        }
        unsigned int old = __hip_atomic_fetch_add(&arrive[p], 1u, __ATOMIC_ACQ_REL,
                                                  __HIP_MEMORY_SCOPE_AGENT);
        if (old == 0)
            return;
        uint32_t l = NodeIO<TP>::link(tree, N, p);
        uint32_t r = NodeIO<TP>::esc(tree, N, l);
        if (l >= 2 * N - 1 || r >= 2 * N - 1) {
            atomicOr(err, 2u);
            return;
        }
        double llo[3], lhi[3], rlo[3], rhi[3];
        uint32_t lt0, lt1, rt0, rt1;
        NodeIO<TP>::get_box(tree, N, l, llo, lhi, lt0, lt1);
        NodeIO<TP>::get_box(tree, N, r, rlo, rhi, rt0, rt1);
        for (int d = 0; d < 3; ++d) {
            lo[d] = fmin(llo[d], rlo[d]);
            hi[d] = fmax(lhi[d], rhi[d]);
        }
        NodeIO<TP>::put_box(tree, N, p, lo, hi, lt0 < rt0 ? lt0 : rt0, lt1 > rt1 ? lt1 : rt1);
        node = p;
    }
    atomicOr(err, 2u);
}

hipError_t launch_refit(const BoxView &b, int box_precision, int tree_precision, uint32_t N,
                        const uint32_t *idx, const uint32_t *parent, unsigned int *arrive,
                        void *tree, unsigned int *err, hipStream_t s)
{
    if (N == 0)
        return hipSuccess;
    hipError_t e = launch_fill_u32(arrive, 0u, N > 1 ? N - 1 : 1, s);
    if (e != hipSuccess)
        return e;
    unsigned g = nblk(N, 256);
    if (box_precision == CD_FP64 && tree_precision == CD_FP64)
        k_refit<CD_FP64, CD_FP64><<<g, 256, 0, s>>>(b, N, idx, parent, arrive, tree, err);
    else if (box_precision == CD_FP64)
        k_refit<CD_FP64, CD_FP32><<<g, 256, 0, s>>>(b, N, idx, parent, arrive, tree, err);
    else
        k_refit<CD_FP32, CD_FP32><<<g, 256, 0, s>>>(b, N, idx, parent, arrive, tree, err);
    return hipGetLastError();
}

} // namespace cd
