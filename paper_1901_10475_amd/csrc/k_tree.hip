// k_tree.hip -- Morton keys and the Karras hierarchy.
//
// The tree is the AABB tree of Sec. 3.2 (leaves hold object boxes, every inner
// box contains the boxes below it) built in bulk over 4D boxes: the time
// dimension enters through the key, whose high bits are the box's time slab
// (t0 / slab_ticks) and whose low 30 bits are the Morton code of its centre.
// Sorting by this key puts each time slab in one contiguous subtree; the
// hierarchy (Karras 2012) is built over the sorted keys with one thread per
// inner node.  The inner boxes are set by the refit (k_refit.hip).
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
                       KV *kv, unsigned int *err, uint64_t *packed, uint32_t ib)
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
    } else if (packed) {
        packed[k] = ((uint64_t)slab << (32 + ib)) | ((uint64_t)m << ib) | k;
    }
}

hipError_t launch_keys(const BoxView &b, int precision, uint32_t N, uint32_t slab_ticks,
                       uint32_t max_slab, uint32_t slab_size, const unsigned long long *bounds,
                       uint32_t *morton, KV *kv, unsigned int *err, hipStream_t s,
                       uint64_t *packed, uint32_t ib)
{
    if (N == 0)
        return hipSuccess;
    if (precision == CD_FP64)
        k_keys<CD_FP64><<<nblk(N, 256), 256, 0, s>>>(b, N, slab_ticks, max_slab, slab_size,
                                                     bounds, morton, kv, err, packed, ib);
    else
        k_keys<CD_FP32><<<nblk(N, 256), 256, 0, s>>>(b, N, slab_ticks, max_slab, slab_size,
                                                     bounds, morton, kv, err, packed, ib);
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

__global__ void k_karras(const uint64_t *__restrict__ keys, uint32_t N, uint2 *kids, LinkSink links,
                         uint32_t *parent, uint8_t *clev, bool leaf_links)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i + 1 >= N)
        return;
    KarrasNode nd = karras_node_u32(KeysFrom32{keys, keys[i]}, N, i);
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
    links.put(i, nd.left, keys_escape32(keys, N, (uint32_t)nd.last));
    if (!leaf_links)
        return;
    links.put(N - 1 + i, 0, keys_escape32(keys, N, i));
    if (i == N - 2)
        links.put(2 * N - 2, 0, kEnd);
}

// Same nodes as k_karras for time-major slabs: one workgroup per slab holds
// the slab's sorted 32-bit codes in LDS and computes every inner node whose
// index lies in the slab (node i's searches always compare key i, a key of the
// slab, so the slab-bits-only view of other slabs is exact).  The binary
// searches then wait on LDS instead of L2.  Leaf skip links come from the
// slab build, or, for boxes that arrive already sorted within their slabs (t0
// given), from here; the codes' order and every box's slab are then checked
// (error bit 1, as the slab build reports a box outside its slab).
__global__ __launch_bounds__(kSegThreads) void k_karras_slabs(const uint32_t *__restrict__ codes,
                                                              uint32_t N, uint32_t slab_size,
                                                              uint2 *kids, LinkSink links,
                                                              uint32_t *parent, uint8_t *clev,
                                                              const uint32_t *__restrict__ t0,
                                                              uint32_t slab_ticks,
                                                              unsigned int *err)
{
    __shared__ uint32_t sk[kSegCap];
    uint64_t slab = blockIdx.x;
    uint64_t base = slab * slab_size;
    uint32_t m = (uint32_t)(base + slab_size <= N ? slab_size : N - base);
    for (uint32_t k = threadIdx.x; k < m; k += blockDim.x)
        sk[k] = codes[base + k];
    __syncthreads();
    const SlabKeys32 K32{sk, (uint32_t)base, slab_size, (uint32_t)slab};
    if (t0) {
        bool bad = false;
        for (uint32_t k = threadIdx.x; k < m; k += blockDim.x) {
            uint32_t i = (uint32_t)(base + k);
            bad |= (k + 1 < m && sk[k] > sk[k + 1]) || t0[i] / slab_ticks != slab;
            links.put(N - 1 + i, 0, slab_escape32(K32, N, i));
        }
        if (bad)
            atomicOr(err, 1u);
    }
    for (uint32_t k = threadIdx.x; k < m; k += blockDim.x) {
        uint32_t i = (uint32_t)(base + k);
        if (i + 1 >= N)
            break;
        KarrasNode nd = karras_node_u32(K32, N, i);
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
        links.put(i, nd.left, slab_escape32(K32, N, (uint32_t)nd.last));
    }
}

// Inner node i of a slab hierarchy, written out: children, refit level,
// parent pointers and skip link.
__device__ inline void put_inner(const SlabKeys32 &K, uint32_t N, uint32_t i,
                                 const KarrasNode &nd, uint2 *kids, const LinkSink &links,
                                 uint32_t *parent, uint8_t *clev)
{
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
    links.put(i, nd.left, slab_escape32(K, N, (uint32_t)nd.last));
}

// Karras over boxes already sorted within their slabs (the sorted layout).
// Slabs of one block of the layout carry the same codes in the same order,
// and when no two codes of a slab are equal, an inner node strictly inside a
// slab (local index 1 .. m-2) is decided by in-slab comparisons alone (every
// probe outside the slab compares below its range's common prefix), so its
// children and range in one slab are those of the group's first slab shifted
// by the slab offset.  Slabs are taken in groups of kKarrasGroup:
// k_group_check marks the groups whose slabs share the first slab's codes
// (with no code repeated), checks every slab's code order and, when tags are
// given, every box's slab (error bit 1); k_karras_parts then runs one
// workgroup per slab, which searches a contiguous 1 / kKarrasGroup share of
// the group's template nodes and writes them for every slab of the group, plus its own slab's two
// end nodes (its subtree root and the node joining it to its neighbours) and
// its leaves' skip links.  A group that fails the check is computed slab by
// slab.
constexpr uint32_t kKarrasGroup = 8;

__global__ __launch_bounds__(kSegThreads) void k_group_check(
    const uint32_t *__restrict__ codes, const uint32_t *__restrict__ t0, uint32_t N, uint32_t m,
    uint32_t slab_ticks, uint8_t *templ, unsigned int *err)
{
    const uint32_t nslabs = N / m;
    const uint32_t s0 = blockIdx.x * kKarrasGroup;
    const uint32_t ns = nslabs - s0 < kKarrasGroup ? nslabs - s0 : kKarrasGroup;
    const size_t base0 = (size_t)s0 * m;
    bool differs = false, dup = false, bad = false;
    for (uint32_t k = threadIdx.x; k < m; k += blockDim.x) {
        uint32_t c0 = codes[base0 + k];
        for (uint32_t q = 0; q < ns; ++q) {
            size_t g = base0 + (size_t)q * m + k;
            uint32_t c = codes[g];
            differs |= c != c0;
            if (k + 1 < m) {
                uint32_t c1 = codes[g + 1];
                bad |= c > c1;
                dup |= q == 0 && c == c1;
            }
            if (t0)   // (otherwise the refit checks the slabs of the leaf records)
                bad |= t0[g] / slab_ticks != s0 + q;
        }
    }
    bool any = __syncthreads_or(differs || dup);
    if (bad)
        atomicOr(err, 1u);
    if (threadIdx.x == 0)
        templ[blockIdx.x] = (!any && m >= 3) ? 1 : 0;
}

__global__ __launch_bounds__(kSegThreads) void k_karras_parts(
    const uint32_t *__restrict__ codes, const uint8_t *__restrict__ templ, uint32_t N,
    uint32_t m, uint2 *kids, LinkSink links, uint32_t *parent, uint8_t *clev)
{
    __shared__ uint32_t sk[kSegCap];
    const uint32_t nslabs = N / m;
    const uint32_t s = blockIdx.x;
    const uint32_t grp = s / kKarrasGroup, part = s % kKarrasGroup;
    const uint32_t s0 = grp * kKarrasGroup;
    const uint32_t ns = nslabs - s0 < kKarrasGroup ? nslabs - s0 : kKarrasGroup;
    const bool tp = templ[grp] != 0;
    const uint32_t base = s * m, base0 = s0 * m;
    // the slab's own codes (the same as the first slab's in a template group)
    for (uint32_t k = threadIdx.x; k < m; k += blockDim.x)
        sk[k] = codes[(size_t)base + k];
    __syncthreads();
    const SlabKeys32 K{sk, base, m, s};
    if (tp) {
        const SlabKeys32 K0{sk, base0, m, s0};
        // template nodes: this part's contiguous share of local indices
        // 1 .. m-2, each written for every slab (contiguous runs per slab)
        const uint32_t inner = m - 2, share = (inner + ns - 1) / ns;
        const uint32_t lo = 1 + (part * share < inner ? part * share : inner);
        const uint32_t hi = 1 + ((part + 1) * share < inner ? (part + 1) * share : inner);
        for (uint32_t l = lo + threadIdx.x; l < hi; l += blockDim.x) {
            KarrasNode nd0 = karras_node_u32(K0, N, base0 + l);
            for (uint32_t q = 0; q < ns; ++q) {
                const uint32_t off = q * m;
                KarrasNode nd = nd0;
                nd.first += off;
                nd.last += off;
                nd.left += off;    // inner ids and leaf ids shift alike
                nd.right += off;
                const SlabKeys32 Kq{sk, base0 + off, m, s0 + q};
                put_inner(Kq, N, base0 + off + l, nd, kids, links, parent, clev);
            }
        }
        // this slab's end nodes
        if (threadIdx.x < 2) {
            const uint32_t i = base + (threadIdx.x ? m - 1 : 0u);
            if (i + 1 < N)
                put_inner(K, N, i, karras_node_u32(K, N, i), kids, links, parent, clev);
        }
    } else {
        for (uint32_t k = threadIdx.x; k < m; k += blockDim.x) {
            const uint32_t i = base + k;
            if (i + 1 < N)
                put_inner(K, N, i, karras_node_u32(K, N, i), kids, links, parent, clev);
        }
    }
    for (uint32_t k = threadIdx.x; k < m; k += blockDim.x)
        links.put(N - 1 + base + k, 0, slab_escape32(K, N, base + k));
}

hipError_t launch_karras_blocks(const uint32_t *codes, const uint32_t *t0, uint32_t N,
                                uint32_t slab_size, uint32_t slab_ticks, uint8_t *templ,
                                uint2 *kids, const LinkSink &links, uint32_t *parent,
                                uint8_t *clev, unsigned int *err, hipStream_t s)
{
    if (N <= 1 || slab_size == 0 || (int64_t)slab_size > kSegCap || N % slab_size ||
        slab_ticks == 0)
        return hipErrorInvalidValue;
    uint32_t nslabs = N / slab_size;
    uint32_t groups = (nslabs + kKarrasGroup - 1) / kKarrasGroup;
    k_group_check<<<groups, kSegThreads, 0, s>>>(codes, t0, N, slab_size, slab_ticks, templ, err);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    k_karras_parts<<<nslabs, kSegThreads, 0, s>>>(codes, templ, N, slab_size, kids, links, parent,
                                                  clev);
    return hipGetLastError();
}

__global__ void k_single_leaf(LinkSink links, uint32_t *parent)
{
    links.put(0, 0, kEnd);
    parent[0] = kEnd;
}

hipError_t launch_karras(const uint64_t *keys, uint32_t N, uint2 *kids, const LinkSink &links,
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

hipError_t launch_karras_slabs(const uint32_t *codes, uint32_t N, uint32_t slab_size, uint2 *kids,
                               const LinkSink &links, uint32_t *parent, uint8_t *clev,
                               const uint32_t *t0, uint32_t slab_ticks, unsigned int *err,
                               hipStream_t s)
{
    if (N <= 1 || slab_size == 0 || (int64_t)slab_size > kSegCap || (t0 && slab_ticks == 0))
        return hipErrorInvalidValue;
    uint32_t nslabs = (uint32_t)((N + slab_size - 1) / slab_size);
    k_karras_slabs<<<nslabs, kSegThreads, 0, s>>>(codes, N, slab_size, kids, links, parent, clev,
                                                  t0, slab_ticks, err);
    return hipGetLastError();
}

} // namespace cd
