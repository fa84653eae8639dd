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
                       KV *kv, unsigned int *err, uint64_t *packed, uint32_t ib, uint32_t cb)
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
    m &= (1u << kKeyCodeBits) - 1;   // the key holds a 30-bit code
    if (kv) {
        KV x;
        x.key = ((uint64_t)slab << 32) | m;
        x.val = k;
        x.pad = 0;
        kv[k] = x;
    } else if (packed) {
        packed[k] = ((uint64_t)slab << (cb + ib)) | ((uint64_t)(m >> (kKeyCodeBits - cb)) << ib) |
                    k;
    }
}

hipError_t launch_keys(const BoxView &b, int precision, uint32_t N, uint32_t slab_ticks,
                       uint32_t max_slab, uint32_t slab_size, const unsigned long long *bounds,
                       uint32_t *morton, KV *kv, unsigned int *err, hipStream_t s,
                       uint64_t *packed, uint32_t ib, uint32_t cb)
{
    if (packed && (cb > kKeyCodeBits || cb == 0))
        return hipErrorInvalidValue;
    if (N == 0)
        return hipSuccess;
    if (precision == CD_FP64)
        k_keys<CD_FP64><<<nblk(N, 256), 256, 0, s>>>(b, N, slab_ticks, max_slab, slab_size,
                                                     bounds, morton, kv, err, packed, ib, cb);
    else
        k_keys<CD_FP32><<<nblk(N, 256), 256, 0, s>>>(b, N, slab_ticks, max_slab, slab_size,
                                                     bounds, morton, kv, err, packed, ib, cb);
    return hipGetLastError();
}

// ---- top-down Karras hierarchy + skip links (slabs sorted by the slab build) ----------
//
// Inner node i over time-major slabs of sorted 32-bit codes (key j = slab(j)
// << 32 | code[j]).  Outputs: kids[i] = {left, right}; links[i] = {left
// child, skip link}; clev[i] = refit level of node i (the smallest k whose
// level-k blocks of refit_block(k) leaves contain its whole leaf range);
// parent[child] = i, with kCross set when clev[i] > 0.  One workgroup per
// slab holds the slab's codes in LDS and computes every inner node whose
// index lies in the slab (node i's searches always compare key i, a key of
// the slab, so the slab-bits-only view of other slabs is exact); the binary
// searches then wait on LDS instead of L2.  Leaf skip links come from the
// slab build.
__global__ __launch_bounds__(kSegThreads) void k_karras_slabs(const uint32_t *__restrict__ codes,
                                                              uint32_t N, uint32_t slab_size,
                                                              uint2 *kids, LinkSink links,
                                                              uint32_t *parent, uint8_t *clev)
{
    __shared__ uint32_t sk[kSegCap];
    uint64_t slab = blockIdx.x;
    uint64_t base = slab * slab_size;
    uint32_t m = (uint32_t)(base + slab_size <= N ? slab_size : N - base);
    for (uint32_t k = threadIdx.x; k < m; k += blockDim.x)
        sk[k] = codes[base + k];
    __syncthreads();
    const SlabKeys32 K32{sk, (uint32_t)base, slab_size, (uint32_t)slab};
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

__global__ void k_single_leaf(LinkSink links, uint32_t *parent)
{
    links.put(0, 0, kEnd);
    parent[0] = kEnd;
}

hipError_t launch_karras_slabs(const uint32_t *codes, uint32_t N, uint32_t slab_size, uint2 *kids,
                               const LinkSink &links, uint32_t *parent, uint8_t *clev,
                               hipStream_t s)
{
    if (N == 0)
        return hipSuccess;
    if (N == 1) {   // the root is the leaf
        k_single_leaf<<<1, 1, 0, s>>>(links, parent);
        return hipGetLastError();
    }
    if (slab_size == 0 || (int64_t)slab_size > kSegCap)
        return hipErrorInvalidValue;
    uint32_t nslabs = (uint32_t)((N + slab_size - 1) / slab_size);
    k_karras_slabs<<<nslabs, kSegThreads, 0, s>>>(codes, N, slab_size, kids, links, parent, clev);
    return hipGetLastError();
}

} // namespace cd
