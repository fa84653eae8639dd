// k_sort.hip -- fills, device-wide exclusive scan, stable LSD radix sorts.
//
// Two radix sorts live here:
//   * radix_sort16 / radix_sort8: device-wide, stable, over 16-byte items
//     (key/value pairs or pair records) or 8-byte ones (a key and its box
//     index packed in one word), 8-bit digits, one histogram + scan + scatter
//     per digit.  They sort tree keys when boxes are not grouped in slabs and
//     put pair records in canonical order.
//   * k_slab_build: one 1024-thread workgroup per time slab; keys stay in
//     registers and move through LDS between digit passes, so a slab of up to
//     kSegCap boxes is sorted with one read and one write of global memory.
// Both rank digits stably with the same wave-level scheme: the lanes holding
// equal digits are found with eight ballots, the lowest of them bumps a
// per-(digit, wave) counter in LDS, and a digit-major scan of those counters
// turns per-wave ranks into positions.
#include "cd_internal.h"

namespace cd {

static inline unsigned nblk(uint64_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

// ---- fills ---------------------------------------------------------------------

__global__ void k_fill_u32(uint32_t *p, uint32_t v, size_t count)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < count; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_u64(unsigned long long *p, unsigned long long v, size_t count)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < count; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, size_t count, hipStream_t s)
{
    if (count == 0)
        return hipSuccess;
    unsigned g = nblk(count, 256);
    k_fill_u32<<<g > 4096 ? 4096 : g, 256, 0, s>>>(p, v, count);
    return hipGetLastError();
}
hipError_t launch_fill_u64(unsigned long long *p, unsigned long long v, size_t count,
                           hipStream_t s)
{
    if (count == 0)
        return hipSuccess;
    unsigned g = nblk(count, 256);
    k_fill_u64<<<g > 4096 ? 4096 : g, 256, 0, s>>>(p, v, count);
    return hipGetLastError();
}

// ---- device-wide exclusive scan of uint32 ---------------------------------------

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(const uint32_t *in, uint32_t *out,
                                                             size_t count, uint32_t *tile_sums)
{
    __shared__ uint32_t tile[kScanTile];
    __shared__ uint32_t wsum[64];
    size_t base = (size_t)blockIdx.x * kScanTile;
    for (int k = 0; k < kScanItems; ++k) {
        size_t g = base + (size_t)k * kScanThreads + threadIdx.x;
        tile[k * kScanThreads + threadIdx.x] = g < count ? in[g] : 0u;
    }
    __syncthreads();
    uint32_t v[kScanItems];
    uint32_t sum = 0;
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = tile[threadIdx.x * kScanItems + k];
        sum += v[k];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan(sum, wsum, &total);
    for (int k = 0; k < kScanItems; ++k) {
        uint32_t x = v[k];
        tile[threadIdx.x * kScanItems + k] = run;
        run += x;
    }
    __syncthreads();
    for (int k = 0; k < kScanItems; ++k) {
        size_t g = base + (size_t)k * kScanThreads + threadIdx.x;
        if (g < count)
            out[g] = tile[k * kScanThreads + threadIdx.x];
    }
    if (threadIdx.x == 0 && tile_sums)
        tile_sums[blockIdx.x] = total;
}

__global__ void k_scan_add(uint32_t *out, size_t count, const uint32_t *tile_off)
{
    size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < count)
        out[g] += tile_off[g / kScanTile];
}

size_t scan_ws_bytes(size_t count)
{
    size_t bytes = 0;
    while (count > (size_t)kScanTile) {
        count = (count + kScanTile - 1) / kScanTile;
        bytes += align_up(count * sizeof(uint32_t), 256);
    }
    return bytes + 256;
}

hipError_t scan_exclusive_u32(const uint32_t *in, uint32_t *out, size_t count, void *ws,
                              hipStream_t s)
{
    if (count == 0)
        return hipSuccess;
    size_t tiles = (count + kScanTile - 1) / kScanTile;
    uint32_t *sums = tiles > 1 ? (uint32_t *)ws : nullptr;
    k_scan_tiles<<<(unsigned)tiles, kScanThreads, 0, s>>>(in, out, count, sums);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || tiles == 1)
        return e;
    void *rest = (char *)ws + align_up(tiles * sizeof(uint32_t), 256);
    e = scan_exclusive_u32(sums, sums, tiles, rest, s);
    if (e != hipSuccess)
        return e;
    k_scan_add<<<nblk(count, 256), 256, 0, s>>>(out, count, sums);
    return hipGetLastError();
}

// ---- device-wide LSD radix sort of 16- and 8-byte items -------------------------------

constexpr int kRadThreads = 256;
constexpr int kRadItems = 16;
constexpr int kRadTile = kRadThreads * kRadItems;  // 4096
constexpr int kRadWaves = kRadThreads / 64;

struct DigitKV {
    uint32_t shift;
    __device__ uint32_t operator()(const uint4 &it) const
    {
        uint64_t key = ((uint64_t)it.y << 32) | it.x;
        return (uint32_t)(key >> shift) & 0xFFu;
    }
};
struct DigitRec {
    uint32_t field, shift;
    __device__ uint32_t operator()(const uint4 &it) const
    {
        uint32_t v = field == 0 ? it.x : field == 1 ? it.y : field == 2 ? it.z : it.w;
        return (v >> shift) & 0xFFu;
    }
};
struct DigitU64 {
    uint32_t shift;
    __device__ uint32_t operator()(const uint2 &it) const
    {
        uint64_t v = ((uint64_t)it.y << 32) | it.x;
        return (uint32_t)(v >> shift) & 0xFFu;
    }
};

// Digit counts of one tile.  Lanes count into one of 16 copies of the
// histogram (by lane mod 16, rows of 257 words so that the copies of one
// digit sit in different banks): a tile whose items share a digit (a slab
// digit, say) then contends 4 lanes deep instead of 4 096.
template <typename Item, typename Digit>
__global__ __launch_bounds__(kRadThreads) void k_radix_upsweep(const Item *in, size_t count,
                                                               Digit dig, uint32_t *hist,
                                                               uint32_t nblocks)
{
    constexpr int kCopies = 16;
    __shared__ uint32_t h[kCopies * 257];
    for (int k = threadIdx.x; k < kCopies * 257; k += kRadThreads)
        h[k] = 0;
    __syncthreads();
    size_t base = (size_t)blockIdx.x * kRadTile;
    uint32_t dg[kRadItems];   // every load in flight before the first count
#pragma unroll
    for (int k = 0; k < kRadItems; ++k) {
        size_t g = base + (size_t)k * kRadThreads + threadIdx.x;
        dg[k] = g < count ? dig(in[g]) : 256u;
    }
    uint32_t *mine = h + (threadIdx.x % kCopies) * 257;
#pragma unroll
    for (int k = 0; k < kRadItems; ++k)
        if (dg[k] < 256u)
            atomicAdd(&mine[dg[k]], 1u);
    __syncthreads();
    uint32_t sum = 0;
#pragma unroll
    for (int q = 0; q < kCopies; ++q)
        sum += h[q * 257 + threadIdx.x];
    hist[(size_t)threadIdx.x * nblocks + blockIdx.x] = sum;
}

template <typename Item, typename Digit>
__global__ __launch_bounds__(kRadThreads) void k_radix_downsweep(const Item *in, Item *out,
                                                                 size_t count, Digit dig,
                                                                 const uint32_t *hist_scan,
                                                                 uint32_t nblocks)
{
    // per-(wave, digit) counters, wave-major with a 257-word row: lanes of a
    // wave (same w, random d) and the per-digit prefix (same d, all w) both
    // spread over the banks
    __shared__ uint32_t cnt[kRadWaves * 257];
    __shared__ uint32_t dbase[256];
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int k = threadIdx.x; k < kRadWaves * 257; k += kRadThreads)
        cnt[k] = 0;
    dbase[threadIdx.x] = hist_scan[(size_t)threadIdx.x * nblocks + blockIdx.x];
    __syncthreads();
    size_t wbase = (size_t)blockIdx.x * kRadTile + (size_t)w * (64 * kRadItems);
    Item item[kRadItems];
    uint32_t dg[kRadItems], rk[kRadItems];
    uint64_t lt = lanemask_lt();
#pragma unroll
    for (int j = 0; j < kRadItems; ++j) {   // every load in flight before the ranking
        size_t g = wbase + (size_t)j * 64 + lane;
        item[j] = g < count ? in[g] : Item{};
    }
    for (int j = 0; j < kRadItems; ++j) {
        size_t g = wbase + (size_t)j * 64 + lane;
        bool valid = g < count;
        uint32_t d = valid ? dig(item[j]) : 0u;
        uint64_t act = __ballot(valid);
        uint64_t peers = match_digit(d, act);
        uint32_t c = valid ? cnt[w * 257 + d] : 0u;
        uint32_t mine = (uint32_t)__popcll(peers & lt);
        if (valid && mine == 0)
            cnt[w * 257 + d] = c + (uint32_t)__popcll(peers);
        dg[j] = d;
        rk[j] = c + mine;
    }
    __syncthreads();
    {   // per digit: exclusive prefix over waves
        uint32_t d = threadIdx.x, run = 0;
        for (int ww = 0; ww < kRadWaves; ++ww) {
            uint32_t t = cnt[ww * 257 + d];
            cnt[ww * 257 + d] = run;
            run += t;
        }
    }
    __syncthreads();
    for (int j = 0; j < kRadItems; ++j) {
        size_t g = wbase + (size_t)j * 64 + lane;
        if (g < count) {
            size_t pos = (size_t)dbase[dg[j]] + cnt[w * 257 + dg[j]] + rk[j];
            if (pos < count)
                out[pos] = item[j];
        }
    }
}

size_t radix_ws_bytes(size_t count)
{
    size_t nb = (count + kRadTile - 1) / kRadTile;
    size_t h = nb * 256;
    return align_up(h * sizeof(uint32_t), 256) + scan_ws_bytes(h);
}

hipError_t radix_sort16(SortKind kind, void *a, void *b, size_t count, const DigitPlan &plan,
                        void *ws, void **result, hipStream_t s)
{
    *result = a;
    if (count <= 1 || plan.npass == 0)
        return hipSuccess;
    uint32_t nb = (uint32_t)((count + kRadTile - 1) / kRadTile);
    size_t h = (size_t)nb * 256;
    uint32_t *hist = (uint32_t *)ws;
    void *sws = (char *)ws + align_up(h * sizeof(uint32_t), 256);
    uint4 *src = (uint4 *)a, *dst = (uint4 *)b;
    for (int p = 0; p < plan.npass; ++p) {
        if (kind == SORT_KV) {
            DigitKV dg{plan.shift[p]};
            k_radix_upsweep<<<nb, kRadThreads, 0, s>>>(src, count, dg, hist, nb);
        } else {
            DigitRec dg{plan.field[p], plan.shift[p]};
            k_radix_upsweep<<<nb, kRadThreads, 0, s>>>(src, count, dg, hist, nb);
        }
        hipError_t e = hipGetLastError();
        if (e == hipSuccess)
            e = scan_exclusive_u32(hist, hist, h, sws, s);
        if (e != hipSuccess)
            return e;
        if (kind == SORT_KV) {
            DigitKV dg{plan.shift[p]};
            k_radix_downsweep<<<nb, kRadThreads, 0, s>>>(src, dst, count, dg, hist, nb);
        } else {
            DigitRec dg{plan.field[p], plan.shift[p]};
            k_radix_downsweep<<<nb, kRadThreads, 0, s>>>(src, dst, count, dg, hist, nb);
        }
        e = hipGetLastError();
        if (e != hipSuccess)
            return e;
        uint4 *t = src;
        src = dst;
        dst = t;
    }
    *result = src;
    return hipSuccess;
}

hipError_t radix_sort8(void *a, void *b, size_t count, const DigitPlan &plan, void *ws,
                       void **result, hipStream_t s)
{
    *result = a;
    if (count <= 1 || plan.npass == 0)
        return hipSuccess;
    uint32_t nb = (uint32_t)((count + kRadTile - 1) / kRadTile);
    size_t h = (size_t)nb * 256;
    uint32_t *hist = (uint32_t *)ws;
    void *sws = (char *)ws + align_up(h * sizeof(uint32_t), 256);
    uint2 *src = (uint2 *)a, *dst = (uint2 *)b;
    for (int p = 0; p < plan.npass; ++p) {
        const DigitU64 dg{plan.shift[p]};
        k_radix_upsweep<<<nb, kRadThreads, 0, s>>>(src, count, dg, hist, nb);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess)
            e = scan_exclusive_u32(hist, hist, h, sws, s);
        if (e == hipSuccess) {
            k_radix_downsweep<<<nb, kRadThreads, 0, s>>>(src, dst, count, dg, hist, nb);
            e = hipGetLastError();
        }
        if (e != hipSuccess)
            return e;
        uint2 *t = src;
        src = dst;
        dst = t;
    }
    *result = src;
    return hipSuccess;
}

// ---- per-slab LDS radix sort ---------------------------------------------------------
//
// Block = kSegThreads (16 waves).  Wave w holds the keys with local index
// w * 64 * kSegItems + j * 64 + lane (item j) in registers.  Per 8-bit digit:
// rank inside the wave per item, scan the (digit, wave) counters, scatter the
// keys and then the values through one LDS exchange buffer, read back.

constexpr int kSegWaves = kSegThreads / 64;

// Sorts the m <= kSegCap keys of one workgroup by 32-bit key, stably, in four
// 8-bit digit passes; item j of lane `lane` of wave w is local index
// w * 64 * kSegItems + j * 64 + lane, before and after.  val travels with
// key.  xch: kSegCap words of LDS; cnt: kSegWaves * 257; wsum: 64.
__device__ inline void lds_sort32(uint32_t (&key)[kSegItems], uint32_t (&val)[kSegItems],
                                  uint32_t m, uint32_t *xch, uint32_t *cnt, uint32_t *wsum)
{
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t li0 = (uint32_t)w * 64 * kSegItems + lane;
    uint64_t lt = lanemask_lt();
    for (int shift = 0; shift < 32; shift += 8) {
        for (int k = threadIdx.x; k < kSegWaves * 257; k += kSegThreads)
            cnt[k] = 0;
        __syncthreads();
        uint32_t rk[kSegItems];  // rank inside (digit, wave), then final position
#pragma unroll
        for (int j = 0; j < kSegItems; ++j) {
            uint32_t li = li0 + j * 64;
            bool valid = li < m;
            uint32_t d = (key[j] >> shift) & 0xFFu;
            uint64_t peers = match_digit(d, __ballot(valid));
            uint32_t c = valid ? cnt[w * 257 + d] : 0u;
            uint32_t mine = (uint32_t)__popcll(peers & lt);
            if (valid && mine == 0)
                cnt[w * 257 + d] = c + (uint32_t)__popcll(peers);
            rk[j] = c + mine;
        }
        __syncthreads();
        {   // exclusive scan of the 4096 counters in (digit, wave) order
            uint32_t v[4], sum = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                uint32_t o = threadIdx.x * 4 + q;   // (digit, wave) order
                v[q] = cnt[(o % kSegWaves) * 257 + o / kSegWaves];
                sum += v[q];
            }
            uint32_t total;
            uint32_t run = block_exclusive_scan(sum, wsum, &total);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                uint32_t o = threadIdx.x * 4 + q;
                cnt[(o % kSegWaves) * 257 + o / kSegWaves] = run;
                run += v[q];
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kSegItems; ++j) {
            uint32_t d = (key[j] >> shift) & 0xFFu;
            rk[j] += cnt[w * 257 + d];
        }
        // keys, then values, through the exchange buffer
#pragma unroll
        for (int j = 0; j < kSegItems; ++j)
            if (li0 + j * 64 < m && rk[j] < (uint32_t)kSegCap)
                xch[rk[j]] = key[j];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kSegItems; ++j)
            if (li0 + j * 64 < m)
                key[j] = xch[li0 + j * 64];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kSegItems; ++j)
            if (li0 + j * 64 < m && rk[j] < (uint32_t)kSegCap)
                xch[rk[j]] = val[j];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kSegItems; ++j)
            if (li0 + j * 64 < m)
                val[j] = xch[li0 + j * 64];
        __syncthreads();
    }
}

template <int PREC, int TP, bool CODES>
__global__ __launch_bounds__(kSegThreads) void k_slab_build(
    BoxView b, uint32_t slab_size, uint32_t N, uint32_t slab_ticks,
    const unsigned long long *bounds, uint32_t *__restrict__ codes_out, void *tree,
    unsigned int *err)
{
    __shared__ uint32_t xch[kSegCap];
    // counters of (digit, wave), stored wave-major with a 257-word row (see
    // k_radix_downsweep): index w * 257 + d
    __shared__ uint32_t cnt[kSegWaves * 257];
    __shared__ uint32_t wsum[64];
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint64_t slab = blockIdx.x;
    uint64_t base = slab * slab_size;
    uint32_t m = slab_size;
    if (base + m > N)
        m = base < N ? (uint32_t)(N - base) : 0u;
    double mn[3], inv[3];
    for (int d = 0; d < 3; ++d) {   // the frame is read only when codes are formed here
        mn[d] = inv[d] = 0.0;
        if (!CODES) {
            mn[d] = from_ordered_bits(bounds[d]);
            double ext = from_ordered_bits(bounds[3 + d]) - mn[d];
            inv[d] = ext > 0.0 ? 1.0 / ext : 0.0;
        }
    }
    uint32_t key[kSegItems], val[kSegItems];
    uint32_t li0 = (uint32_t)w * 64 * kSegItems + lane;
    bool bad = false;
#pragma unroll
    for (int j = 0; j < kSegItems; ++j) {
        uint32_t li = li0 + j * 64;
        key[j] = 0xFFFFFFFFu;
        if (li < m) {
            if (CODES) {   // codes written with the boxes: 4 bytes instead of 48
                key[j] = b.code[base + li];
            } else {
                double lo[3], hi[3];
                load_box<PREC>(b, base + li, lo, hi);
                key[j] = morton30(0.5 * (lo[0] + hi[0]), 0.5 * (lo[1] + hi[1]),
                                  0.5 * (lo[2] + hi[2]), mn, inv);
            }
            bad |= (b.t0[base + li] / slab_ticks) != slab;
        }
        val[j] = li;
    }
    if (bad)
        atomicOr(err, 1u);
    lds_sort32(key, val, m, xch, cnt, wsum);
    // Leaf records.  Reading boxes by sorted position would gather 4-8 byte
    // words from all over the slab; instead each box is read in source order
    // (coalesced) and its whole record is written to its sorted slot.  LDS
    // holds the sorted codes (for the skip links) and the inverse permutation.
    __shared__ uint32_t vsrc[kSegCap];  // source box -> sorted position
#pragma unroll
    for (int j = 0; j < kSegItems; ++j) {
        uint32_t p = li0 + j * 64;
        if (p < m) {
            xch[p] = key[j];
            vsrc[val[j]] = p;
            // the sorted 32-bit codes (a slab's key bits above them are its
            // index); streaming stores: lanes write consecutive words
            __builtin_nontemporal_store(key[j], &codes_out[base + p]);
        }
    }
    __syncthreads();
    const SlabKeys32 K{xch, (uint32_t)base, slab_size, (uint32_t)slab};
    // kScatterBatch boxes per lane at a time: their loads are all in flight
    // before the first record is written
    constexpr int kScatterBatch = 4;
#pragma unroll 1
    for (uint32_t l0 = threadIdx.x; l0 < m; l0 += kSegThreads * kScatterBatch) {
        double lo[kScatterBatch][3], hi[kScatterBatch][3];
        uint32_t t0[kScatterBatch], t1[kScatterBatch], ob[kScatterBatch];
#pragma unroll
        for (int q = 0; q < kScatterBatch; ++q) {
            uint32_t li = l0 + q * kSegThreads;
            if (li < m) {
                uint64_t src = base + li;
                load_box<PREC>(b, src, lo[q], hi[q]);
                t0[q] = b.t0[src];
                t1[q] = b.t1[src];
                ob[q] = b.obj[src];
            }
        }
#pragma unroll
        for (int q = 0; q < kScatterBatch; ++q) {
            uint32_t li = l0 + q * kSegThreads;
            if (li < m) {
                uint32_t p = vsrc[li];
                uint32_t esc = slab_escape32(K, N, (uint32_t)(base + p));
                NodeIO<TP>::put(tree, N, (uint32_t)(N - 1 + base + p), lo[q], hi[q], t0[q],
                                t1[q], ob[q], esc);
            }
        }
    }
}


// Per-object Morton order of each block of slabs: block B's unsorted codes
// (code of object i at ucode[i * es]) are sorted with their object ids; rank
// r's code and object go to scode[r * es] and sobj[r * es].  One workgroup
// per block; blocks are `stride` entries (of es words) apart.
// Run r (grid.y) of block b (grid.x): entries [r S, min(n, (r + 1) S)) of
// the block (entry k at (b stride + k) es words) sorted in LDS by code,
// stable, each with its block-local index; written to the same entries of
// scode / sobj.  With one run (S = n) that is the block's whole order.
__global__ __launch_bounds__(kSegThreads) void k_block_sort(const uint32_t *ucode, uint32_t n,
                                                            uint32_t S, uint64_t stride,
                                                            uint32_t es, uint32_t *scode,
                                                            uint32_t *sobj)
{
    __shared__ uint32_t xch[kSegCap];
    __shared__ uint32_t cnt[kSegWaves * 257];
    __shared__ uint32_t wsum[64];
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t r0 = blockIdx.y * S;
    if (r0 >= n)
        return;   // (the whole workgroup)
    const uint32_t m = n - r0 < S ? n - r0 : S;
    uint64_t base = (uint64_t)blockIdx.x * stride + r0;
    uint32_t key[kSegItems], val[kSegItems];
    uint32_t li0 = (uint32_t)w * 64 * kSegItems + lane;
#pragma unroll
    for (int j = 0; j < kSegItems; ++j) {
        uint32_t li = li0 + j * 64;
        key[j] = li < m ? ucode[(base + li) * es] : 0xFFFFFFFFu;
        val[j] = r0 + li;
    }
    lds_sort32(key, val, m, xch, cnt, wsum);
#pragma unroll
    for (int j = 0; j < kSegItems; ++j) {
        uint32_t r = li0 + j * 64;
        if (r < m) {
            scode[(base + r) * es] = key[j];
            sobj[(base + r) * es] = val[j];
        }
    }
}

// The R sorted runs of each block merged: entry e of run r goes to position
// (its index in run r) + (entries of earlier runs with a code <= its code) +
// (entries of later runs with a smaller code), which is its place in the
// block's (code, index) order, as one stable sort of the whole block gives.
__global__ __launch_bounds__(256) void k_block_merge(const uint32_t *rcode, const uint32_t *robj,
                                                     uint32_t n, uint32_t S, uint32_t R,
                                                     uint64_t stride, uint32_t es,
                                                     uint32_t *scode, uint32_t *sobj)
{
    const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n)
        return;
    const uint64_t base = (uint64_t)blockIdx.y * stride;
    const uint32_t r = e / S;
    const uint32_t x = rcode[(base + e) * es], id = robj[(base + e) * es];
    uint32_t rank = e - r * S;
    for (uint32_t q = 0; q < R; ++q) {
        if (q == r)
            continue;
        const uint32_t lo0 = q * S, len = n - lo0 < S ? n - lo0 : S;
        // entries of run q before x: code <= x (q < r) or code < x (q > r)
        uint32_t lo = 0, hi = len;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1, c = rcode[(base + lo0 + mid) * es];
            if (q < r ? c <= x : c < x)
                lo = mid + 1;
            else
                hi = mid;
        }
        rank += lo;
    }
    scode[(base + rank) * es] = x;
    sobj[(base + rank) * es] = id;
}

hipError_t launch_block_sort(const uint32_t *ucode, uint32_t n, uint32_t nblocks, uint64_t stride,
                             uint32_t es, uint32_t *scode, uint32_t *sobj, uint32_t *rcode,
                             uint32_t *robj, hipStream_t s)
{
    if (n == 0 || nblocks == 0)
        return hipSuccess;
    const uint32_t R = (uint32_t)((n + kSegCap - 1) / kSegCap);
    if (R > (uint32_t)kBlockRuns || (R > 1 && (!rcode || !robj)))
        return hipErrorInvalidValue;
    const uint32_t S = (n + R - 1) / R;
    if (R == 1) {
        k_block_sort<<<dim3(nblocks, 1), kSegThreads, 0, s>>>(ucode, n, S, stride, es, scode,
                                                              sobj);
        return hipGetLastError();
    }
    k_block_sort<<<dim3(nblocks, R), kSegThreads, 0, s>>>(ucode, n, S, stride, es, rcode, robj);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    k_block_merge<<<dim3((n + 255) / 256, nblocks), 256, 0, s>>>(rcode, robj, n, S, R, stride, es,
                                                                  scode, sobj);
    return hipGetLastError();
}

hipError_t launch_slab_build(const BoxView &b, int box_precision, int tree_precision,
                             uint32_t nslabs, uint32_t slab_size, uint32_t N,
                             uint32_t slab_ticks, const unsigned long long *bounds,
                             uint32_t *codes_out, void *tree, unsigned int *err,
                             hipStream_t s)
{
    if (nslabs == 0 || N == 0)
        return hipSuccess;
    if ((int64_t)slab_size > kSegCap)
        return hipErrorInvalidValue;
#define CD_SLAB_LAUNCH(P, T, C)                                                             \
    k_slab_build<P, T, C><<<nslabs, kSegThreads, 0, s>>>(b, slab_size, N, slab_ticks, bounds,  \
                                                         codes_out, tree, err)
    const bool codes = b.code != nullptr;
    if (box_precision == CD_FP64 && tree_precision == CD_FP64) {
        if (codes)
            CD_SLAB_LAUNCH(CD_FP64, CD_FP64, true);
        else
            CD_SLAB_LAUNCH(CD_FP64, CD_FP64, false);
    } else if (box_precision == CD_FP64) {
        if (codes)
            CD_SLAB_LAUNCH(CD_FP64, CD_FP32, true);
        else
            CD_SLAB_LAUNCH(CD_FP64, CD_FP32, false);
    } else {
        if (codes)
            CD_SLAB_LAUNCH(CD_FP32, CD_FP32, true);
        else
            CD_SLAB_LAUNCH(CD_FP32, CD_FP32, false);
    }
#undef CD_SLAB_LAUNCH
    return hipGetLastError();
}

} // namespace cd
