// cd_logic.h -- index arithmetic of the LBVH, usable on the device and on the
// host.  The kernels call these functions; a host build of the same header
// (cd_hostcheck.hip) runs them on the CPU so that termination and tree
// invariants can be checked before any GPU run.
//
// Node numbering: internal nodes 0 .. N-2, leaves N-1 .. 2N-2 (leaf i is the
// i-th box in sorted key order).  The root is internal node 0 (leaf 0 when
// N == 1).  kEnd marks "no node".
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cd {

constexpr uint32_t kEnd = 0xFFFFFFFFu;

// ---- Morton codes -----------------------------------------------------------

// Spread the low 10 bits of v so that bit k moves to bit 3k.
__host__ __device__ inline uint32_t spread3_10(uint32_t v)
{
    v &= 0x3FFu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

// 30-bit Morton code of a point quantised to a 1024^3 grid over [mn, mx].
__host__ __device__ inline uint32_t morton30(double x, double y, double z, const double mn[3],
                                             const double inv_ext[3])
{
    double c[3] = {x, y, z};
    uint32_t q[3];
    for (int d = 0; d < 3; ++d) {
        double u = (c[d] - mn[d]) * inv_ext[d];
        u = u < 0.0 ? 0.0 : (u > 1.0 ? 1.0 : u);
        uint32_t v = (uint32_t)(u * 1023.0 + 0.5);
        q[d] = v > 1023u ? 1023u : v;
    }
    return (spread3_10(q[0]) << 2) | (spread3_10(q[1]) << 1) | spread3_10(q[2]);
}

// ---- Karras hierarchy over sorted keys ----------------------------------------------
//
// Keys are read through an accessor K (K(i) = key of sorted leaf i), so the
// same code runs over a key array in memory or over keys held in LDS.
// delta(i, j): length of the common prefix of keys i and j, with the index
// appended as a tie-break so that equal keys still give a strict order;
// -1 outside [0, N).

struct KeyArray {
    const uint64_t *keys;
    __host__ __device__ uint64_t operator()(int64_t i) const { return keys[i]; }
};

template <class K>
__host__ __device__ inline int karras_delta(const K &key, int64_t N, int64_t i, int64_t j)
{
    if (j < 0 || j >= N)
        return -1;
    uint64_t a = key(i), b = key(j);
    if (a != b)
        return __builtin_clzll(a ^ b);
    uint64_t x = (uint64_t)i ^ (uint64_t)j;
    return 64 + __builtin_clzll(x);
}

// Direction of internal node i: +1 if its leaf range extends right of i.
template <class K>
__host__ __device__ inline int karras_dir(const K &key, int64_t N, int64_t i)
{
    return karras_delta(key, N, i, i + 1) >= karras_delta(key, N, i, i - 1) ? 1 : -1;
}

// Node id of the right sibling of the lowest left-child ancestor of a node
// whose leaf range ends at r: the next node in depth-first pre-order once that
// node's subtree is skipped.  It starts at leaf r + 1 and is a right child, so
// it is internal node r + 1 when that node's range starts at r + 1, and leaf
// r + 1 otherwise.
template <class K>
__host__ __device__ inline uint32_t karras_escape(const K &key, int64_t N, int64_t r)
{
    if (r >= N - 1)
        return kEnd;
    int64_t s = r + 1;
    if (s <= N - 2 && karras_dir(key, N, s) > 0)
        return (uint32_t)s;
    return (uint32_t)(N - 1 + s);
}

struct KarrasNode {
    uint32_t left, right;   // node ids
    int64_t first, last;    // leaf range
};

// Internal node i of the Karras (2012) radix tree: find the range by an
// exponential then a binary search on delta, then the split by a binary
// search.  Requires N >= 2 and 0 <= i <= N - 2.
template <class K>
__host__ __device__ inline KarrasNode karras_node(const K &key, int64_t N, int64_t i)
{
    int d = karras_dir(key, N, i);
    int dmin = karras_delta(key, N, i, i - d);
    int64_t lmax = 2;
    while (karras_delta(key, N, i, i + lmax * d) > dmin)
        lmax *= 2;
    int64_t l = 0;
    for (int64_t t = lmax / 2; t >= 1; t /= 2)
        if (karras_delta(key, N, i, i + (l + t) * d) > dmin)
            l += t;
    int64_t j = i + l * d;
    int dnode = karras_delta(key, N, i, j);
    int64_t s = 0;
    int64_t t = l;
    do {
        t = (t + 1) >> 1;
        if (karras_delta(key, N, i, i + (s + t) * d) > dnode)
            s += t;
    } while (t > 1);
    int64_t gamma = i + s * d + (d < 0 ? -1 : 0);
    KarrasNode nd;
    nd.first = i < j ? i : j;
    nd.last = i < j ? j : i;
    nd.left = (nd.first == gamma) ? (uint32_t)(N - 1 + gamma) : (uint32_t)gamma;
    nd.right = (nd.last == gamma + 1) ? (uint32_t)(N - 1 + gamma + 1) : (uint32_t)(gamma + 1);
    return nd;
}

// ---- 4D box overlap ------------------------------------------------------------

// Time tags [t0, t1) overlap (integer ticks, half-open).
__host__ __device__ inline bool time_overlap(uint32_t a0, uint32_t a1, uint32_t b0, uint32_t b1)
{
    return a0 < b1 && b0 < a1;
}

// Closed extents overlap on all three axes.
template <typename F>
__host__ __device__ inline bool space_overlap(const F *alo, const F *ahi, const F *blo,
                                              const F *bhi)
{
    return alo[0] <= bhi[0] && blo[0] <= ahi[0] && alo[1] <= bhi[1] && blo[1] <= ahi[1] &&
           alo[2] <= bhi[2] && blo[2] <= ahi[2];
}

// ---- 32-bit views for the Karras passes ----------------------------------------

// Keys of a Karras hierarchy over time-major slabs of m leaves, key(g) =
// slab(g) << 32 | code(g), seen from one slab whose 32-bit codes are in LDS.
// Every comparison involves a key of that slab (the node's own position i),
// so it is exact without the other slabs' codes: two keys of the slab share
// their slab bits, so their common prefix is 32 plus that of their codes
// (equal keys: 64 plus that of the 64-bit positions, 96 + clz of the 32-bit
// XOR), and a key of another slab differs from key(i) in its slab bits, j / m.
// 32-bit arithmetic throughout: a probe below 0 wraps to at least N (N < 2^31).
struct SlabKeys32 {
    const uint32_t *lds;
    uint32_t base, m, slab;
    __host__ __device__ int delta(uint32_t N, uint32_t i, uint32_t j) const
    {
        if (j >= N)
            return -1;
        uint32_t uj = j - base;
        if (uj < m) {
            uint32_t a = lds[i - base], b = lds[uj];
            return a != b ? 32 + __builtin_clz(a ^ b) : 96 + __builtin_clz(i ^ j);
        }
        return __builtin_clz(slab ^ (j / m));
    }
};

// 64-bit sorted keys seen from node i (its key loaded once), in 32-bit
// position arithmetic; equal keys compare positions (96 + clz of the 32-bit
// XOR, i.e. 64 + clz of the 64-bit one).
struct KeysFrom32 {
    const uint64_t *keys;
    uint64_t ki;
    __host__ __device__ int delta(uint32_t N, uint32_t i, uint32_t j) const
    {
        if (j >= N)
            return -1;
        uint64_t b = keys[j];
        return ki != b ? __builtin_clzll(ki ^ b) : 96 + __builtin_clz(i ^ j);
    }
};

// Karras (2012) node i over a view V (V::delta(N, i, j), -1 outside [0, N)),
// in 32-bit arithmetic: a probe below 0 wraps to at least N (N < 2^31), and
// every probe i + offset stays below 2^32.  Same node as karras_node.
template <class V>
__host__ __device__ inline KarrasNode karras_node_u32(const V &k, uint32_t N, uint32_t i)
{
    int d = k.delta(N, i, i + 1) >= k.delta(N, i, i - 1) ? 1 : -1;
    auto at = [&](uint32_t off) { return d > 0 ? i + off : i - off; };
    int dmin = k.delta(N, i, d > 0 ? i - 1 : i + 1);   // delta to i - d
    uint32_t lmax = 2;
    while (k.delta(N, i, at(lmax)) > dmin)
        lmax *= 2;
    uint32_t l = 0;
    for (uint32_t t = lmax / 2; t >= 1; t /= 2)
        if (k.delta(N, i, at(l + t)) > dmin)
            l += t;
    uint32_t j = at(l);
    int dnode = k.delta(N, i, j);
    uint32_t s = 0, t = l;
    do {
        t = (t + 1) >> 1;
        if (k.delta(N, i, at(s + t)) > dnode)
            s += t;
    } while (t > 1);
    int gamma = (int)i + (int)s * d + (d < 0 ? -1 : 0);
    KarrasNode nd;
    nd.first = i < j ? i : j;
    nd.last = i < j ? j : i;
    nd.left = (nd.first == gamma) ? (uint32_t)(N - 1 + gamma) : (uint32_t)gamma;
    nd.right = (nd.last == gamma + 1) ? (uint32_t)(N - 1 + gamma + 1) : (uint32_t)(gamma + 1);
    return nd;
}

// karras_escape over 64-bit sorted keys in 32-bit position arithmetic
__host__ __device__ inline uint32_t keys_escape32(const uint64_t *keys, uint32_t N, uint32_t r)
{
    if (r >= N - 1)
        return kEnd;
    uint32_t s = r + 1;
    if (s <= N - 2) {
        KeysFrom32 k{keys, keys[s]};
        if (k.delta(N, s, s + 1) >= k.delta(N, s, s - 1))
            return s;
    }
    return N - 1 + s;
}

// karras_escape over the 32-bit slab view, for a leaf range ending at r that
// ends in this slab or at the end of a later one: the next node starts at
// s = r + 1, and when s starts another slab its direction follows from slab
// bits alone (with two or more keys per slab it extends right).
__host__ __device__ inline uint32_t slab_escape32(const SlabKeys32 &k, uint32_t N, uint32_t r)
{
    if (r >= N - 1)
        return kEnd;
    uint32_t s = r + 1;
    if (s > N - 2)
        return N - 1 + s;
    bool right;
    if (s - k.base < k.m)
        right = k.delta(N, s, s + 1) >= k.delta(N, s, s - 1);
    else if (k.m >= 2)
        right = true;
    else   // one key per slab: s - 1, s and s + 1 are slabs s - 1, s and s + 1
        right = __builtin_clz(s ^ (s + 1)) >= __builtin_clz(s ^ (s - 1));
    return right ? s : N - 1 + s;
}

} // namespace cd
