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

// ---- bottom-up construction of the same tree -----------------------------------
//
// A node covering leaves [f, l] is the left child of its parent when keys l
// and l+1 share a longer prefix than keys f-1 and f (the parent is [f, l'],
// split after leaf l), else the right child (parent [f', l], split after
// f-1); with positions breaking equal keys the two prefixes always differ.
// Its id in the numbering above: leaf N-1+f when f == l, else l for a left
// child and f for a right child (the root, [0, N-1], is 0).

// Common prefix of keys a (at position i) and b (at j), equal keys broken by
// position: clz of the 64-bit XOR, or 96 + clz of the 32-bit position XOR
// (i != j); written as selects, without branches.
__host__ __device__ inline int key_prefix(uint64_t a, uint64_t b, uint32_t i, uint32_t j)
{
    uint64_t x = a ^ b;
    uint32_t h = (uint32_t)(x >> 32), l = (uint32_t)x, p = i ^ j;
    int ch = h ? __builtin_clz(h) : 0, cl = l ? __builtin_clz(l) : 0;
    int cp = p ? __builtin_clz(p) : 0;
    return h ? ch : (l ? 32 + cl : 96 + cp);
}

// key(j) = (j / ms) << 32 | code[j]: time slabs of ms leaves above 32-bit codes.
struct CodeKeys {
    const uint32_t *code;
    uint32_t ms, N;
    __host__ __device__ uint64_t key(uint32_t j) const
    {
        return ((uint64_t)(j / ms) << 32) | code[j];
    }
    __host__ __device__ int delta(uint32_t i, uint32_t j) const
    {
        return j >= N ? -1 : key_prefix(key(i), key(j), i, j);
    }
};

// The same keys for the positions lo, lo + 1, ... held in a window sk (lo may
// wrap below 0: such positions are outside [0, N) and never read).
struct WindowKeys {
    const uint64_t *sk;
    uint32_t lo, N;
    __host__ __device__ int delta(uint32_t i, uint32_t j) const
    {
        return j >= N ? -1 : key_prefix(sk[i - lo], sk[j - lo], i, j);
    }
};

// Adjacent prefixes a(j) = delta(j, j+1), -1 at j = N-1 and below 0, held
// as a(j) + 1 in one byte each (at most 128) for the positions lo, lo + 1, ...
// A node's parent side, its sibling's shape and the skip links need only these.
struct AdjBytes {
    const uint8_t *d;
    uint32_t lo, N;
    __host__ __device__ int at(uint32_t j) const { return j >= N - 1 ? -1 : (int)d[j - lo] - 1; }
};

// karras_escape from adjacent prefixes: node s = r + 1 extends right when
// a(s) >= a(s - 1).
template <class A>
__host__ __device__ inline uint32_t escape_adj(const A &a, uint32_t N, uint32_t r)
{
    if (r >= N - 1)
        return kEnd;
    uint32_t s = r + 1;
    if (s <= N - 2 && a.at(s) >= a.at(s - 1))
        return s;
    return N - 1 + s;
}

// Children of the inner node [f, l] split after leaf g.
__host__ __device__ inline uint2 agglo_children(uint32_t N, uint32_t f, uint32_t l, uint32_t g)
{
    return make_uint2(f == g ? N - 1 + g : g, l == g + 1 ? N - 1 + g + 1 : g + 1);
}

// Where node [f, l] (not the root) meets its sibling, from dl = a(f - 1) and
// dr = a(l).
struct AggloStep {
    bool right;      // a left child: the parent extends right
    int prefix;      // key bits the parent's leaves share
    uint32_t id;     // the node's own id
    uint32_t split;  // the parent's split: after leaf l (right) or f - 1
};
__host__ __device__ inline AggloStep agglo_step(int dl, int dr, uint32_t N, uint32_t f,
                                                uint32_t l)
{
    AggloStep st;
    st.right = dr > dl;
    st.prefix = st.right ? dr : dl;
    st.id = f == l ? N - 1 + f : (st.right ? l : f);
    st.split = st.right ? l : f - 1;
    return st;
}

// Whether the sibling is the single leaf next to the node (l + 1 or f - 1):
// it is when that leaf's own parent is this node's parent.  Otherwise the
// sibling is the inner node numbered by that same position (a right child is
// numbered by its first leaf, a left child by its last).
template <class A>
__host__ __device__ inline bool agglo_sibling_is_leaf(const A &a, const AggloStep &st,
                                                      uint32_t f, uint32_t l)
{
    return st.right ? st.prefix > a.at(l + 1) : st.prefix > a.at(f - 2);
}

// Does the parent of node [f, l] lie within leaves [b0, b1)?  (The node does.)
template <class V>
__host__ __device__ inline bool agglo_parent_within(const V &k, uint32_t N, const AggloStep &st,
                                                    uint32_t f, uint32_t l, uint64_t b0,
                                                    uint64_t b1)
{
    return st.right ? (b1 >= N || k.delta(l, (uint32_t)b1) < st.prefix)
                    : (b0 == 0 || k.delta(f, (uint32_t)(b0 - 1)) < st.prefix);
}

} // namespace cd
