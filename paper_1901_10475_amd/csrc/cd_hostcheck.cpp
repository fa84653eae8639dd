// cd_hostcheck.cpp -- the LBVH index arithmetic of cd_logic.h run on the CPU.
//
// Pre-flight only: the tests use it to check, without a GPU, that the Karras
// topology is a proper binary tree, that the skip links follow pre-order, and
// that the stackless walk the traversal kernel performs terminates and finds
// the same pairs as the oracle.  It is not a fallback for any library call.
#include <stdint.h>
#include <vector>

#include "cd_logic.h"

using namespace cd;

extern "C" {

// Topology of the tree over N sorted keys: for inner node i, its children,
// leaf range and skip link; for leaf i, its skip link.
int hc_karras(const uint64_t *keys, int64_t N, uint32_t *left, uint32_t *right, int64_t *first,
              int64_t *last, uint32_t *esc_inner, uint32_t *esc_leaf)
{
    if (N < 1)
        return 0;
    KeyArray K{keys};
    for (int64_t i = 0; i + 1 < N; ++i) {
        KarrasNode nd = karras_node(K, N, i);
        left[i] = nd.left;
        right[i] = nd.right;
        first[i] = nd.first;
        last[i] = nd.last;
        esc_inner[i] = karras_escape(K, N, nd.last);
    }
    for (int64_t i = 0; i < N; ++i)
        esc_leaf[i] = karras_escape(K, N, i);
    return 0;
}

// The same topology through the 32-bit views the kernels use: over the 64-bit
// keys (slab_size == 0), or over time-major slabs of slab_size keys whose
// upper 32 bits are the slab index (codes = the low 32 bits).
int hc_karras32(const uint64_t *keys, int64_t N, uint32_t slab_size, uint32_t *left,
                uint32_t *right, int64_t *first, int64_t *last, uint32_t *esc_inner,
                uint32_t *esc_leaf)
{
    if (N < 1 || N >= (int64_t)1 << 31)
        return -1;
    const uint32_t n = (uint32_t)N;
    std::vector<uint32_t> codes;
    if (slab_size) {
        if (n % slab_size)
            return -1;
        codes.resize(n);
        for (uint32_t i = 0; i < n; ++i)
            codes[i] = (uint32_t)keys[i];
    }
    for (uint32_t i = 0; i < n; ++i) {
        uint32_t s = slab_size ? i / slab_size : 0;
        SlabKeys32 V{slab_size ? codes.data() + (size_t)s * slab_size : nullptr,
                     s * slab_size, slab_size, s};
        if (i + 1 < n) {
            KarrasNode nd = slab_size ? karras_node_u32(V, n, i)
                                      : karras_node_u32(KeysFrom32{keys, keys[i]}, n, i);
            left[i] = nd.left;
            right[i] = nd.right;
            first[i] = nd.first;
            last[i] = nd.last;
            esc_inner[i] = slab_size ? slab_escape32(V, n, (uint32_t)nd.last)
                                     : keys_escape32(keys, n, (uint32_t)nd.last);
        }
        esc_leaf[i] = slab_size ? slab_escape32(V, n, i) : keys_escape32(keys, n, i);
    }
    return 0;
}

uint32_t hc_morton30(double x, double y, double z, const double *mn, const double *inv_ext)
{
    return morton30(x, y, z, mn, inv_ext);
}

// The traversal kernel's walk for every leaf, over node arrays in the same
// numbering (inner 0..N-2, leaves N-1..2N-2): lo/hi [2N-1][3], t0/t1 [2N-1],
// link [2N-1] (left child or object id), esc [2N-1].  Writes up to cap records
// (i, j, t_lo, t_hi) and returns the number found, or -1 if a walk exceeded
// 2N + 2 steps.
int64_t hc_traverse(int64_t N, const double *lo, const double *hi, const uint32_t *t0,
                    const uint32_t *t1, const uint32_t *link, const uint32_t *esc,
                    uint32_t slab_ticks, uint32_t *out, int64_t cap)
{
    int64_t count = 0;
    for (int64_t i = 0; i < N; ++i) {
        int64_t q = N - 1 + i;
        uint64_t stop = (uint64_t)t1[q] + slab_ticks - 1;
        uint32_t node = esc[q];
        int64_t steps = 0;
        while (node != kEnd) {
            if (++steps > 2 * N + 2)
                return -1;
            if ((uint64_t)t0[node] >= stop)
                break;
            bool ov = time_overlap(t0[q], t1[q], t0[node], t1[node]) &&
                      space_overlap(lo + 3 * q, hi + 3 * q, lo + 3 * (int64_t)node,
                                    hi + 3 * (int64_t)node);
            bool leaf = node >= N - 1;
            if (ov && leaf && link[node] != link[q]) {
                if (count < cap) {
                    uint32_t a = link[q], b = link[node];
                    out[4 * count + 0] = a < b ? a : b;
                    out[4 * count + 1] = a < b ? b : a;
                    out[4 * count + 2] = t0[q] > t0[node] ? t0[q] : t0[node];
                    out[4 * count + 3] = t1[q] < t1[node] ? t1[q] : t1[node];
                }
                ++count;
            }
            node = (ov && !leaf) ? link[node] : esc[node];
        }
    }
    return count;
}

} // extern "C"
