// cd_hostcheck.cpp -- the LBVH index arithmetic of cd_logic.h run on the CPU.
//
// Pre-flight only: the tests use it to check, without a GPU, that the Karras
// topology is a proper binary tree, that the skip links follow pre-order, and
// that the stackless walk the traversal kernel performs terminates and finds
// the same pairs as the oracle.  It is not a fallback for any library call.
#include <stdint.h>
#include <algorithm>
#include <random>
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

// The bottom-up build of k_agglo.hip replayed on the CPU: passes over chunks
// of C items (pass 1: the leaves; later passes: the roots each chunk handed
// up, in position order), each chunk's lanes run one after another in a
// shuffled order (every order is one the GPU may take).  Every read of the
// chunk's LDS window is bounds-checked, every meeting is checked to find the
// sibling's box where the kernel reads it (the box slot an item shares with
// the nodes of that id end), and each chunk's hand-ups to stay within the
// kernel's limit.  Writes each inner node's children and skip link and each
// leaf's skip link, as hc_karras32 does.  Returns 0, or a negative code
// naming the first violated check.
namespace {
struct CheckedAdj {
    const uint8_t *d;
    uint32_t lo, N, len;
    int *fault;
    int at(uint32_t j) const
    {
        if (j >= N - 1)
            return -1;
        if (j - lo >= len) {
            *fault = 1;
            return -1;
        }
        return (int)d[j - lo] - 1;
    }
};
struct HcItem {
    uint32_t f, l, id;
    int af, al;   // adjacent prefixes after the first and after the last leaf
};
}  // namespace

int hc_agglo(const uint32_t *codes, int64_t N64, uint32_t ms, uint32_t C, uint64_t seed,
             uint32_t *left, uint32_t *right, uint32_t *esc_inner, uint32_t *esc_leaf)
{
    if (N64 < 1 || N64 >= ((int64_t)1 << 31) || ms == 0 || C < 4 || C > 1024 || (C & (C - 1)))
        return -1;
    const uint32_t N = (uint32_t)N64, kOut = 256;
    const CodeKeys G{codes, ms, N};
    std::mt19937_64 rng(seed);
    std::vector<uint8_t> formed(N, 0);
    std::vector<HcItem> items(N);
    for (uint32_t j = 0; j < N; ++j) {
        int a = j + 1 < N ? G.delta(j, j + 1) : -1;
        items[j] = HcItem{j, j, N - 1 + j, a, a};
    }
    int fault = 0;
    for (int pass = 0; !items.empty(); ++pass) {
        const uint32_t M = (uint32_t)items.size();
        std::vector<HcItem> next;
        for (uint32_t C0 = 0; C0 < M; C0 += C) {
            const uint32_t m = std::min(M - C0, C), wlo = C0 - 2;
            std::vector<uint8_t> sa(m + 3, 0);
            for (uint32_t k = 0; k < m + 3; ++k)
                if (wlo + k < M)
                    sa[k] = (uint8_t)(items[wlo + k].al + 1);
            const CheckedAdj A{sa.data(), wlo, M, m + 3, &fault};
            auto in_chunk = [&](uint32_t K, uint32_t lim) {
                if (K - C0 >= lim)
                    fault = 1;
                return K - C0 < lim ? K : C0;
            };
            auto first = [&](uint32_t K) { return items[in_chunk(K, m)].f; };
            auto last = [&](uint32_t K) { return items[in_chunk(K, m)].l; };
            auto item_id = [&](uint32_t K) { return items[in_chunk(K, m)].id; };
            auto a_first = [&](uint32_t K) { return items[in_chunk(K, m + 1)].af; };
            if (pass == 0)
                for (uint32_t K = C0; K < C0 + m; ++K)
                    esc_leaf[K] = escape_adj(A, N, K);
            // items partition the leaves in order (each starts one leaf after
            // the previous one ends) and carry their Karras number: the leaf's
            // own for an item of one leaf, else the last leaf for a left child
            // (prefix after the last leaf above the one before the first) and
            // the first for a right child
            if (pass > 0)
                for (uint32_t K = C0; K < C0 + m; ++K) {
                    const uint32_t f = K == 0 ? 0u : items[K - 1].l + 1;
                    const uint32_t l = items[K].l;
                    const uint32_t id = f == l ? N - 1 + f : (A.at(K) > A.at(K - 1) ? l : f);
                    if (items[K].f != f)
                        return -13;
                    if (items[K].id != id)
                        return -14;
                }
            // slot k: the node whose box it holds, its other end, end
            // prefixes and split (kEnd: still the item itself)
            std::vector<uint32_t> slot_node(m), other(m), spl(m, kEnd), cnt(m, 0);
            std::vector<int> sdl(m), sdr(m);
            for (uint32_t k = 0; k < m; ++k) {
                slot_node[k] = items[C0 + k].id;
                other[k] = C0 + k;
                sdl[k] = A.at(C0 + k - 1);
                sdr[k] = A.at(C0 + k);
            }
            std::vector<HcItem> roots;
            auto hand_up = [&](uint32_t F, uint32_t L, uint32_t id, int dr) {
                roots.push_back(HcItem{first(F), last(L), id, a_first(F), dr});
            };
            // rounds: every lane climbs at most kSteps merges, then parks its
            // node in its slot; the next round resumes the parked ones
            const int kSteps = 3;
            std::vector<uint32_t> lanes(m), parked;
            for (uint32_t k = 0; k < m; ++k)
                lanes[k] = k;
            bool first_round = true;
            for (int round = 0; !lanes.empty(); ++round) {
                if (round > (int)C)
                    return -3;
                std::shuffle(lanes.begin(), lanes.end(), rng);
                parked.clear();
                for (uint32_t lane : lanes) {
                    uint32_t F, L, gx;
                    int dl, dr;
                    bool resumed = !first_round;
                    if (first_round) {
                        F = L = C0 + lane;
                        dl = A.at(F - 1);
                        dr = A.at(L);
                        gx = kEnd;
                    } else {   // a parked node: resume from its slot
                        const uint32_t K = C0 + lane, e = other[lane];
                        F = e < K ? e : K;
                        L = e < K ? K : e;
                        dl = sdl[lane];
                        dr = sdr[lane];
                        gx = spl[lane];
                    }
                    for (int merges = 0;; ++merges) {
                        if (F == 0 && L == M - 1) {
                            if (F < L) {
                                slot_node[0] = 0;
                                other[0] = L;
                                sdl[0] = dl;
                                sdr[0] = dr;
                                spl[0] = gx;
                            }
                            break;
                        }
                        const bool rt = dr > dl;
                        const uint32_t id = F == L ? item_id(F) : (rt ? last(L) : first(F));
                        const uint32_t s = (rt ? L : F) - C0;
                        if (s >= m)
                            return -4;
                        if (F < L && !resumed) {
                            slot_node[s] = id;
                            other[s] = rt ? F : L;
                            sdl[s] = dl;
                            sdr[s] = dr;
                            spl[s] = gx;
                        }
                        resumed = false;
                        if (merges == kSteps) {
                            if (F == L || slot_node[s] != id)
                                return -11;   // only formed nodes park, in their own slot
                            parked.push_back(s);
                            break;
                        }
                        const uint32_t g = rt ? L : F - 1;
                        if (g < C0 || g + 1 >= C0 + m) {
                            hand_up(F, L, id, dr);
                            break;
                        }
                        if (cnt[g - C0] & (rt ? 1u : 2u))
                            return -6;   // one child arrived twice
                        const uint32_t old = cnt[g - C0];
                        cnt[g - C0] |= rt ? 1u : 2u;
                        if (old == 0)
                            break;
                        const uint32_t near = rt ? L + 1 : F - 1, ns = near - C0;
                        if (ns >= m)
                            return -4;
                        const bool single = spl[ns] == kEnd;
                        const uint32_t far = other[ns];
                        if (far - C0 >= m || (rt ? far < near : far > near))
                            return -6;
                        // the kernel's choice agrees with the prefixes: the
                        // sibling is a single item exactly when that item's
                        // own parent is this node's parent
                        if (single != ((rt ? dr : dl) > A.at(rt ? near : near - 1)))
                            return -12;
                        const uint32_t sid = single ? item_id(near) : (rt ? first(near) : last(near));
                        if (slot_node[ns] != sid)
                            return -6;   // the slot does not hold the sibling's box
                        gx = g;
                        if (rt) {
                            L = far;
                            dr = sdr[ns];
                        } else {
                            F = far;
                            dl = sdl[ns];
                        }
                    }
                    if (fault)
                        return -7;
                }
                lanes = parked;
                first_round = false;
            }
            for (uint32_t t = 0; t + 1 < m; ++t) {
                const uint32_t c = cnt[t];
                if (c == 1 || c == 2) {
                    const uint32_t s = c == 1 ? t : t + 1, K = C0 + s;
                    const bool isformed =
                        spl[s] != kEnd && (c == 1 ? other[s] < K : other[s] > K);
                    const uint32_t F = isformed && c == 1 ? other[s] : K;
                    const uint32_t L = isformed && c == 2 ? other[s] : K;
                    hand_up(F, L, F == L ? item_id(K) : (c == 1 ? last(L) : first(F)), A.at(L));
                }
            }
            for (uint32_t r = 0; r < m; ++r) {
                if (spl[r] == kEnd)
                    continue;
                const uint32_t K = C0 + r, e = other[r];
                const uint32_t F = e < K ? e : K, L = e < K ? K : e, g = spl[r];
                const uint32_t id = e < K ? last(L) : first(F);
                if (id >= N - 1 || formed[id])
                    return -2;
                formed[id] = 1;
                left[id] = F == g ? item_id(g) : last(g);
                right[id] = g + 1 == L ? item_id(L) : first(g + 1);
                const uint32_t rr = last(L);
                esc_inner[id] = rr >= N - 1 ? kEnd
                                : (rr + 1 <= N - 2 && a_first(L + 1) >= A.at(L) ? rr + 1
                                                                              : N + rr);
            }
            if (roots.size() > kOut)
                return -5;
            std::sort(roots.begin(), roots.end(),
                      [](const HcItem &x, const HcItem &y) { return x.f < y.f; });
            next.insert(next.end(), roots.begin(), roots.end());
            if (fault)
                return -7;
        }
        if (next.size() >= items.size() && !next.empty())
            return -8;   // no progress
        items.swap(next);
    }
    for (uint32_t i = 0; i + 1 < N; ++i)
        if (!formed[i])
            return -10;   // an inner node never formed
    return 0;
}

} // extern "C"
