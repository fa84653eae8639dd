// k_agglo.hip -- hierarchy, inner boxes and skip links in one bottom-up pass,
// over leaf records that are already in place in key order.
//
// The tree is the AABB tree of Sec. 3.2 over 4D boxes, with the key of leaf j
// being its time slab (j / m for slabs of m leaves) above the 30-bit Morton
// code of its centre, as in the top-down build (k_tree.hip).  The same binary
// radix tree can be found from the leaves up (Apetrei 2014): a node covering
// leaves [f, l] is the left child of its parent when keys l and l+1 share a
// longer prefix than keys f-1 and f (the parent is then [f, l'], split after
// leaf l) and the right child otherwise (parent [f', l], split after f-1).
// Every split between two neighbouring leaves belongs to exactly one inner
// node, so it is where that node's two children meet; as in the atomic refit,
// the second child to arrive goes on with the union of the two boxes and
// records the pair when the two overlap (a seed of the node-pair traversal).
// Ties cannot occur: with positions breaking equal keys, the prefixes on the
// two sides of a node always differ.  A node's parent side, its sibling's
// shape and every skip link follow from the adjacent prefixes
// a(j) = delta(j, j+1) alone.
//
// Node ids are those of the top-down build: an inner node is numbered by the
// last leaf of its range when it is a left child, by the first when it is a
// right child, and the root is 0.  So the tree written here (records, child
// pairs, skip links, leaf skip links in the side array) is the same tree, and
// the build needs none of the per-node binary searches nor the parent, level
// and skip-link arrays that pass the top-down hierarchy to the refit.
//
// Passes: one workgroup per chunk of C consecutive items, every meeting held
// in LDS.  A chunk's nodes whose parents reach outside it (a split at the
// chunk's edge, or a split whose other child never arrives) are its roots;
// they are handed up, in position order, as the items of the next pass, which
// builds the tree above them the same way (the adjacent prefix between two
// consecutive roots is the one between their end leaves).  Pass 1's items are
// the leaves; the pass whose items fit one chunk forms the root.  The item
// counts of later passes stay on the device: each later pass is launched for
// a bound on its count, as a small grid that strides over the chunks holding
// items.
//
// Leaves come either in place (FP64 records the sorted-layout box build wrote
// in key order; keys from the slab of each position and the packed codes) or
// from the general key sort (per-object steps): pass 1 then reads each leaf's
// box through the sorted (key, box index) items, writes its leaf record and
// takes the keys from the same items.  An FP32 tree holds the outward-rounded
// boxes; its nodes are formed from those rounded values (held as doubles,
// exactly), so unions and sibling tests equal what its float records give.
#include <type_traits>

#include "cd_internal.h"

namespace cd {

namespace {

inline unsigned nblk(uint64_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

constexpr int kAggChunk = 1024;
constexpr int kAggOut = 256;   // roots one chunk may hand up
constexpr int kAggScanThreads = 1024;

// A node handed to the next pass: leaf range, id, and the adjacent prefixes
// after its first and after its last leaf, a(f) + 1 | (a(l) + 1) << 8.
struct AggItem {
    uint32_t f, l, id, a;
};
static_assert(sizeof(AggItem) == 16, "AggItem layout");

// Keys and boxes of the gathered leaves: the key sort's output, (slab << 32
// | code, box) items or words slab << (cb + ib) | code << ib | box (pk set);
// or boxes already in key order (code set: leaf j is box j, its key
// (j / ms) << 32 | code[j], as for records in place).
struct KVKeys {
    const KV *kv;
    uint32_t N;
    const uint64_t *pk;
    uint32_t ib, cb;
    const uint32_t *code;
    uint32_t ms;
    __device__ uint64_t key(uint32_t j) const
    {
        if (code)
            return ((uint64_t)(j / ms) << 32) | code[j];
        if (!pk)
            return kv[j].key;
        const uint64_t w = pk[j];
        return ((w >> (cb + ib)) << 32) | ((uint32_t)(w >> ib) & ((1u << cb) - 1));
    }
    __device__ uint32_t box(uint32_t j) const
    {
        return code ? j : pk ? (uint32_t)(pk[j] & ((1ull << ib) - 1)) : kv[j].val;
    }
};

// Pass 1's leaf source.  GATHER < 0: FP64 leaf records in place, CodeKeys;
// otherwise boxes of precision GATHER read through KVKeys.
template <int GATHER>
using LeafKeys = typename std::conditional<(GATHER >= 0), KVKeys, CodeKeys>::type;

// The node at one item position in LDS: four 16-byte words laid out as an
// FP64 tree record's (lo0 lo1 | lo2 hi0 | hi1 hi2 | t0 t1 other packed): its
// box, its other range end and packed = (dl + 1) | (dr + 1) << 8 |
// split << 16, with dl and dr the adjacent prefixes before its first and
// after its last item and split its split relative to the chunk (kNoSplit:
// the item itself, not yet replaced by a node formed here).  Word q of slot s
// sits at position q ^ ((s >> 1) & 3) of the slot, so that 16-byte accesses
// by lanes at neighbouring slots fall in different LDS banks.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
struct SlotRec {
    double lo[3], hi[3];
    uint32_t t0, t1, other, packed;
};
constexpr uint32_t kNoSplit = 0xFFFFu;
constexpr int kAggSteps = 3;   // merges per round before a climber is parked

__device__ inline uint32_t pack_ends(int dl, int dr, uint32_t split)
{
    return (uint32_t)(dl + 1) | ((uint32_t)(dr + 1) << 8) | (split << 16);
}

__device__ inline uint32_t swz(uint32_t s) { return (s >> 1) & 3u; }

__device__ inline u32x4 two_doubles(double a, double b)
{
    const uint64_t x = __builtin_bit_cast(uint64_t, a), y = __builtin_bit_cast(uint64_t, b);
    return u32x4{(uint32_t)x, (uint32_t)(x >> 32), (uint32_t)y, (uint32_t)(y >> 32)};
}
__device__ inline double first_double(u32x4 v)
{
    return __builtin_bit_cast(double, (uint64_t)v.x | ((uint64_t)v.y << 32));
}
__device__ inline double second_double(u32x4 v)
{
    return __builtin_bit_cast(double, (uint64_t)v.z | ((uint64_t)v.w << 32));
}

__device__ inline void put_slot(u32x4 (*rec)[4], uint32_t s, const double lo[3],
                                const double hi[3], uint32_t t0, uint32_t t1, uint32_t other,
                                uint32_t packed)
{
    const uint32_t z = swz(s);
    rec[s][0 ^ z] = two_doubles(lo[0], lo[1]);
    rec[s][1 ^ z] = two_doubles(lo[2], hi[0]);
    rec[s][2 ^ z] = two_doubles(hi[1], hi[2]);
    rec[s][3 ^ z] = u32x4{t0, t1, other, packed};
}
__device__ inline SlotRec get_slot(const u32x4 (*rec)[4], uint32_t s)
{
    const uint32_t z = swz(s);
    const u32x4 a = rec[s][0 ^ z], b = rec[s][1 ^ z], c = rec[s][2 ^ z], d = rec[s][3 ^ z];
    SlotRec r;
    r.lo[0] = first_double(a);
    r.lo[1] = second_double(a);
    r.lo[2] = first_double(b);
    r.hi[0] = second_double(b);
    r.hi[1] = first_double(c);
    r.hi[2] = second_double(c);
    r.t0 = d.x;
    r.t1 = d.y;
    r.other = d.z;
    r.packed = d.w;
    return r;
}
// word 3 alone: {t0, t1, other, packed}
__device__ inline u32x4 slot_tags(const u32x4 (*rec)[4], uint32_t s) { return rec[s][3 ^ swz(s)]; }

// LDS of one chunk pass.
template <int C, bool LEAVES>
struct AggShared {
    uint8_t sa[C + 4];                // a(last leaf) + 1, items C0 - 2 .. C0 + m
    uint8_t sf[LEAVES ? 1 : C + 1];   // a(first leaf) + 1, items C0 .. C0 + m
    uint32_t itf[LEAVES ? 1 : C], itl[LEAVES ? 1 : C], itd[LEAVES ? 1 : C];
    u32x4 rec[C][4];                  // slot records, words swizzled
    unsigned int cnt[C / 4];          // four 8-bit arrival counts per word
    uint32_t park[2][C / 4];          // parked climbers (slots), alternate rounds
    uint2 sbuf[kSeedStage];
    AggItem pst[kAggOut];
    unsigned int sn, sbase, pn, npark[2];
};

}  // namespace

// One chunk of one pass over M items (LEAVES: the N leaves themselves), C
// threads, one item per thread.  Every meeting is in LDS: a step is the
// arrival atomic on the split's count (1: the left child arrived, 2: the
// right child, 3: both) and one 64-byte read of the sibling's slot.  A slot
// first holds its item; the node formed with that position as its id end
// overwrites it (by then the item's parent is formed, and only an ancestor of
// an item can end at it).  Climbs run in rounds of kAggSteps merges: a
// climber still going after that many is parked in its node's slot, and the
// next round resumes the parked ones packed into the first lanes, so the
// sparse top of the chunk's tree costs one wave rather than every wave.
// Roots go to out[chunk][0 .. kAggOut) in position order, their count to
// out_count[chunk].
// TP: tree precision (FP32 only with GATHER >= 0).  The leaf skip links go to
// leaf_esc (FP64 trees) or into the FP32 tree's link records.
template <int C, bool LEAVES, int TP, int GATHER>
__device__ void agglo_chunk(AggShared<C, LEAVES> &S, uint32_t chunk, uint32_t M,
                            LeafKeys<GATHER> G, const BoxView &bv, uint32_t slab_ticks,
                            const AggItem *__restrict__ in, void *__restrict__ nodes,
                            uint2 *__restrict__ kids, uint32_t *__restrict__ leaf_esc,
                            AggItem *__restrict__ out, uint32_t *__restrict__ out_count,
                            const SeedSink &seeds, bool &bad, bool &misplaced)
{
    static_assert(TP == CD_FP64 || GATHER >= 0, "FP32 trees take their leaves by gather");
    const SeedStage stage{S.sbuf, &S.sn};
    const uint32_t N = G.N, t = threadIdx.x, C0 = chunk * (uint32_t)C;
    const uint32_t m = M - C0 < (uint32_t)C ? M - C0 : (uint32_t)C;
    const uint32_t wlo = C0 - 2;   // LDS window: items C0 - 2 .. C0 + m
    double lo[3], hi[3];
    uint32_t t0 = 0, t1 = 0, lobj = 0;
    if (LEAVES && t < m) {   // the leaf's box, in flight with the keys
        if constexpr (GATHER >= 0) {
            const uint32_t src = G.box(C0 + t);
            load_box<(GATHER >= 0 ? GATHER : CD_FP64)>(bv, src, lo, hi);
            if (TP == CD_FP32)
                for (int d = 0; d < 3; ++d) {
                    lo[d] = (double)__double2float_rd(lo[d]);
                    hi[d] = (double)__double2float_ru(hi[d]);
                }
            t0 = bv.t0[src];
            t1 = bv.t1[src];
            lobj = bv.obj[src];
            if (G.code)   // boxes in key order: each in its slab
                misplaced |= t0 / slab_ticks != (C0 + t) / G.ms;
        } else {
            NodeIO<CD_FP64>::get_box(nodes, N, N - 1 + C0 + t, lo, hi, t0, t1);
            misplaced |= t0 / slab_ticks != (C0 + t) / G.ms;
        }
    }
    for (uint32_t k = t; k < m + 3; k += C) {
        const uint32_t K = wlo + k;
        if (LEAVES) {   // a(j) and the key order, from the codes
            uint8_t v = 0;
            if (K < N - 1) {
                const uint64_t a = G.key(K), b = G.key(K + 1);
                v = (uint8_t)(key_prefix(a, b, K, K + 1) + 1);
                misplaced |= a > b;
            }
            S.sa[k] = v;
        } else {
            const AggItem it = K < M ? in[K] : AggItem{0, 0, 0, 0};
            S.sa[k] = (uint8_t)(it.a >> 8);
            if (k >= 2) {
                S.sf[k - 2] = (uint8_t)it.a;
                if (k - 2 < m) {
                    S.itf[k - 2] = it.f;
                    S.itl[k - 2] = it.l;
                    S.itd[k - 2] = it.id;
                }
            }
        }
    }
    if (t == 0) {
        S.sn = 0;
        S.pn = 0;
        S.npark[0] = 0;
        S.npark[1] = 0;
    }
    if (t < (uint32_t)C / 4)
        S.cnt[t] = 0;
    __syncthreads();
    // item K (in this chunk): first and last leaf, id, prefix after its first leaf
    const AdjBytes A{S.sa, wlo, M};
    auto first = [&](uint32_t K) { return LEAVES ? K : S.itf[K - C0]; };
    auto last = [&](uint32_t K) { return LEAVES ? K : S.itl[K - C0]; };
    auto item_id = [&](uint32_t K) { return LEAVES ? N - 1 + K : S.itd[K - C0]; };
    auto a_first = [&](uint32_t K) { return LEAVES ? A.at(K) : (int)S.sf[K - C0] - 1; };
    if (t < m) {
        const uint32_t K = C0 + t;
        if (LEAVES) {
            const uint32_t e = escape_adj(A, N, K);
            if (GATHER >= 0 && TP == CD_FP32) {   // the leaf record with its links
                NodeIO<TP>::put(nodes, N, N - 1 + K, lo, hi, t0, t1, lobj, e);
            } else {
                if (GATHER >= 0)   // the record; its skip link goes to the side
                    NodeIO<CD_FP64>::put(nodes, N, N - 1 + K, lo, hi, t0, t1, lobj, 0u);
                leaf_esc[K] = e;
            }
        } else {
            NodeIO<TP>::get_box(nodes, N, item_id(K), lo, hi, t0, t1);
        }
        put_slot(S.rec, t, lo, hi, t0, t1, K, pack_ends(A.at(K - 1), A.at(K), kNoSplit));
    }
    __syncthreads();
    // hand node [F, L] (items) up to the next pass
    auto hand_up = [&](uint32_t F, uint32_t L, uint32_t id, int dr) {
        const unsigned int k = atomicAdd(&S.pn, 1u);
        if (k < (unsigned)kAggOut)
            S.pst[k] = AggItem{first(F), last(L), id,
                               (uint32_t)(a_first(F) + 1) | ((uint32_t)(dr + 1) << 8)};
    };
    uint32_t F = C0 + t, L = F, gx = kNoSplit;
    int dl = A.at(F - 1), dr = A.at(L);
    bool go = t < m, resumed = false;
    for (uint32_t round = 0;; ++round) {
        for (int merges = 0; go; ++merges) {
            if (F == 0 && L == M - 1) {   // the root
                if (F < L)
                    put_slot(S.rec, 0, lo, hi, t0, t1, L, pack_ends(dl, dr, gx));
                go = false;
                break;
            }
            const bool right = dr > dl;   // a left child: the parent extends right
            const uint32_t id = F == L ? item_id(F) : (right ? last(L) : first(F));
            const uint32_t s = (right ? L : F) - C0;
            if (F < L && !resumed)   // formed here: its slot (the id end's)
                put_slot(S.rec, s, lo, hi, t0, t1, right ? F : L, pack_ends(dl, dr, gx));
            resumed = false;
            if (merges == kAggSteps) {   // park it for the next round
                S.park[round & 1][atomicAdd(&S.npark[round & 1], 1u)] = s;
                go = false;
                break;
            }
            const uint32_t g = right ? L : F - 1;
            if (g < C0 || g + 1 >= C0 + m) {   // a split at the chunk's edge
                hand_up(F, L, id, dr);
                go = false;
                break;
            }
            const uint32_t gs = g - C0, sh = 8u * (gs & 3u);
            const unsigned int old = __hip_atomic_fetch_add(&S.cnt[gs >> 2], (right ? 1u : 2u) << sh,
                                                            __ATOMIC_ACQ_REL,
                                                            __HIP_MEMORY_SCOPE_WORKGROUP);
            if (((old >> sh) & 0xFFu) == 0) {   // first to arrive: the sibling goes on
                go = false;
                break;
            }
            // the sibling's slot (inside the chunk: the split is not at its
            // edge) holds the single item next to this node, or the node
            // formed with that item as its id end
            const uint32_t near = right ? L + 1 : F - 1;
            const SlotRec o = get_slot(S.rec, near - C0);
            const bool single = (o.packed >> 16) == kNoSplit;
            const uint32_t sid = single ? item_id(near) : (right ? first(near) : last(near));
            bad |= o.other - C0 >= m || (right ? o.other < near : o.other > near);
            if (time_overlap(t0, t1, o.t0, o.t1) && space_overlap(lo, hi, o.lo, o.hi))
                stage.push(seeds, right ? id : sid, right ? sid : id);
            unite(lo, hi, t0, t1, o.lo, o.hi, o.t0, o.t1);
            gx = gs;
            if (right) {
                L = o.other;
                dr = (int)((o.packed >> 8) & 0xFFu) - 1;
            } else {
                F = o.other;
                dl = (int)(o.packed & 0xFFu) - 1;
            }
        }
        __syncthreads();
        const uint32_t np = S.npark[round & 1];
        __syncthreads();
        if (np == 0 || round > (uint32_t)C)
            break;
        if (t == 0)
            S.npark[round & 1] = 0;   // next written two rounds on, after a barrier
        go = t < np;
        if (go) {   // resume a parked climber from its slot
            const uint32_t s = S.park[round & 1][t];
            const SlotRec o = get_slot(S.rec, s);
            const uint32_t K = C0 + s;
            F = o.other < K ? o.other : K;
            L = o.other < K ? K : o.other;
            dl = (int)(o.packed & 0xFFu) - 1;
            dr = (int)((o.packed >> 8) & 0xFFu) - 1;
            gx = o.packed >> 16;
            for (int d = 0; d < 3; ++d) {
                lo[d] = o.lo[d];
                hi[d] = o.hi[d];
            }
            t0 = o.t0;
            t1 = o.t1;
            resumed = true;
        }
    }
    // roots whose sibling never arrived (count 1: the left child, 2: the right)
    if (t + 1 < m) {
        const uint32_t c = (S.cnt[t >> 2] >> (8u * (t & 3u))) & 0xFFu;
        if (c == 1 || c == 2) {
            const uint32_t s = c == 1 ? t : t + 1, K = C0 + s;
            const u32x4 w = slot_tags(S.rec, s);
            const uint32_t e = w.z;
            const bool formed = (w.w >> 16) != kNoSplit && (c == 1 ? e < K : e > K);
            const uint32_t F = formed && c == 1 ? e : K, L = formed && c == 2 ? e : K;
            const uint32_t id = F == L ? item_id(K) : (c == 1 ? last(L) : first(F));
            hand_up(F, L, id, A.at(L));
        }
    }
    // records of the nodes formed here: the id end of a left child is its
    // last item, of a right child (or the root) its first
    auto node_of = [&](uint32_t r, uint32_t &F, uint32_t &L) {
        const uint32_t K = C0 + r, e = slot_tags(S.rec, r).z;
        F = e < K ? e : K;
        L = e < K ? K : e;
        return e < K ? last(L) : first(F);
    };
    auto kids_of = [&](uint32_t F, uint32_t L, uint32_t g) {
        return make_uint2(F == g ? item_id(g) : last(g), g + 1 == L ? item_id(L) : first(g + 1));
    };
    auto esc_of = [&](uint32_t L) {   // skip link of a node ending with item L
        const uint32_t r = last(L);
        if (r >= N - 1)
            return kEnd;
        const uint32_t s = r + 1;
        return s <= N - 2 && a_first(L + 1) >= A.at(L) ? s : N - 1 + s;
    };
    auto split_at = [&](uint32_t r) { return slot_tags(S.rec, r).w >> 16; };
    if (LEAVES && TP == CD_FP64) {
        // id = C0 + r: four lanes per record, each writing 16 bytes, so a
        // wave's store writes 16 whole consecutive records
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t x = t + (uint32_t)C * (uint32_t)j, r = x >> 2, q = x & 3u;
            if (r < m && split_at(r) != kNoSplit) {
                uint32_t F, L;
                const uint32_t id = node_of(r, F, L);
                u32x4 v = S.rec[r][q ^ swz(r)];
                if (q == 3) {
                    v.z = kids_of(F, L, C0 + (v.w >> 16)).x;
                    v.w = esc_of(L);
                }
                __builtin_nontemporal_store(v, (u32x4 *)((Node64 *)nodes + id) + q);
            }
        }
        if (t < m && split_at(t) != kNoSplit) {
            uint32_t F, L;
            const uint32_t id = node_of(t, F, L);
            kids[id] = kids_of(F, L, C0 + split_at(t));
        }
    } else if (t < m && split_at(t) != kNoSplit) {
        uint32_t F, L;
        const uint32_t id = node_of(t, F, L);
        const uint2 kd = kids_of(F, L, C0 + split_at(t));
        const SlotRec o = get_slot(S.rec, t);
        NodeIO<TP>::put(nodes, N, id, o.lo, o.hi, o.t0, o.t1, kd.x, esc_of(L));
        kids[id] = kd;
    }
    __syncthreads();
    // seeds out; roots out in position order (rank: roots starting before)
    const uint32_t np = S.pn < (unsigned)kAggOut ? S.pn : (unsigned)kAggOut;
    if (t == 0) {
        const uint32_t ms = S.sn < (unsigned)kSeedStage ? S.sn : (unsigned)kSeedStage;
        S.sbase = ms ? seeds.reserve(ms) : 0u;
        out_count[chunk] = np;
        bad |= S.pn > (unsigned)kAggOut;
    }
    for (uint32_t k = t; k < np; k += C) {
        const AggItem it = S.pst[k];
        uint32_t rank = 0;
        for (uint32_t q = 0; q < np; ++q)
            rank += S.pst[q].f < it.f;
        out[(size_t)chunk * kAggOut + rank] = it;
    }
    __syncthreads();
    const uint32_t ms = S.sn < (unsigned)kSeedStage ? S.sn : (unsigned)kSeedStage;
    for (uint32_t k = t; k < ms; k += C)
        if (S.sbase + k < seeds.cap)
            seeds.items[S.sbase + k] = S.sbuf[k];
    __syncthreads();   // the LDS is reused by the next chunk
}

// Pass 1: one workgroup per chunk of leaves (consecutive chunks on one XCD).
template <int C, int TP, int GATHER>
__global__ __launch_bounds__(C) __attribute__((amdgpu_waves_per_eu(8))) void k_agglo_leaves(
    LeafKeys<GATHER> G, BoxView bv, uint32_t slab_ticks, void *__restrict__ nodes,
    uint2 *__restrict__ kids, uint32_t *__restrict__ leaf_esc, AggItem *__restrict__ out,
    uint32_t *__restrict__ out_count, SeedSink seeds, unsigned int *err)
{
    __shared__ AggShared<C, true> S;
    bool bad = false, misplaced = false;
    agglo_chunk<C, true, TP, GATHER>(S, xcd_block(blockIdx.x, gridDim.x), G.N, G, bv, slab_ticks,
                                     nullptr, nodes, kids, leaf_esc, out, out_count, seeds, bad,
                                     misplaced);
    if (misplaced)
        atomicOr(err, 1u);
    if (bad)
        atomicOr(err, 2u);
}

// Later passes: the item count is on the device; a small grid strides over
// the chunks that hold items.
template <int C, int TP>
__global__ __launch_bounds__(C) void k_agglo_items(uint32_t N, const AggItem *__restrict__ in,
                                                   const uint32_t *__restrict__ in_count,
                                                   void *__restrict__ nodes,
                                                   uint2 *__restrict__ kids,
                                                   AggItem *__restrict__ out,
                                                   uint32_t *__restrict__ out_count,
                                                   SeedSink seeds, unsigned int *err)
{
    __shared__ AggShared<C, false> S;
    const uint32_t M = *in_count;
    const KVKeys G{nullptr, N, nullptr, 0, 0, nullptr, 1};   // items carry their prefixes
    const BoxView bv{};
    bool bad = false, misplaced = false;
    for (uint32_t c = blockIdx.x; (uint64_t)c * C < M; c += gridDim.x)
        agglo_chunk<C, false, TP, 0>(S, c, M, G, bv, 1, in, nodes, kids, nullptr, out, out_count,
                                     seeds, bad, misplaced);
    if (bad)
        atomicOr(err, 2u);
}

// Exclusive scan of the chunks' root counts (one workgroup) into offsets, and
// the next pass's item count into *next_count.  Only the ceil(M / C) chunks
// that had items wrote a count.  Each wave owns one contiguous segment, read
// 64 counts at a time with kScanBatch reads in flight: a first sweep sums it,
// the segment sums are scanned across the waves, and a second sweep writes
// the offsets.
// With `next` set (passes with few chunks) the same workgroup then moves
// every chunk's roots to their places, as k_agglo_compact does.
__global__ __launch_bounds__(kAggScanThreads) void k_agglo_scan(const uint32_t *counts,
                                                                const uint32_t *in_count,
                                                                uint32_t M_host, uint32_t C,
                                                                uint32_t *offsets,
                                                                uint32_t *next_count,
                                                                const AggItem *stage,
                                                                AggItem *next)
{
    __shared__ uint32_t wsum[33];
    const uint32_t M = in_count ? *in_count : M_host;
    const uint32_t nc = (M + C - 1) / C;
    const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = kAggScanThreads / 64;
    const uint32_t seg = ((nc + nw - 1) / nw + 63) & ~63u;
    const uint32_t b0 = w * seg, b1 = b0 + seg < nc ? b0 + seg : nc;
    constexpr uint32_t kScanBatch = 8;
    uint32_t part = 0;
    for (uint32_t k0 = b0; k0 < b1; k0 += 64 * kScanBatch) {
        uint32_t v[kScanBatch];
#pragma unroll
        for (uint32_t u = 0; u < kScanBatch; ++u) {
            const uint32_t k = k0 + 64 * u + lane;
            v[u] = k < b1 ? counts[k] : 0u;
        }
#pragma unroll
        for (uint32_t u = 0; u < kScanBatch; ++u)
            part += v[u];
    }
    for (int o = 32; o >= 1; o >>= 1)
        part += __shfl_xor(part, o, 64);
    uint32_t total;
    // every lane of wave w holds the segment sum; lane 0 enters it
    uint32_t run = block_exclusive_scan(lane == 0 ? part : 0u, wsum, &total);
    run = __shfl(run, 0, 64);
    for (uint32_t k0 = b0; k0 < b1; k0 += 64 * kScanBatch) {
        uint32_t v[kScanBatch];
#pragma unroll
        for (uint32_t u = 0; u < kScanBatch; ++u) {
            const uint32_t k = k0 + 64 * u + lane;
            v[u] = k < b1 ? counts[k] : 0u;
        }
#pragma unroll
        for (uint32_t u = 0; u < kScanBatch; ++u) {
            const uint32_t k = k0 + 64 * u + lane;
            const uint32_t inc = wave_inclusive_scan(v[u]);
            if (k < b1)
                offsets[k] = run + inc - v[u];
            run += __shfl(inc, 63, 64);
        }
    }
    if (threadIdx.x == 0)
        *next_count = total;
    if (!next)
        return;
    __syncthreads();   // the offsets written by the other waves
    for (uint32_t c = w; c < nc; c += nw) {
        const uint32_t n = counts[c], o = offsets[c];
        for (uint32_t k = lane; k < n; k += 64)
            next[o + k] = stage[(size_t)c * kAggOut + k];
    }
}

// Every chunk's roots to their places in the next pass's item list: one wave
// per chunk, a small grid striding over the chunks that held items.
__global__ __launch_bounds__(256) void k_agglo_compact(const AggItem *stage, const uint32_t *counts,
                                                       const uint32_t *offsets,
                                                       const uint32_t *in_count, uint32_t M_host,
                                                       uint32_t C, AggItem *next)
{
    const uint32_t M = in_count ? *in_count : M_host;
    const uint32_t nc = (M + C - 1) / C;
    const uint32_t lane = threadIdx.x & 63, waves = gridDim.x * (blockDim.x / 64);
    for (uint32_t c = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); c < nc; c += waves) {
        const uint32_t n = counts[c], o = offsets[c];
        for (uint32_t k = lane; k < n; k += 64)
            next[o + k] = stage[(size_t)c * kAggOut + k];
    }
}

size_t agglo_ws_bytes(uint32_t N)
{
    const size_t chunks = (N + kAggChunk - 1) / kAggChunk;
    return 3 * align_up(chunks * kAggOut * sizeof(AggItem), 256) +
           2 * align_up((chunks + 1) * sizeof(uint32_t), 256) + 256 + 6 * 256;
}

namespace {

// The workspace: pass 1's roots per chunk (stage), two item lists for
// alternate passes, per-chunk root counts and offsets, the item counts.
struct AggPlan {
    AggItem *stage, *items[2];
    uint32_t *counts, *offsets, *totals;
};

AggPlan agglo_plan(void *ws, uint32_t N)
{
    const size_t chunks1 = (N + kAggChunk - 1) / kAggChunk;
    Carve cv(ws, agglo_ws_bytes(N));
    AggPlan P;
    P.stage = cv.take<AggItem>(chunks1 * kAggOut);
    P.items[0] = cv.take<AggItem>(chunks1 * kAggOut);
    P.items[1] = cv.take<AggItem>(chunks1 * kAggOut);
    P.counts = cv.take<uint32_t>(chunks1 + 1);
    P.offsets = cv.take<uint32_t>(chunks1 + 1);
    P.totals = cv.take<uint32_t>(2);
    return P;
}

}  // namespace

namespace {

// Passes 2, 3, ... over the roots pass 1 left in its chunks' slots.
template <int TP>
hipError_t agglo_item_passes(uint32_t N, void *nodes, uint2 *kids, const AggPlan &P,
                             const SeedSink &seeds, unsigned int *err, hipStream_t s)
{
    constexpr int C = kAggChunk;
    // item passes: workgroups striding over the chunks; compaction grid; up
    // to kFuseChunks chunks the scan's workgroup also compacts
    constexpr uint32_t kItemGrid = 512, kCompactGrid = 4096, kFuseChunks = 1024;
    uint32_t bound = N;   // pass 1: the leaves
    const uint32_t *in_count = nullptr;   // null: the count is `bound` (pass 1)
    int cur = 0;
    hipError_t e = hipSuccess;
    while (e == hipSuccess && bound > (uint32_t)C) {
        const uint32_t nchunks = nblk(bound, C);
        uint32_t *next_count = P.totals + cur;
        const bool fuse = nchunks <= kFuseChunks;
        k_agglo_scan<<<1, kAggScanThreads, 0, s>>>(P.counts, in_count, bound, C, P.offsets,
                                                   next_count, fuse ? P.stage : nullptr,
                                                   fuse ? P.items[cur] : nullptr);
        if ((e = hipGetLastError()) != hipSuccess)
            break;
        if (!fuse) {
            const uint32_t cgrid = nblk(nchunks, 4);
            k_agglo_compact<<<cgrid < kCompactGrid ? cgrid : kCompactGrid, 256, 0, s>>>(
                P.stage, P.counts, P.offsets, in_count, bound, C, P.items[cur]);
            if ((e = hipGetLastError()) != hipSuccess)
                break;
        }
        in_count = next_count;
        const uint64_t b = (uint64_t)nchunks * kAggOut;
        bound = b < bound ? (uint32_t)b : bound;
        const uint32_t grid = nblk(bound, C) < kItemGrid ? nblk(bound, C) : kItemGrid;
        k_agglo_items<C, TP><<<grid, C, 0, s>>>(N, P.items[cur], in_count, nodes, kids, P.stage,
                                                 P.counts, seeds, err);
        e = hipGetLastError();
        cur ^= 1;
    }
    return e;
}

}  // namespace

hipError_t launch_agglo(const uint32_t *code, uint32_t slab_size, uint32_t slab_ticks,
                        uint32_t N, void *nodes, uint2 *kids, uint32_t *leaf_esc, void *ws,
                        const SeedSink &seeds, unsigned int *err, hipStream_t s)
{
    if (N == 0)
        return hipSuccess;
    if (!code || slab_size == 0 || slab_ticks == 0 || !ws)
        return hipErrorInvalidValue;
    constexpr int C = kAggChunk;
    const AggPlan P = agglo_plan(ws, N);
    const CodeKeys G{code, slab_size, N};
    k_agglo_leaves<C, CD_FP64, -1><<<nblk(N, C), C, 0, s>>>(G, BoxView{}, slab_ticks, nodes, kids,
                                                            leaf_esc, P.stage, P.counts, seeds,
                                                            err);
    hipError_t e = hipGetLastError();
    return e != hipSuccess ? e : agglo_item_passes<CD_FP64>(N, nodes, kids, P, seeds, err, s);
}

hipError_t launch_agglo_gather(const AggLeafSource &src, const BoxView &bv, int box_precision,
                               int tree_precision, uint32_t N, void *nodes, uint2 *kids,
                               uint32_t *leaf_esc, void *ws, const SeedSink &seeds,
                               unsigned int *err, hipStream_t s)
{
    if (N == 0)
        return hipSuccess;
    const bool by_code = src.code && src.slab_size > 0 && src.slab_ticks > 0;
    const bool by_packed = src.packed && src.ib >= 1 && src.ib <= 32 &&
                           (uint64_t)N <= (1ull << src.ib) && src.cb >= 1 &&
                           src.cb <= kKeyCodeBits;
    if (!(by_code || by_packed || src.kv) || !ws ||
        (tree_precision == CD_FP64 && (!leaf_esc || box_precision != CD_FP64)))
        return hipErrorInvalidValue;
    constexpr int C = kAggChunk;
    const AggPlan P = agglo_plan(ws, N);
    const KVKeys G{by_code || by_packed ? nullptr : src.kv, N, by_code ? nullptr : src.packed,
                   src.ib, src.cb, by_code ? src.code : nullptr, by_code ? src.slab_size : 1u};
    const uint32_t w = by_code ? src.slab_ticks : 1u;
    const unsigned g = nblk(N, C);
    if (tree_precision == CD_FP64)
        k_agglo_leaves<C, CD_FP64, CD_FP64><<<g, C, 0, s>>>(G, bv, w, nodes, kids, leaf_esc,
                                                             P.stage, P.counts, seeds, err);
    else if (box_precision == CD_FP64)
        k_agglo_leaves<C, CD_FP32, CD_FP64><<<g, C, 0, s>>>(G, bv, w, nodes, kids, nullptr,
                                                             P.stage, P.counts, seeds, err);
    else
        k_agglo_leaves<C, CD_FP32, CD_FP32><<<g, C, 0, s>>>(G, bv, w, nodes, kids, nullptr,
                                                             P.stage, P.counts, seeds, err);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    return tree_precision == CD_FP64
               ? agglo_item_passes<CD_FP64>(N, nodes, kids, P, seeds, err, s)
               : agglo_item_passes<CD_FP32>(N, nodes, kids, P, seeds, err, s);
}

} // namespace cd
