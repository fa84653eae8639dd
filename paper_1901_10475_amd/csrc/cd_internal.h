// cd_internal.h -- types and launchers shared by the library's translation
// units.  Not installed; the public surface is include/cd4d.h.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "cd4d.h"
#include "cd_logic.h"

namespace cd {

// Per-object constants of the Kepler ellipse (row of object setup).
struct ObjConst {
    double a, e, b, n, m0, vmax;  // b = a sqrt(1 - e^2); n = mean motion (rad/s)
    double P[3], Q[3];            // perifocal unit vectors in ECI
};

// Coordinate d of the orbit as one sinusoid of the eccentric anomaly:
// x_d(E) = ctr_d + R_d cos(E - phi_d) (for the eccentric-anomaly interval box).
struct ObjSinus {
    double R[3], phi[3], ctr[3];
};

// Per-object interval bookkeeping for per-object steps (object-major boxes).
struct ObjSteps {
    uint32_t dt, K;      // step and interval count
    uint32_t box_off;    // first box of the object
    uint32_t pad;
};

// Tree node layouts.  FP64: one 64-byte record per node.  FP32: a 32-byte box
// record plus an 8-byte link record in a separate array.  link is the left
// child of an inner node and the object id of a leaf; esc is the next node in
// pre-order once the node's subtree is skipped.
struct alignas(16) Node64 {
    double lo[3];
    double hi[3];
    uint32_t t0, t1, link, esc;
};
struct alignas(16) Box32 {
    float lo[3];
    float hi[3];
    uint32_t t0, t1;
};
struct Link {
    uint32_t link, esc;
};
static_assert(sizeof(Node64) == 64, "Node64 layout");
// Where the Karras pass leaves each node's (link, esc) for the refit: the
// FP32 tree's own link records, or, for an FP64 tree (whose records get both
// words from the refit, the link being the left child), the escapes alone.
struct LinkSink {
    Link *rec;       // FP32 tree link records, or nullptr
    uint32_t *esc;   // escapes only, when rec == nullptr
    __device__ void put(uint32_t id, uint32_t link, uint32_t e) const
    {
        if (rec) {
            Link l;
            l.link = link;
            l.esc = e;
            rec[id] = l;
        } else {
            esc[id] = e;
        }
    }
    __device__ uint32_t esc_of(uint32_t id) const { return rec ? rec[id].esc : esc[id]; }
};

static_assert(sizeof(Box32) == 32, "Box32 layout");

// Radix-sort items: 16 bytes each.
struct KV {
    uint64_t key;
    uint32_t val, pad;
};
struct Rec {
    uint32_t i, j, tlo, thi;
};

// Raw device view of a box set (pointers typed by precision at the use site).
struct BoxView {
    const void *lo[3], *hi[3];
    const uint32_t *t0, *t1, *obj;
    const uint32_t *code;   // Morton codes written with the boxes, or nullptr
};
struct BoxOut {
    void *lo[3], *hi[3];
    uint32_t *t0, *t1, *obj;
    uint32_t *code;                        // Morton code of each box centre, or nullptr
    const unsigned long long *frame;       // code frame: ordered bits, min xyz, max xyz
    uint64_t cap;  // entries the arrays hold; stores beyond are dropped
    // FP64 box records {lo[3], hi[3]; t0, t1, obj, code} (the layout of an
    // FP64 tree's leaf records) written instead of the arrays, or nullptr
    Node64 *rec;
};
// Word offsets of the tag fields inside a 64-byte box record (16 words).
constexpr uint32_t kRecWords = 16, kRecT0 = 12, kRecT1 = 13, kRecObj = 14, kRecCode = 15;

template <int PREC>
__device__ inline void load_box(const BoxView &b, uint64_t k, double lo[3], double hi[3])
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

// ---- wave helpers -----------------------------------------------------------------

__device__ inline uint32_t wave_inclusive_scan(uint32_t v)
{
    int lane = threadIdx.x & 63;
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t u = __shfl_up(v, o, 64);
        if (lane >= o)
            v += u;
    }
    return v;
}

// Lanes (among `active`) whose 8-bit digit equals this lane's digit.
__device__ inline uint64_t match_digit(uint32_t d, uint64_t active)
{
    uint64_t peers = active;
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
        uint64_t b = __ballot((d >> bit) & 1u);
        peers &= ((d >> bit) & 1u) ? b : ~b;
    }
    return peers;
}

__device__ inline uint64_t lanemask_lt()
{
    int lane = threadIdx.x & 63;
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// LDS written by some lanes of a wave and then read by others: the wave
// executes its LDS operations in order, so only the compiler must keep them
// in order (a fence at wavefront scope).
__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Exclusive scan over all threads of a block (blockDim multiple of 64, <= 1024).
// `wsum` is LDS scratch of blockDim/64 entries.  Returns the exclusive prefix;
// *total gets the block sum.
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t *wsum, uint32_t *total)
{
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    uint32_t inc = wave_inclusive_scan(v);
    if (lane == 63)
        wsum[w] = inc;
    __syncthreads();
    if (w == 0) {
        uint32_t x = lane < nw ? wsum[lane] : 0u;
        uint32_t xi = wave_inclusive_scan(x);
        if (lane < nw)
            wsum[lane] = xi - x;
        if (lane == nw - 1)
            wsum[32] = xi;
    }
    __syncthreads();
    uint32_t r = wsum[w] + inc - v;
    *total = wsum[32];
    __syncthreads();
    return r;
}

// ---- node records ----------------------------------------------------------------

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

struct LBox {
    double lo[3], hi[3];
    uint32_t t0, t1;
};

__device__ inline void unite(double lo[3], double hi[3], uint32_t &t0, uint32_t &t1,
                             const double olo[3], const double ohi[3], uint32_t ot0, uint32_t ot1)
{
    for (int d = 0; d < 3; ++d) {
        lo[d] = fmin(lo[d], olo[d]);
        hi[d] = fmax(hi[d], ohi[d]);
    }
    t0 = t0 < ot0 ? t0 : ot0;
    t1 = t1 > ot1 ? t1 : ot1;
}

// Order-preserving map from double to uint64 (for atomic min/max).
__host__ __device__ inline uint64_t ordered_bits(double x)
{
    uint64_t u = __builtin_bit_cast(uint64_t, x);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__host__ __device__ inline double from_ordered_bits(uint64_t u)
{
    u = (u >> 63) ? (u & 0x7FFFFFFFFFFFFFFFull) : ~u;
    return __builtin_bit_cast(double, u);
}

// Step from the bound vmax * dt <= max_disp: floor(max_disp / (vmax * tick)),
// clamped to [1, max(T, 1)] ticks.
__device__ inline uint32_t heuristic_step(double vmax, double tick_s, double max_disp,
                                          uint32_t T)
{
    double d = floor(max_disp / (vmax * tick_s));
    double cap = T > 0 ? (double)T : 1.0;
    if (!(d >= 1.0))
        d = 1.0;
    if (d > cap)
        d = cap;
    return (uint32_t)d;
}

// Step network: 5 -> 64 -> 64 -> 1, parameters W1 [64][5], b1, W2 [64][64],
// b2, w3, b3 in one flat vector.
constexpr int kMlpIn = 5;
constexpr int kMlpHid = 64;
constexpr int kMlpW1 = 0;
constexpr int kMlpB1 = kMlpW1 + kMlpHid * kMlpIn;
constexpr int kMlpW2 = kMlpB1 + kMlpHid;
constexpr int kMlpB2 = kMlpW2 + kMlpHid * kMlpHid;
constexpr int kMlpW3 = kMlpB2 + kMlpHid;
constexpr int kMlpB3 = kMlpW3 + kMlpHid;
constexpr int kMlpParams = kMlpB3 + 1;   // 4609
constexpr int kMlpOuterThreads = 256;
constexpr int kMlpOuterSamples = 128;    // samples per outer-product block

// ---- launchers (each returns the launch status) -----------------------------

// boxes
// Per-object constants; with frame set, also the orbit frame's empty start
// (launch_orbit_frame then forms the frame over it).
hipError_t launch_object_setup(const cd_elements &el, double mu, double start_s, ObjConst *oc,
                               ObjSinus *os, unsigned long long *frame, hipStream_t s);
// union of the orbits' bounding boxes (ordered bits: min xyz, max xyz), over
// the start launch_object_setup wrote
hipError_t launch_orbit_frame(const ObjConst *oc, uint32_t n, unsigned long long *frame,
                              hipStream_t s);
hipError_t launch_validate(const cd_elements &el, unsigned long long *first_bad, hipStream_t s);
hipError_t launch_steps(const uint32_t *dt, uint32_t n, uint32_t T, ObjSteps *st, uint32_t *Kc,
                        unsigned long long *total, unsigned int *bad_dt, hipStream_t s);
hipError_t launch_steps_apply_offsets(ObjSteps *st, const uint32_t *box_off, uint32_t n,
                                      hipStream_t s);
hipError_t launch_dt_heuristic(const cd_elements &el, double mu, double tick_s,
                               double max_disp, uint32_t T, uint32_t *dt_out, hipStream_t s);
// rule: CD_BOX_SPEED, CD_BOX_INTERVAL_NU or CD_BOX_INTERVAL_E
// Uniform step, time-major boxes.  sorted: within each block of
// uniform_chunk(K) slabs the boxes follow the Morton order of their objects'
// positions at the block's middle (codes = that order's keys; needs out.code
// and out.frame; n <= kSegCap, or n <= kSortedMaxObjects with out.rec);
// otherwise box (i, k) at k n + i.
uint32_t uniform_chunk(uint32_t K);
hipError_t launch_boxes_uniform(const ObjConst *oc, const ObjSinus *os, uint32_t n, uint32_t K,
                                uint32_t dt, uint32_t T, double tick_s, double half_thr,
                                int precision, int rule, bool sorted, const BoxOut &out,
                                hipStream_t s);
// Block b (entries [b stride, b stride + n), es words apart): sorts ucode
// with the local ids 0..n-1 into scode / sobj, stable.  n <= kSegCap: one
// LDS sort per block; up to kBlockRuns kSegCap runs: the runs are sorted into
// rcode / robj (same entries, not overlapping ucode, scode or sobj) and
// merged by rank.
hipError_t launch_block_sort(const uint32_t *ucode, uint32_t n, uint32_t nblocks, uint64_t stride,
                             uint32_t es, uint32_t *scode, uint32_t *sobj, uint32_t *rcode,
                             uint32_t *robj, hipStream_t s);
hipError_t launch_boxes_variable(const ObjConst *oc, const ObjSinus *os, const ObjSteps *st,
                                 uint32_t n, uint32_t T, double tick_s, double half_thr,
                                 int precision, int rule, const BoxOut &out, hipStream_t s);

// scans / sorts / fills
// step network
hipError_t launch_mlp_features(const cd_elements &el, double mu, float *x, hipStream_t s);
hipError_t launch_dt_mlp(const cd_elements &el, const uint16_t *w, double mu, double tick_s,
                         double fallback_disp, uint32_t T, uint32_t *dt, float *y,
                         hipStream_t s);
hipError_t launch_mlp_forward(const float *w, const float *x, uint32_t B, float *y,
                              hipStream_t s);
// act: [4 * 64 + 1][B] (h1, dz1, h2, dz2, dy), part: [blocks][kMlpParams + 1]
hipError_t launch_mlp_grad(const float *w, const float *x, const float *target, uint32_t B,
                           float *act, float *part, float *grad, float *loss, hipStream_t s);
hipError_t launch_mlp_adam(float *w, float *m, float *v, const float *g, int64_t step,
                           float lr, float beta1, float beta2, float eps, uint16_t *w_bf16,
                           hipStream_t s);
hipError_t launch_pair_object_counts(const cd_pair *pairs, uint64_t count, uint32_t n,
                                     uint32_t *counts, hipStream_t s);
// narrow phase
hipError_t launch_first_witness(const cd_elements &el, double mu, double tick_s, uint32_t start,
                                double thr, uint32_t T, uint32_t delta, const cd_pair *pairs,
                                uint64_t count, uint32_t *witness, unsigned long long *first,
                                hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, size_t count, hipStream_t s);
hipError_t launch_stream_copy(const void *src, void *dst, uint64_t words, hipStream_t s);
// Sets the thread-local message of cd_last_error and returns code.
int set_error(int code, const char *fmt, ...);
hipError_t launch_fill_u64(unsigned long long *p, unsigned long long v, size_t count,
                           hipStream_t s);
size_t scan_ws_bytes(size_t count);
hipError_t scan_exclusive_u32(const uint32_t *in, uint32_t *out, size_t count, void *ws,
                              hipStream_t s);
size_t radix_ws_bytes(size_t count);
// Stable LSD sort of 16-byte items by the digits given by `fields`; the result
// ends in *result (one of a, b).
enum SortKind { SORT_KV = 0, SORT_REC = 1 };
struct DigitPlan {
    int npass;
    uint8_t field[16];  // KV: ignored; Rec: 0..3 = i, j, tlo, thi
    uint8_t shift[16];
};
hipError_t radix_sort16(SortKind kind, void *a, void *b, size_t count, const DigitPlan &plan,
                        void *ws, void **result, hipStream_t s);
// The same over 8-byte items (one 64-bit word each; plan.field ignored).
hipError_t radix_sort8(void *a, void *b, size_t count, const DigitPlan &plan, void *ws,
                       void **result, hipStream_t s);
// One workgroup per slab: compute the Morton codes of the slab's boxes, sort
// (code, box index) inside LDS and write 64-bit keys (slab << 32 | code) and
// box indices in sorted order.  err bit 1: a box's t0 is outside its slab.
constexpr int kSegThreads = 1024;
constexpr int kSegItems = 17;
constexpr int64_t kSegCap = (int64_t)kSegThreads * kSegItems;
// Largest object count of the sorted layout: the block sort's runs of kSegCap.
constexpr int kBlockRuns = 16;
constexpr int64_t kSortedMaxObjects = kBlockRuns * kSegCap;
static_assert(kSegCap == CD_SORTED_MAX_ARRAYS && kSortedMaxObjects == CD_SORTED_MAX_RECORDS,
              "sorted-layout limits of the header");
// Fixed-step slabs: one workgroup per slab sorts the slab's Morton codes in
// LDS, writes the sorted 64-bit keys, and writes the slab's leaf records in
// sorted order while the slab's boxes are still cached.  A leaf's skip link
// needs only the keys next to it: those of this slab come from LDS, those of
// other slabs differ in their slab bits, which alone decide the comparison.
hipError_t launch_slab_build(const BoxView &b, int box_precision, int tree_precision,
                             uint32_t nslabs, uint32_t slab_size, uint32_t N,
                             uint32_t slab_ticks, const unsigned long long *bounds,
                             uint32_t *codes_out, void *tree, unsigned int *err,
                             hipStream_t s);

// tree
hipError_t launch_bounds(const BoxView &b, int precision, uint32_t N,
                         unsigned long long *bounds /*[6]: min xyz, max xyz*/, hipStream_t s);
// The device-wide key sort's keys: slab << 32 | the code's low kKeyCodeBits
// bits (Morton codes have 30).  kv: (key, box index) items; packed (with kv
// == nullptr): one word per box, slab << (cb + ib) | code' << ib | box index
// (N <= 2^ib), code' the code's top cb bits (cb <= kKeyCodeBits: large box
// sets give up the lowest code bits, which only shape the tree, to keep
// 8-byte sort items).
constexpr uint32_t kKeyCodeBits = 30, kMinPackedCodeBits = 24;
hipError_t launch_keys(const BoxView &b, int precision, uint32_t N, uint32_t slab_ticks,
                       uint32_t max_slab, uint32_t slab_size,
                       const unsigned long long *bounds, uint32_t *morton, KV *kv,
                       unsigned int *err, hipStream_t s, uint64_t *packed = nullptr,
                       uint32_t ib = 0, uint32_t cb = kKeyCodeBits);
// Refit levels: level-k blocks hold refit_block(k) = kRefitChunk * 16^k
// leaves.  Level 0 runs one workgroup per block with LDS-resident climbing;
// higher levels climb in global memory from per-block queues.
constexpr int kRefitChunkLog = 10;
constexpr int kRefitChunk = 1 << kRefitChunkLog;
constexpr int kRefitListCap = 4096;   // queued nodes per block
constexpr int kRefitMaxLevels = 8;
constexpr int kPushLevels = 6;    // levels whose hand-offs the chunk refit stages in LDS
constexpr int kPushStage = 64;    // staged hand-offs per level and chunk
constexpr uint32_t kCross = 0x80000000u;   // parent pointer flag: parent level > 0
constexpr uint32_t kNodeMask = 0x7FFFFFFFu;
__host__ __device__ inline uint32_t refit_shift(uint32_t lev)
{
    return (uint32_t)kRefitChunkLog + 4u * lev;
}

// Tree buffer header (the first 256 bytes of cd_tree.mem).
struct TreeHeader {
    uint32_t err;            // bit 0: slab hint / horizon violated, 1: refit, 2: traversal
    uint32_t nseeds;         // overlapping sibling pairs found by the refit
    uint32_t seed_overflow;  // set when more than seed_cap(N) pairs were found
    uint32_t leaf_esc_side;  // FP64: leaf skip links in the side array (bottom-up build)
    uint32_t pad[60];
};
static_assert(sizeof(TreeHeader) == 256, "TreeHeader layout");
inline size_t seed_cap(uint64_t N) { return (size_t)(N / 4 + 4096); }
// Tree buffer layout: header | nodes (FP64: 64-byte records; FP32: 32-byte
// boxes, then 8-byte links) | kids[N - 1] (both children of each inner node)
// | seeds[seed_cap(N)] | FP64 only: leaf skip links[N] (used by the bottom-up
// build: leaf records written in place by the box build keep their code
// words where the skip link would go).
inline size_t tree_kids_offset(uint64_t N, int precision)
{
    return sizeof(TreeHeader) + (size_t)(2 * N - 1) *
                                    (precision == CD_FP64 ? 64u : 40u);
}
inline size_t tree_seeds_offset(uint64_t N, int precision)
{
    return tree_kids_offset(N, precision) + (size_t)(N > 1 ? N - 1 : 1) * 8u;
}
inline size_t tree_leaf_esc_offset(uint64_t N, int precision)
{
    return tree_seeds_offset(N, precision) + seed_cap(N) * 8u;
}

// Overlapping sibling pairs recorded while the refit forms each union: the
// seeds of the node-pair self-traversal.  Workgroups stage them in LDS and
// reserve space with one atomic per flush.
struct SeedSink {
    uint2 *items;
    uint32_t cap;
    TreeHeader *hdr;
    __device__ void put_many(const uint2 *src, uint32_t n, uint32_t base) const
    {
        for (uint32_t k = 0; k < n; ++k)
            if (base + k < cap)
                items[base + k] = src[k];
    }
    __device__ uint32_t reserve(uint32_t n) const
    {
        uint32_t base = atomicAdd(&hdr->nseeds, n);
        if (base + n > cap)
            atomicOr(&hdr->seed_overflow, 1u);
        return base;
    }
};
constexpr int kSeedStage = 256;  // LDS-staged seeds per workgroup before a flush

// Per-workgroup seed staging: lanes append to LDS; a full stage or the end of
// the kernel flushes it with one global atomic.
struct SeedStage {
    uint2 *buf;            // LDS, kSeedStage entries
    unsigned int *n;       // LDS counter
    __device__ void push(const SeedSink &sink, uint32_t a, uint32_t b) const
    {
        unsigned int k = atomicAdd(n, 1u);
        if (k < (unsigned)kSeedStage) {
            buf[k] = make_uint2(a, b);
        } else {  // stage full: this one goes straight out
            uint2 one = make_uint2(a, b);
            sink.put_many(&one, 1, sink.reserve(1));
        }
    }
    // all threads of the block call this after the last push
    __device__ void flush(const SeedSink &sink, unsigned int *base_lds) const
    {
        __syncthreads();
        uint32_t m = *n < (unsigned)kSeedStage ? *n : (unsigned)kSeedStage;
        if (threadIdx.x == 0)
            *base_lds = m ? sink.reserve(m) : 0u;
        __syncthreads();
        for (uint32_t k = threadIdx.x; k < m; k += blockDim.x)
            if (*base_lds + k < sink.cap)
                sink.items[*base_lds + k] = buf[k];
    }
};

constexpr int kRefitLevelThreads = 256;  // queue levels (measured: 64, 128, 256, 512, 1024)

struct RefitLists {
    uint32_t *items;            // [slots][kRefitListCap]
    uint32_t *count;            // [slots]
    uint32_t base[kRefitMaxLevels];  // first slot of each level (levels >= 1)
    // queue `node` for the level-`lev` block that holds leaf `leaf`
    __device__ bool push(uint32_t lev, uint64_t leaf, uint32_t node) const
    {
        if (lev == 0 || lev >= (uint32_t)kRefitMaxLevels)
            return false;
        uint32_t slot = base[lev] + (uint32_t)(leaf >> refit_shift(lev));
        unsigned int k = atomicAdd(&count[slot], 1u);
        if (k >= (unsigned)kRefitListCap)
            return false;
        items[(size_t)slot * kRefitListCap + k] = node;
        return true;
    }
};
uint32_t refit_levels(uint32_t N);
size_t refit_list_slots(uint32_t N, uint32_t *base);
// Top-down Karras over the slab build's output (time-major slabs of
// slab_size leaves, slab_size <= kSegCap, codes sorted in each slab); the
// leaf links are written by the slab build.  N == 1: the leaf alone.
hipError_t launch_karras_slabs(const uint32_t *codes, uint32_t N, uint32_t slab_size, uint2 *kids,
                               const LinkSink &links, uint32_t *parent, uint8_t *clev,
                               hipStream_t s);
// Hierarchy and inner boxes in one bottom-up pass (k_agglo.hip) over FP64
// leaf records already in place in key order (keys: slab j / slab_size above
// code[j]): inner records, child pairs, leaf skip links (leaf_esc, one per
// leaf), refit seeds; the leaves' slabs (t0 / slab_ticks) and the key order
// are checked (error bit 1).  ws: agglo_ws_bytes(N).
size_t agglo_ws_bytes(uint32_t N);
hipError_t launch_agglo(const uint32_t *code, uint32_t slab_size, uint32_t slab_ticks,
                        uint32_t N, void *nodes, uint2 *kids, uint32_t *leaf_esc, void *ws,
                        const SeedSink &seeds, unsigned int *err, hipStream_t s);
// Where the same pass takes its leaves when they are not records in place:
// the general key sort's N items in key order (kv: (key, box index) pairs,
// or packed: launch_keys' words of ib index and cb code bits), or box arrays already in
// key order (code set: the sorted layout, keys (j / slab_size) << 32 |
// code[j], each box checked against its slab of slab_ticks).
struct AggLeafSource {
    const KV *kv;
    const uint64_t *packed;
    uint32_t ib, cb;   // packed words: index and code bits
    const uint32_t *code;
    uint32_t slab_size, slab_ticks;
};
// Pass 1 writes each leaf's record from its box (outward-rounded for an FP32
// tree).  FP64 trees (FP64 boxes) put the leaf skip links in leaf_esc; FP32
// trees in their link records (leaf_esc unused).  Key order is checked
// (error bit 1).
hipError_t launch_agglo_gather(const AggLeafSource &src, const BoxView &bv, int box_precision,
                               int tree_precision, uint32_t N, void *nodes, uint2 *kids,
                               uint32_t *leaf_esc, void *ws, const SeedSink &seeds,
                               unsigned int *err, hipStream_t s);
// Refit of the top-down hierarchy over the leaf records the slab build wrote.
hipError_t launch_refit(int tree_precision, uint32_t N, const uint32_t *parent,
                        const uint2 *kids,
                        const LinkSink &links, const uint8_t *clev, unsigned int *arrive,
                        uint32_t *list_items, uint32_t *list_count, void *tree,
                        const SeedSink &seeds, unsigned int *err, hipStream_t s);

// Physical block b runs on XCD b % 8.  Maps it to a logical block so that each
// XCD gets one contiguous range of logical blocks (their data then shares that
// XCD's L2).  A bijection on [0, nb).
__device__ inline uint32_t xcd_block(uint32_t b, uint32_t nb)
{
    uint32_t x = b & 7u, q = nb >> 3, r = nb & 7u;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// query
hipError_t launch_traverse(const void *tree, int precision, uint32_t N, uint32_t slab_ticks,
                           Rec *out, unsigned long long capacity, unsigned long long *counter,
                           unsigned int *err, const unsigned int *run_if, uint32_t threads,
                           const unsigned int *side_on, const uint32_t *side, hipStream_t s);
// One breadth-first level of the node-pair self-traversal: every pair in
// `in` (count *n_in, at most in_cap) is expanded into the overlapping pairs of
// its children; pairs of two leaves are emitted as records, the others queued
// in `outq` (count *n_out, capacity out_cap; bit 0 of *flags on overflow,
// bit 1 on a bad node, bit 3 when *n_in is 0).  gated: return at once if any
// flag is set.
hipError_t launch_expand(const void *tree, const uint2 *kids, int precision, uint32_t N,
                         const uint2 *in, const unsigned int *n_in, uint32_t in_cap, uint2 *outq,
                         unsigned int *n_out, uint32_t out_cap, Rec *out,
                         unsigned long long capacity, unsigned long long *counter,
                         unsigned int *flags, int gated, uint32_t blocks, uint32_t threads,
                         hipStream_t s);
// Every level in one launch of a resident grid (at most `blocks` workgroups of
// 1 024 lanes), levels separated by a device-wide wait on *bar (zero before
// the launch).  Level l reads the seeds (l = 0) or the queue written by level
// l - 1 (qa for even l - 1, qb for odd), its count in qcount[l] (zero before
// the launch).  Flags as for launch_expand; bit 2 (handover to the per-leaf
// walk) also when a wait times out or the levels run out with pairs left.
hipError_t launch_expand_all(const void *tree, const uint2 *kids, int precision, uint32_t N,
                             const uint2 *seeds, const unsigned int *nseeds, uint32_t seed_cap,
                             uint2 *qa, uint2 *qb, unsigned int *qcount, uint32_t qcap,
                             uint32_t max_levels, Rec *out, unsigned long long capacity,
                             unsigned long long *counter, unsigned int *flags, unsigned int *bar,
                             uint32_t blocks, hipStream_t s);
// Executed-work counters of the traversal (built with CD_COUNTERS only):
// reset binds `visits` (n per-object counts, or NULL) and zeroes the totals;
// read copies the kCounterWords totals.  Both wait for the stream.
constexpr int kCounterWords = 6;
#ifdef CD_COUNTERS
hipError_t counters_reset(uint32_t *visits, uint32_t nobj, hipStream_t s);
hipError_t counters_read(unsigned long long *out, hipStream_t s);
#endif
// out[0..2] = low and high words of *counter, *tree_err
hipError_t launch_query_status(const unsigned long long *counter, const unsigned int *tree_err,
                               unsigned int *out, hipStream_t s);
hipError_t launch_query_begin(const TreeHeader *hdr, unsigned int *qflags, hipStream_t s);
hipError_t launch_query_decide(const unsigned int *last_count, const unsigned int *qflags,
                               unsigned long long *counter, unsigned int *walk, hipStream_t s);
hipError_t launch_pad_records(Rec *raw, const unsigned long long *counter, uint32_t cap,
                              hipStream_t s);
hipError_t launch_query_finish(const unsigned long long *counter, const unsigned int *tree_err,
                               const uint32_t *uniq, uint32_t cap, unsigned long long *count_out,
                               unsigned int *status_out, hipStream_t s);
// bulk interval refinement (items {record, first instant, last instant, 0})
hipError_t launch_refine_seed(const cd_pair *pairs, uint32_t count, uint32_t start, uint32_t T,
                              uint32_t delta, uint4 *items, hipStream_t s);
hipError_t launch_refine_level(int rule, const ObjConst *oc, const ObjSinus *os, uint32_t n,
                               const cd_pair *pairs, const uint4 *in, const unsigned int *n_in,
                               uint32_t in_cap, uint4 *outq, unsigned int *n_out,
                               uint32_t out_cap, Rec *leaves, unsigned long long leaf_cap,
                               unsigned long long *leaf_count, unsigned int *flags,
                               uint32_t delta, uint32_t min_steps, double tick_s,
                               double half_thr, uint32_t blocks, hipStream_t s);
hipError_t launch_refine_status(const unsigned long long *leaf_count, const unsigned int *flags,
                                const unsigned int *last_count, unsigned int *out, hipStream_t s);
// altitude bands (potential-collision graph); pad = sqrt(3) thr / 2
hipError_t launch_band_flags(const cd_elements &el, double pad, const cd_pair *pairs,
                             uint32_t count, uint32_t *flags, hipStream_t s);
hipError_t launch_compact_pairs(const cd_pair *pairs, const uint32_t *flags, const uint32_t *pos,
                                uint32_t count, cd_pair *out, hipStream_t s);
hipError_t launch_band_axis_keys(const cd_elements &el, KV *kv, hipStream_t s);
hipError_t launch_band_edges(const KV *sorted, uint32_t n, uint32_t p, double *edges,
                             hipStream_t s);
// out == nullptr: cnt[i] = bands met by object i; else keys (k << 32 | i) at out + off[i]
hipError_t launch_band_members(const cd_elements &el, double pad, const double *edges, uint32_t p,
                               uint32_t *cnt, const uint32_t *off, KV *out, hipStream_t s);
hipError_t launch_band_csr(const KV *sorted, uint32_t total, uint32_t p, uint32_t *members,
                           uint32_t *offsets, hipStream_t s);
hipError_t launch_gather_elements(const cd_elements &el, const uint32_t *ids, uint32_t count,
                                  double *out, hipStream_t s);
hipError_t launch_remap_records(const cd_pair *in, uint32_t count, const uint32_t *ids,
                                uint32_t nids, cd_pair *out, hipStream_t s);
// The canonical list of at most kSmallCanon records in one workgroup (LDS
// radix sort + repeat removal); *total = records written.
constexpr int kSmallCanon = 4096;
hipError_t launch_small_canon(const Rec *in, uint32_t count, Rec *out, uint32_t *total,
                              hipStream_t s);
// The same with the count still on the device: runs only if the node-pair
// levels drained (*qflags == 8), *tree_err == 0 and *counter <= min(capacity,
// kSmallCanon); then *done = records written + 1 (else *done is untouched).
hipError_t launch_small_canon_gated(const Rec *in, const unsigned long long *counter,
                                    const unsigned int *qflags, const unsigned int *tree_err,
                                    uint32_t capacity, Rec *out, unsigned int *done,
                                    hipStream_t s);
// kSmallCanon < count <= kMediumCanon: tiles sorted in LDS, merged pairwise,
// then repeats removed (launch_unique; total at pos[count]).  a holds the
// records and is overwritten; b is scratch of count records.  Up to 2^18
// records six merge passes cost less than the radix path's ten digit passes
// (three launches each): 69 589 records took 0.72 ms by radix.
constexpr int kMediumCanon = 1 << 18;
// A record count read on the device when the kernels run, for lists
// enqueued before the host knows it: valid when the node-pair levels drained
// (*qflags == 8), the tree has no error bits and lo < count <= hi; the
// kernels then use it (the host's count, an upper bound, sizes their grids)
// and do nothing otherwise.  counter == nullptr: the host's count.
struct DevCount {
    const unsigned long long *counter;
    const unsigned int *qflags, *tree_err;
    uint32_t lo, hi;
    __device__ bool get(uint32_t host, uint32_t &count) const
    {
        if (!counter) {
            count = host;
            return true;
        }
        const unsigned long long c = *counter;
        if (*qflags != 8u || *tree_err != 0u || c <= lo || c > hi)
            return false;
        count = (uint32_t)c;
        return true;
    }
};
// With g.counter set, count is the bound g.hi and the list's length + bias
// goes to *total (else to pos[count]).
hipError_t launch_medium_canon(Rec *a, Rec *b, uint32_t count, uint32_t *flags, uint32_t *pos,
                               void *scan_ws, Rec *out, hipStream_t s, const DevCount &g = {},
                               unsigned int *total = nullptr, uint32_t bias = 0);
hipError_t launch_unique(const Rec *in, uint32_t count, uint32_t *flags, uint32_t *pos,
                         void *scan_ws, Rec *out, hipStream_t s, const DevCount &g = {},
                         unsigned int *total = nullptr, uint32_t bias = 0);

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Bump allocator over a caller workspace.
struct Carve {
    char *base;
    size_t size, off;
    explicit Carve(void *p, size_t n) : base((char *)p), size(n), off(0) {}
    template <typename T>
    T *take(size_t count)
    {
        off = align_up(off, 256);
        T *p = (T *)(base ? base + off : nullptr);
        off += count * sizeof(T);
        return p;
    }
    void *take_bytes(size_t bytes)
    {
        off = align_up(off, 256);
        void *p = base ? base + off : nullptr;
        off += bytes;
        return p;
    }
    bool fits() const { return off <= size; }
};

inline size_t tree_node_bytes(int precision)
{
    return precision == CD_FP64 ? sizeof(Node64) : sizeof(Box32) + sizeof(Link);
}

} // namespace cd
