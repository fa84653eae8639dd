// k_refine.hip -- bulk interval refinement of candidate records.
//
// Procedure resolveCollisions shortens the time interval of two objects whose
// 4D boxes meet by halving it, until the boxes separate or both intervals are
// single instants (a collision).  Here every candidate record is refined at
// once: an item is a record and a span of its instants on the delta grid
// (first and last instant, ticks relative to the horizon's start).  One launch
// per level: a lane takes an item, solves Kepler's equation for both objects
// at both ends of the span, forms both occ-int boxes under the query's box
// rule, and drops the item if they do not meet (no instant of the span can
// collide); a span of at most min_steps instants is emitted as a leaf, a
// longer one is queued as its two halves (the first taking half the steps,
// rounded down).  A box over a single instant is the occupancy cube
// (Property 1), so single-instant leaves of the speed box are exactly the
// collision instants.  Appends are aggregated per workgroup (one scan, one
// atomic per queue).
#include "boxrule.h"
#include "cd_internal.h"
#include "orbit.h"

namespace cd {

// Record r's instants: the first grid instant at or after t_lo and the last at
// or before min(t_hi - 1, T); an empty record gets first > last.
__global__ void k_refine_seed(const cd_pair *__restrict__ pairs, uint32_t count, uint32_t start,
                              uint32_t T, uint32_t delta, uint4 *__restrict__ items)
{
    uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= count)
        return;
    cd_pair pr = pairs[r];
    uint32_t a = 1, b = 0;
    if (pr.t_hi > pr.t_lo) {
        uint64_t last = (uint64_t)pr.t_hi - 1 < (uint64_t)T ? (uint64_t)pr.t_hi - 1 : T;
        if ((uint64_t)pr.t_lo <= last) {
            uint64_t u = ((uint64_t)start + pr.t_lo + delta - 1) / delta;
            uint64_t v = ((uint64_t)start + last) / delta;
            if (u <= v) {
                a = (uint32_t)(u * delta - start);
                b = (uint32_t)(v * delta - start);
            }
        }
    }
    items[r] = make_uint4(r, a, b, 0u);
}

__device__ inline void solve_at(const ObjConst &c, double t_s, EndPt &P, double p[3])
{
    P.M = c.m0 + c.n * t_s;
    P.E = P.M + c.e * sin(P.M);
    kepler(P.M, c.e, P.E, P.sE, P.cE);
    position(c, P.sE, P.cE, p);
}

template <int RULE>
__global__ __launch_bounds__(256) void k_refine_level(
    const ObjConst *__restrict__ oc, const ObjSinus *__restrict__ os, uint32_t n,
    const cd_pair *__restrict__ pairs, const uint4 *__restrict__ in, const unsigned int *n_in,
    uint32_t in_cap, uint4 *__restrict__ outq, unsigned int *n_out, uint32_t out_cap,
    Rec *__restrict__ leaves, unsigned long long leaf_cap, unsigned long long *leaf_count,
    unsigned int *flags, uint32_t delta, uint32_t min_steps, double tick_s, double half_thr)
{
    __shared__ uint32_t wsum[64];
    __shared__ unsigned int qbase;
    __shared__ unsigned long long lbase;
    if (*flags)
        return;
    uint32_t m = *n_in;
    m = m < in_cap ? m : in_cap;
    if (m == 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0)
            atomicOr(flags, 8u);
        return;
    }
    for (uint32_t base = blockIdx.x * blockDim.x; base < m; base += gridDim.x * blockDim.x) {
        uint32_t k = base + threadIdx.x;
        bool keep = false;
        uint4 it = make_uint4(0u, 1u, 0u, 0u);
        cd_pair pr;
        pr.i = pr.j = 0;
        if (k < m) {
            it = in[k];
            pr = pairs[it.x];
            if (it.y <= it.z && pr.i < n && pr.j < n) {
                double ta = (double)it.y * tick_s, tb = (double)it.z * tick_s;
                double lo_i[3], hi_i[3], lo_j[3], hi_j[3];
                {
                    const ObjConst ci = oc[pr.i];
                    EndPt A, B;
                    double pa[3], pb[3];
                    solve_at(ci, ta, A, pa);
                    solve_at(ci, tb, B, pb);
                    box_bounds<RULE>(ci, os, pr.i, A, B, pa, pb, tb - ta, half_thr, lo_i, hi_i);
                }
                {
                    const ObjConst cj = oc[pr.j];
                    EndPt A, B;
                    double pa[3], pb[3];
                    solve_at(cj, ta, A, pa);
                    solve_at(cj, tb, B, pb);
                    box_bounds<RULE>(cj, os, pr.j, A, B, pa, pb, tb - ta, half_thr, lo_j, hi_j);
                }
                keep = true;
                for (int d = 0; d < 3; ++d)
                    keep = keep && lo_i[d] <= hi_j[d] && lo_j[d] <= hi_i[d];
            }
        }
        uint32_t steps = keep ? (it.z - it.y) / delta + 1 : 0u;
        bool leaf = keep && steps <= min_steps;
        bool split = keep && !leaf;
        // one scan packs both counts: halves queued in the low 16 bits, leaves above
        uint32_t mine = (split ? 2u : 0u) | ((leaf ? 1u : 0u) << 16);
        uint32_t total;
        uint32_t pre = block_exclusive_scan(mine, wsum, &total);
        if (threadIdx.x == 0) {
            qbase = (total & 0xFFFFu) ? atomicAdd(n_out, total & 0xFFFFu) : 0u;
            lbase = (total >> 16) ? atomicAdd(leaf_count, (unsigned long long)(total >> 16))
                                  : 0ull;
        }
        __syncthreads();
        if (split) {
            uint32_t q = qbase + (pre & 0xFFFFu);
            uint32_t half = (steps - 1) / 2;   // the first half holds half + 1 instants
            uint32_t mid = it.y + half * delta;
            if (q + 1 < out_cap) {
                outq[q] = make_uint4(it.x, it.y, mid, 0u);
                outq[q + 1] = make_uint4(it.x, mid + delta, it.z, 0u);
            } else {
                atomicOr(flags, 1u);
            }
        }
        if (leaf) {
            unsigned long long l = lbase + (pre >> 16);
            if (l < leaf_cap) {
                Rec rec;
                rec.i = pr.i;
                rec.j = pr.j;
                rec.tlo = it.y;
                rec.thi = it.z + 1;
                leaves[l] = rec;
            }
        }
        __syncthreads();
    }
}

// out[0..3] = low and high words of *leaf_count, *flags, *last_count.
__global__ void k_refine_status(const unsigned long long *leaf_count, const unsigned int *flags,
                                const unsigned int *last_count, unsigned int *out)
{
    unsigned long long c = *leaf_count;
    out[0] = (unsigned int)c;
    out[1] = (unsigned int)(c >> 32);
    out[2] = *flags;
    out[3] = *last_count;
}

static inline unsigned blocks_for(uint64_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

hipError_t launch_refine_status(const unsigned long long *leaf_count, const unsigned int *flags,
                                const unsigned int *last_count, unsigned int *out, hipStream_t s)
{
    k_refine_status<<<1, 1, 0, s>>>(leaf_count, flags, last_count, out);
    return hipGetLastError();
}

hipError_t launch_refine_seed(const cd_pair *pairs, uint32_t count, uint32_t start, uint32_t T,
                              uint32_t delta, uint4 *items, hipStream_t s)
{
    if (count == 0)
        return hipSuccess;
    k_refine_seed<<<blocks_for(count, 256), 256, 0, s>>>(pairs, count, start, T, delta, items);
    return hipGetLastError();
}

hipError_t launch_refine_level(int rule, const ObjConst *oc, const ObjSinus *os, uint32_t n,
                               const cd_pair *pairs, const uint4 *in, const unsigned int *n_in,
                               uint32_t in_cap, uint4 *outq, unsigned int *n_out,
                               uint32_t out_cap, Rec *leaves, unsigned long long leaf_cap,
                               unsigned long long *leaf_count, unsigned int *flags,
                               uint32_t delta, uint32_t min_steps, double tick_s,
                               double half_thr, uint32_t blocks, hipStream_t s)
{
#define CD_REFINE_LEVEL(R)                                                                       \
    k_refine_level<R><<<blocks, 256, 0, s>>>(oc, os, n, pairs, in, n_in, in_cap, outq, n_out,    \
                                             out_cap, leaves, leaf_cap, leaf_count, flags,       \
                                             delta, min_steps, tick_s, half_thr)
    if (rule == CD_BOX_INTERVAL_NU)
        CD_REFINE_LEVEL(CD_BOX_INTERVAL_NU);
    else if (rule == CD_BOX_INTERVAL_E)
        CD_REFINE_LEVEL(CD_BOX_INTERVAL_E);
    else
        CD_REFINE_LEVEL(CD_BOX_SPEED);
#undef CD_REFINE_LEVEL
    return hipGetLastError();
}

} // namespace cd
