// k_bands.hip -- the potential-collision graph by altitude bands.
//
// Def. Potential-Collision Graph joins two objects when a collision between
// them is possible; for orbits the paper uses perigee and apogee: every
// position lies at a distance from the Earth's centre between a(1 - e) and
// a(1 + e), and every point of an occupancy cube (radius r = thr / 2, inf-norm)
// within sqrt(3) r of its centre, so two objects whose widened radial bands
// are disjoint never collide.  The edge partition places each object in every
// altitude band that its radial band meets, the band edges being every
// (n / p)-th semi-major axis in sorted order; a possible collision lies in the
// band holding its common radius, so every edge of the graph stays inside
// some band and the bands are independent problems.
#include "cd_internal.h"

namespace cd {

__device__ inline void radial_band(double a, double e, double pad, double &lo, double &hi)
{
    lo = a * (1.0 - e) - pad;
    hi = a * (1.0 + e) + pad;
}

// flags[r] = 1 if record r's objects are band-compatible (ids out of range: 0)
__global__ void k_band_flags(const double *__restrict__ a, const double *__restrict__ e,
                             int64_t n, double pad, const cd_pair *__restrict__ pairs,
                             uint32_t count, uint32_t *__restrict__ flags)
{
    uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= count)
        return;
    cd_pair pr = pairs[r];
    uint32_t f = 0;
    if (pr.i < (uint64_t)n && pr.j < (uint64_t)n) {
        double li, hi, lj, hj;
        radial_band(a[pr.i], e[pr.i], pad, li, hi);
        radial_band(a[pr.j], e[pr.j], pad, lj, hj);
        f = (li <= hj && lj <= hi) ? 1u : 0u;
    }
    flags[r] = f;
}

// out[pos[r]] = pairs[r] where flags[r] (pos = exclusive scan of flags)
__global__ void k_compact_pairs(const cd_pair *__restrict__ pairs, const uint32_t *flags,
                                const uint32_t *pos, uint32_t count, cd_pair *__restrict__ out)
{
    uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < count && flags[r])
        out[pos[r]] = pairs[r];
}

// kv[i] = {ordered bits of a_i, i}: sorting gives the semi-major axes in order
__global__ void k_band_axis_keys(const double *__restrict__ a, uint32_t n, KV *__restrict__ kv)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    KV x;
    x.key = ordered_bits(a[i]);
    x.val = i;
    x.pad = 0;
    kv[i] = x;
}

// edges[0] = -inf, edges[p] = +inf, edges[k] = the (k d)-th smallest axis
__global__ void k_band_edges(const KV *__restrict__ sorted, uint32_t n, uint32_t p,
                             double *__restrict__ edges)
{
    uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > p)
        return;
    uint64_t d = n / p > 0 ? n / p : 1;
    double v;
    if (k == 0)
        v = -INFINITY;
    else if (k == p)
        v = INFINITY;
    else {
        uint64_t at = (uint64_t)k * d;
        v = from_ordered_bits(sorted[at < n ? at : n - 1].key);
    }
    edges[k] = v;
}

// Bands met by object i: band k holds i when lo_i < edges[k + 1] and
// hi_i >= edges[k].  emit == nullptr: cnt[i] = their number; otherwise the
// keys (k << 32 | i) are written from out[off[i]] on.
__global__ void k_band_members(const double *__restrict__ a, const double *__restrict__ e,
                               uint32_t n, double pad, const double *__restrict__ edges,
                               uint32_t p, uint32_t *__restrict__ cnt,
                               const uint32_t *__restrict__ off, KV *__restrict__ out)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    double lo, hi;
    radial_band(a[i], e[i], pad, lo, hi);
    uint32_t c = 0;
    for (uint32_t k = 0; k < p; ++k) {
        if (lo < edges[k + 1] && hi >= edges[k]) {
            if (out) {
                KV x;
                x.key = ((uint64_t)k << 32) | i;
                x.val = i;
                x.pad = 0;
                out[off[i] + c] = x;
            }
            ++c;
        }
    }
    if (!out)
        cnt[i] = c;
}

// members[m] = object id of sorted key m; offsets[k] = first key of band k
// (binary search), offsets[p] = total.
__global__ void k_band_csr(const KV *__restrict__ sorted, uint32_t total, uint32_t p,
                           uint32_t *__restrict__ members, uint32_t *__restrict__ offsets)
{
    uint32_t m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < total)
        members[m] = sorted[m].val;
    if (m <= p) {
        uint32_t lo = 0, hi = total;
        uint64_t want = (uint64_t)m << 32;
        while (lo < hi) {
            uint32_t mid = (lo + hi) >> 1;
            if (sorted[mid].key < want)
                lo = mid + 1;
            else
                hi = mid;
        }
        offsets[m] = lo;
    }
}

// out row d (a, e, inc, raan, argp, m0) at out + d * count
__global__ void k_gather_elements(cd_elements el, const uint32_t *__restrict__ ids,
                                  uint32_t count, double *__restrict__ out)
{
    uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count)
        return;
    uint32_t i = ids[k];
    if (i >= (uint64_t)el.n)
        return;
    out[k] = el.a[i];
    out[(uint64_t)count + k] = el.e[i];
    out[2ull * count + k] = el.inc[i];
    out[3ull * count + k] = el.raan[i];
    out[4ull * count + k] = el.argp[i];
    out[5ull * count + k] = el.m0[i];
}

__global__ void k_remap_records(const cd_pair *__restrict__ in, uint32_t count,
                                const uint32_t *__restrict__ ids, uint32_t nids,
                                cd_pair *__restrict__ out)
{
    uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= count)
        return;
    cd_pair pr = in[r];
    uint32_t gi = pr.i < nids ? ids[pr.i] : 0xFFFFFFFFu;
    uint32_t gj = pr.j < nids ? ids[pr.j] : 0xFFFFFFFFu;
    cd_pair o;
    o.i = gi < gj ? gi : gj;
    o.j = gi < gj ? gj : gi;
    o.t_lo = pr.t_lo;
    o.t_hi = pr.t_hi;
    out[r] = o;
}

static inline unsigned blocks_for(uint64_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

hipError_t launch_band_flags(const cd_elements &el, double pad, const cd_pair *pairs,
                             uint32_t count, uint32_t *flags, hipStream_t s)
{
    if (count == 0)
        return hipSuccess;
    k_band_flags<<<blocks_for(count, 256), 256, 0, s>>>(el.a, el.e, el.n, pad, pairs, count,
                                                        flags);
    return hipGetLastError();
}

hipError_t launch_compact_pairs(const cd_pair *pairs, const uint32_t *flags, const uint32_t *pos,
                                uint32_t count, cd_pair *out, hipStream_t s)
{
    if (count == 0)
        return hipSuccess;
    k_compact_pairs<<<blocks_for(count, 256), 256, 0, s>>>(pairs, flags, pos, count, out);
    return hipGetLastError();
}

hipError_t launch_band_axis_keys(const cd_elements &el, KV *kv, hipStream_t s)
{
    if (el.n == 0)
        return hipSuccess;
    k_band_axis_keys<<<blocks_for(el.n, 256), 256, 0, s>>>(el.a, (uint32_t)el.n, kv);
    return hipGetLastError();
}

hipError_t launch_band_edges(const KV *sorted, uint32_t n, uint32_t p, double *edges,
                             hipStream_t s)
{
    k_band_edges<<<blocks_for(p + 1, 256), 256, 0, s>>>(sorted, n, p, edges);
    return hipGetLastError();
}

hipError_t launch_band_members(const cd_elements &el, double pad, const double *edges, uint32_t p,
                               uint32_t *cnt, const uint32_t *off, KV *out, hipStream_t s)
{
    if (el.n == 0)
        return hipSuccess;
    k_band_members<<<blocks_for(el.n, 256), 256, 0, s>>>(el.a, el.e, (uint32_t)el.n, pad, edges,
                                                          p, cnt, off, out);
    return hipGetLastError();
}

hipError_t launch_band_csr(const KV *sorted, uint32_t total, uint32_t p, uint32_t *members,
                           uint32_t *offsets, hipStream_t s)
{
    uint64_t m = (uint64_t)total > (uint64_t)p + 1 ? total : (uint64_t)p + 1;
    k_band_csr<<<blocks_for(m, 256), 256, 0, s>>>(sorted, total, p, members, offsets);
    return hipGetLastError();
}

hipError_t launch_gather_elements(const cd_elements &el, const uint32_t *ids, uint32_t count,
                                  double *out, hipStream_t s)
{
    if (count == 0)
        return hipSuccess;
    k_gather_elements<<<blocks_for(count, 256), 256, 0, s>>>(el, ids, count, out);
    return hipGetLastError();
}

hipError_t launch_remap_records(const cd_pair *in, uint32_t count, const uint32_t *ids,
                                uint32_t nids, cd_pair *out, hipStream_t s)
{
    if (count == 0)
        return hipSuccess;
    k_remap_records<<<blocks_for(count, 256), 256, 0, s>>>(in, count, ids, nids, out);
    return hipGetLastError();
}

} // namespace cd
