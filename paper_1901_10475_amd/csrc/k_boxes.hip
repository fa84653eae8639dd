// k_boxes.hip -- object setup, per-object steps and 4D box construction.
//
// Box (i, k) is the 4D occupancy region of object i over interval k
// (Def. Interval Occupancy Region, Def. 4D Occupancy Region): the hull of the
// two endpoint positions, grown by vmax * dt / 2 (no point of a path whose
// speed is at most vmax can stray further from both endpoints) and by the
// radius thr / 2; the tag is the half-open tick interval, the last one closed
// at T (advanceTime's clamp).  Positions come from Kepler's equation, the exact
// solution of Eq. (nu-dot), mapped to ECI by three rotations (Sec. 7.1).
//
// The alternative boxes of Sec. 4.5 evaluate the map from one orbit variable
// to ECI in interval arithmetic over the variable's range between the two
// endpoints: the true anomaly (the variable Sec. 7.1 names), or the eccentric
// anomaly with each coordinate written as one sinusoid (the variable occurs
// once, so the box is the hull of the path).  Both variables grow with time,
// so their range over an interval lies between the endpoint values, which the
// Kepler solve already has.  The true-anomaly box runs the interval
// operations; the eccentric-anomaly box is that exact range, which needs no
// trigonometry beyond the solve: the endpoint positions, extended to a
// sinusoid's extreme where the interval crosses it.
//
// One thread owns one object and a run of consecutive intervals, so each new
// endpoint's Newton solve starts from the previous one (1-3 iterations) and
// each endpoint is solved once.  With a uniform step the boxes are written
// time-major (box k * n + i), so the lanes of a wave store consecutive boxes.
#include <type_traits>

#include "boxrule.h"
#include "cd_internal.h"
#include "interval.h"
#include "orbit.h"

namespace cd {

// m0 is advanced to the horizon's start: M(start + t) = m0 + n (start + t).
// x_d(E) = a (cos E - e) P_d + b sin E Q_d = -a e P_d + R_d cos(E - phi_d) with
// R_d cos phi_d = a P_d and R_d sin phi_d = b Q_d.
__global__ void k_object_setup(cd_elements el, double mu, double start_s, ObjConst *oc,
                               ObjSinus *os, unsigned long long *frame)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (frame && i < 6)   // the orbit frame's start: empty (min at the top, max at 0)
        frame[i] = i < 3 ? ~0ull : 0ull;
    if (i >= el.n)
        return;
    ObjConst c = object_const(el.a[i], el.e[i], el.inc[i], el.raan[i], el.argp[i], el.m0[i], mu,
                              start_s);
    oc[i] = c;
    ObjSinus w;
    for (int d = 0; d < 3; ++d) {
        double A = c.a * c.P[d], B = c.b * c.Q[d];
        w.R[d] = sqrt(A * A + B * B);
        w.phi[d] = atan2(B, A);
        w.ctr[d] = -c.a * c.e * c.P[d];
    }
    os[i] = w;
}

// Union of the orbits' bounding boxes: on the ellipse,
// x_d(E) = -a e P_d + a P_d cos E + b Q_d sin E, so x_d spans
// -a e P_d +- sqrt((a P_d)^2 + (b Q_d)^2).  Every box centre (the midpoint of
// two orbit points) lies inside it, so Morton codes in this frame never clamp.
__global__ void k_orbit_frame(const ObjConst *oc, uint32_t n, unsigned long long *frame)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long mn[3] = {~0ull, ~0ull, ~0ull}, mx[3] = {0ull, 0ull, 0ull};
    if (i < n) {
        ObjConst c = oc[i];
        for (int d = 0; d < 3; ++d) {
            double ctr = -c.a * c.e * c.P[d];
            double w = sqrt(c.a * c.P[d] * c.a * c.P[d] + c.b * c.Q[d] * c.b * c.Q[d]);
            mn[d] = ordered_bits(ctr - w);
            mx[d] = ordered_bits(ctr + w);
        }
    }
    for (int d = 0; d < 3; ++d)
        for (int o = 32; o >= 1; o >>= 1) {
            unsigned long long a = __shfl_xor(mn[d], o, 64), b = __shfl_xor(mx[d], o, 64);
            mn[d] = a < mn[d] ? a : mn[d];
            mx[d] = b > mx[d] ? b : mx[d];
        }
    if ((threadIdx.x & 63) == 0)
        for (int d = 0; d < 3; ++d) {
            atomicMin(&frame[d], mn[d]);
            atomicMax(&frame[3 + d], mx[d]);
        }
}

__global__ void k_validate(cd_elements el, unsigned long long *first_bad)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= el.n)
        return;
    double v[6] = {el.a[i], el.e[i], el.inc[i], el.raan[i], el.argp[i], el.m0[i]};
    bool ok = true;
    for (int k = 0; k < 6; ++k)
        ok = ok && isfinite(v[k]);
    ok = ok && v[0] > 0.0 && v[1] >= 0.0 && v[1] < 1.0;
    if (!ok)
        atomicMin(first_bad, (unsigned long long)i);
}

// K_i = max(1, ceil(T / dt_i)) of each object and their total.
__global__ void k_steps(const uint32_t *dt, uint32_t n, uint32_t T, ObjSteps *st, uint32_t *Kc,
                        unsigned long long *total, unsigned int *bad_dt)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    uint32_t d = dt[i];
    if (d == 0) {
        atomicOr(bad_dt, 1u);
        d = 1;
    }
    uint64_t K = T == 0 ? 1 : ((uint64_t)T + d - 1) / d;
    ObjSteps s;
    s.dt = d;
    s.K = (uint32_t)(K > 0xFFFFFFFFull ? 0xFFFFFFFFull : K);
    s.box_off = 0;
    st[i] = s;
    Kc[i] = s.K;
    atomicAdd(total, (unsigned long long)K);
}

__global__ void k_dt_heuristic(cd_elements el, double mu, double tick_s, double max_disp,
                               uint32_t T, uint32_t *dt_out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= el.n)
        return;
    double a = el.a[i], e = el.e[i];
    double vmax = sqrt(mu * (1.0 + e) / (a * (1.0 - e)));
    dt_out[i] = heuristic_step(vmax, tick_s, max_disp, T);
}

// Morton frame of the box codes (decoded once per thread).
struct CodeFrame {
    double mn[3], inv[3];
    __device__ explicit CodeFrame(const BoxOut &o)
    {
        for (int d = 0; d < 3; ++d) {
            mn[d] = inv[d] = 0.0;
            if (o.code || o.rec) {
                mn[d] = from_ordered_bits(o.frame[d]);
                double ext = from_ordered_bits(o.frame[3 + d]) - mn[d];
                inv[d] = ext > 0.0 ? 1.0 / ext : 0.0;
            }
        }
    }
};

// A box's Morton code is that of its centre, unless the caller fixes it
// (kNoCode: compute it).
constexpr int64_t kNoCode = -1;

template <int PREC>
__device__ inline void store_box(const BoxOut &o, const CodeFrame &f, uint64_t b,
                                 const double pa[3], const double pb[3], const double blo[3],
                                 const double bhi[3], uint32_t t0, uint32_t t1, uint32_t obj,
                                 int64_t code)
{
    if (b >= o.cap)
        return;

    // Non-temporal stores: consecutive lanes write consecutive boxes, so each
    // store instruction fills whole cache lines of one array, and the boxes
    // are read again only by the tree build, long after they would have left
    // the caches (0.94 -> 0.78 ms for the 60.65 M boxes of the tracked hour).
    if (o.code)
        __builtin_nontemporal_store(
            code != kNoCode ? (uint32_t)code
                            : morton30(0.5 * (pa[0] + pb[0]), 0.5 * (pa[1] + pb[1]),
                                       0.5 * (pa[2] + pb[2]), f.mn, f.inv),
            &o.code[b]);
    for (int d = 0; d < 3; ++d) {
        double lo = blo[d];
        double hi = bhi[d];
        if (PREC == CD_FP64) {
            __builtin_nontemporal_store(lo, &((double *)o.lo[d])[b]);
            __builtin_nontemporal_store(hi, &((double *)o.hi[d])[b]);
        } else {
            __builtin_nontemporal_store(__double2float_rd(lo), &((float *)o.lo[d])[b]);
            __builtin_nontemporal_store(__double2float_ru(hi), &((float *)o.hi[d])[b]);
        }
    }
    __builtin_nontemporal_store(t0, &o.t0[b]);
    __builtin_nontemporal_store(t1, &o.t1[b]);
    __builtin_nontemporal_store(obj, &o.obj[b]);
}

// Intervals [k0, k1) of object i: each box is handed to sink(k, pa, pb, lo,
// hi, t0, t1).  Both store forms (arrays, records) run this one loop, so
// they hold the same bits.
template <int RULE, class Sink>
__device__ inline void object_steps(const ObjConst &c, const ObjSinus *os, uint32_t i,
                                    uint64_t k0, uint64_t k1, uint64_t K, uint64_t dt,
                                    uint64_t T, double tick_s, double half_thr, Sink &sink)
{
    uint64_t ta = k0 * dt < T ? k0 * dt : T;
    EndPt A;
    A.M = c.m0 + c.n * ((double)ta * tick_s);
    A.E = A.M + c.e * sin(A.M);
    kepler(A.M, c.e, A.E, A.sE, A.cE);
    double pa[3];
    position(c, A.sE, A.cE, pa);
    for (uint64_t k = k0; k < k1; ++k) {
        uint64_t tb = (k + 1) * dt < T ? (k + 1) * dt : T;
        EndPt B;
        B.M = c.m0 + c.n * ((double)tb * tick_s);
        B.E = A.E + (B.M - A.M) / (1.0 - c.e * A.cE);
        kepler(B.M, c.e, B.E, B.sE, B.cE);
        double pb[3];
        position(c, B.sE, B.cE, pb);
        double lo[3], hi[3];
        box_bounds<RULE>(c, os, i, A, B, pa, pb, (double)(tb - ta) * tick_s, half_thr, lo, hi);
        uint32_t t1 = (k + 1 == K) ? (uint32_t)(T + 1) : (uint32_t)tb;
        sink(k, pa, pb, lo, hi, (uint32_t)ta, t1);
        pa[0] = pb[0];
        pa[1] = pb[1];
        pa[2] = pb[2];
        ta = tb;
        A = B;
    }
}

// Boxes to the arrays: box of interval k at index base + k * stride, with
// Morton code `code` (kNoCode: the box centre's).
template <int PREC>
struct ArraySink {
    const BoxOut &out;
    CodeFrame f;
    uint64_t base, stride;
    uint32_t obj;
    int64_t code;
    __device__ void operator()(uint64_t k, const double pa[3], const double pb[3],
                               const double lo[3], const double hi[3], uint32_t t0,
                               uint32_t t1) const
    {
        store_box<PREC>(out, f, base + k * stride, pa, pb, lo, hi, t0, t1, obj, code);
    }
};

template <int PREC, int RULE>
__device__ inline void object_run(const ObjConst &c, const ObjSinus *os, uint32_t i,
                                  uint64_t k0, uint64_t k1, uint64_t K, uint64_t dt, uint64_t T,
                                  double tick_s, double half_thr, const BoxOut &out,
                                  uint64_t base, uint64_t stride, int64_t code)
{
    ArraySink<PREC> sink{out, CodeFrame(out), base, stride, i, code};
    object_steps<RULE>(c, os, i, k0, k1, K, dt, T, tick_s, half_thr, sink);
}

// Box records (FP64): each wave's 64 records of one interval (consecutive
// slots, 4 KB) are staged in the wave's own LDS area and written back so
// that each store instruction covers 1 KB of whole lines (non-temporal); the
// packed codes go to their array as well.  Every lane of the wave runs the
// loop (lanes past n compute object 0 and store nothing), because a record's
// pieces are stored by other lanes than the one that formed it.
struct RecordSink {
    const BoxOut &out;
    uint32_t n, r0, obj, code;
    bool valid;
    uint4 *stage;   // this wave's 64 records
    __device__ void operator()(uint64_t k, const double pa[3], const double pb[3],
                               const double lo[3], const double hi[3], uint32_t t0,
                               uint32_t t1) const
    {
        const uint32_t lane = threadIdx.x & 63;
        if (valid && out.code)
            __builtin_nontemporal_store(code, &out.code[k * n + r0 + lane]);
        uint4 *mine = stage + 4 * lane;
        mine[0] = make_uint4(__double2loint(lo[0]), __double2hiint(lo[0]), __double2loint(lo[1]),
                             __double2hiint(lo[1]));
        mine[1] = make_uint4(__double2loint(lo[2]), __double2hiint(lo[2]), __double2loint(hi[0]),
                             __double2hiint(hi[0]));
        mine[2] = make_uint4(__double2loint(hi[1]), __double2hiint(hi[1]), __double2loint(hi[2]),
                             __double2hiint(hi[2]));
        mine[3] = make_uint4(t0, t1, obj, code);
        wave_lds_sync();
        // piece q of the wave's 4 KB (record q / 4, quarter q % 4)
        typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
        u32x4 *dst = (u32x4 *)(out.rec + k * n + r0);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            uint32_t q = (uint32_t)j * 64 + lane;
            if (r0 + (q >> 2) < n) {
                uint4 v = stage[q];
                u32x4 x = {v.x, v.y, v.z, v.w};
                __builtin_nontemporal_store(x, dst + q);
            }
        }
        wave_lds_sync();
    }
};

template <int PREC, int RULE>
__global__ __launch_bounds__(128) void k_boxes_uniform(const ObjConst *__restrict__ oc,
                                                       const ObjSinus *__restrict__ os,
                                                       uint32_t n, uint32_t K, uint32_t dt,
                                                       uint32_t T, double tick_s, double half_thr,
                                                       uint32_t chunk, bool sorted,
                                                       const uint32_t *rank_code,
                                                       const uint32_t *rank_obj, uint32_t res,
                                                       BoxOut out)
{
    uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t k0 = (uint64_t)blockIdx.y * chunk;
    if (k0 >= K)
        return;
    uint64_t k1 = k0 + chunk < K ? k0 + chunk : K;
    if (PREC == CD_FP64 && out.rec) {
        // records come with the sorted layout only (the launcher checks)
        __shared__ uint4 stage_all[2 * 64 * 4];
        bool valid = r < n;
        uint32_t i = 0, code = 0;
        if (valid) {
            // rank r's object and code, as k_block_sort left them in entries
            // that only this thread rewrites (rank r of the block's slabs)
            i = rank_obj[(k0 * n + r) * res];
            code = rank_code[(k0 * n + r) * res];
            valid = i < n;   // always: k_block_sort wrote a permutation
            i = valid ? i : 0;
        }
        RecordSink sink{out, n, r - (threadIdx.x & 63), i, code, valid,
                        stage_all + 4 * 64 * (threadIdx.x >> 6)};
        object_steps<RULE>(oc[i], os, i, k0, k1, K, dt, T, tick_s, half_thr, sink);
        return;
    }
    if (r >= n)
        return;
    uint32_t i = r;
    int64_t code = kNoCode;
    if (sorted) {
        // rank r's object and code, left by k_block_sort in the obj and code
        // entries of box k0 n + r, which this thread overwrites itself
        i = rank_obj[(k0 * n + r) * res];
        code = rank_code[(k0 * n + r) * res];
        if (i >= n)   // cannot happen: k_block_sort wrote a permutation
            return;
    }
    object_run<PREC, RULE>(oc[i], os, i, k0, k1, K, dt, T, tick_s, half_thr, out, r, n, code);
}

// Morton code (in the orbit frame) of object i's position at the middle of
// block B of `chunk` slabs: the key of the block's per-object order.  Written
// to ucode[(B * chunk * n + i) * stride].
__global__ void k_block_codes(const ObjConst *__restrict__ oc, uint32_t n, uint32_t K,
                              uint32_t dt, uint32_t T, double tick_s, uint32_t chunk,
                              const unsigned long long *frame, uint32_t *ucode, uint32_t stride)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    uint64_t k0 = (uint64_t)blockIdx.y * chunk;
    if (k0 >= K)
        return;
    uint64_t k1 = k0 + chunk < K ? k0 + chunk : K;
    uint64_t ta = k0 * dt < T ? k0 * dt : T;
    uint64_t tb = k1 * dt < T ? k1 * dt : T;
    ObjConst c = oc[i];
    double M = c.m0 + c.n * (0.5 * (double)(ta + tb) * tick_s);
    double E = M + c.e * sin(M), sE, cE;
    kepler(M, c.e, E, sE, cE);
    double p[3];
    position(c, sE, cE, p);
    double mn[3], inv[3];
    for (int d = 0; d < 3; ++d) {
        mn[d] = from_ordered_bits(frame[d]);
        double ext = from_ordered_bits(frame[3 + d]) - mn[d];
        inv[d] = ext > 0.0 ? 1.0 / ext : 0.0;
    }
    ucode[(k0 * n + i) * stride] = morton30(p[0], p[1], p[2], mn, inv);
}

// Per-object steps, object-major output (box off_i + k).  One lane per box, so
// consecutive lanes store consecutive boxes.  Each lane solves Kepler's
// equation for the start of its interval; the end of the interval is the next
// box's start, taken from the next lane by a shuffle (a second solve only for
// the last box of a wave or of an object).
template <int PREC, int RULE>
__global__ __launch_bounds__(256) void k_boxes_variable(const ObjConst *__restrict__ oc,
                                                        const ObjSinus *__restrict__ os,
                                                        const ObjSteps *__restrict__ st,
                                                        uint32_t n, uint32_t T, double tick_s,
                                                        double half_thr, BoxOut out)
{
    uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool active = b < out.cap;
    // object owning box b: last i with box_off[i] <= b
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (st[mid].box_off <= b)
            lo = mid;
        else
            hi = mid;
    }
    uint32_t i = lo;
    ObjSteps s = st[i];
    uint64_t k = active ? b - s.box_off : 0;
    active = active && k < s.K;
    ObjConst c = oc[i];
    uint64_t ta = k * s.dt < T ? k * s.dt : T;
    uint64_t tb = (k + 1) * s.dt < T ? (k + 1) * s.dt : T;
    EndPt A;
    A.M = c.m0 + c.n * ((double)ta * tick_s);
    A.E = A.M + c.e * sin(A.M);
    kepler(A.M, c.e, A.E, A.sE, A.cE);
    double pa[3];
    position(c, A.sE, A.cE, pa);
    // the next lane holds the start of this box's end, if it is the same object
    int lane = threadIdx.x & 63;
    double nx = __shfl_down(pa[0], 1, 64), ny = __shfl_down(pa[1], 1, 64),
           nz = __shfl_down(pa[2], 1, 64);
    uint32_t ni = __shfl_down(i, 1, 64);
    uint64_t nk = __shfl_down(k, 1, 64);
    EndPt B;
    B.M = c.m0 + c.n * ((double)tb * tick_s);
    if (RULE != CD_BOX_SPEED) {
        B.E = __shfl_down(A.E, 1, 64);
        B.sE = __shfl_down(A.sE, 1, 64);
        B.cE = __shfl_down(A.cE, 1, 64);
    }
    double pb[3];
    if (lane < 63 && ni == i && nk == k + 1 && k + 1 < s.K) {
        pb[0] = nx;
        pb[1] = ny;
        pb[2] = nz;
    } else {
        B.E = A.E + (B.M - A.M) / (1.0 - c.e * A.cE);
        kepler(B.M, c.e, B.E, B.sE, B.cE);
        position(c, B.sE, B.cE, pb);
    }
    if (!active)
        return;
    double blo[3], bhi[3];
    box_bounds<RULE>(c, os, i, A, B, pa, pb, (double)(tb - ta) * tick_s, half_thr, blo, bhi);
    uint32_t t1 = (k + 1 == s.K) ? (uint32_t)(T + 1) : (uint32_t)tb;
    const CodeFrame f(out);
    store_box<PREC>(out, f, b, pa, pb, blo, bhi, (uint32_t)ta, t1, i, kNoCode);
}

// After the interval counts have been scanned into first-box offsets.
__global__ void k_steps_apply_offsets(ObjSteps *st, const uint32_t *box_off, uint32_t n)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    st[i].box_off = box_off[i];
}

static inline unsigned blocks_for(uint64_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

// Calls go(precision tag, rule tag) with compile-time constants; the caller
// has checked both values.
template <class F>
static void dispatch_rule(int precision, int rule, F &&go)
{
    using P64 = std::integral_constant<int, CD_FP64>;
    using P32 = std::integral_constant<int, CD_FP32>;
    using R0 = std::integral_constant<int, CD_BOX_SPEED>;
    using R1 = std::integral_constant<int, CD_BOX_INTERVAL_NU>;
    using R2 = std::integral_constant<int, CD_BOX_INTERVAL_E>;
    if (precision == CD_FP64) {
        if (rule == CD_BOX_INTERVAL_NU)
            go(P64{}, R1{});
        else if (rule == CD_BOX_INTERVAL_E)
            go(P64{}, R2{});
        else
            go(P64{}, R0{});
    } else {
        if (rule == CD_BOX_INTERVAL_NU)
            go(P32{}, R1{});
        else if (rule == CD_BOX_INTERVAL_E)
            go(P32{}, R2{});
        else
            go(P32{}, R0{});
    }
}

hipError_t launch_object_setup(const cd_elements &el, double mu, double start_s, ObjConst *oc,
                               ObjSinus *os, unsigned long long *frame, hipStream_t s)
{
    if (el.n == 0 && !frame)
        return hipSuccess;
    const uint64_t threads = el.n > 6 ? (uint64_t)el.n : 6u;
    k_object_setup<<<blocks_for(threads, 256), 256, 0, s>>>(el, mu, start_s, oc, os, frame);
    return hipGetLastError();
}

hipError_t launch_orbit_frame(const ObjConst *oc, uint32_t n, unsigned long long *frame,
                              hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    k_orbit_frame<<<blocks_for(n, 256), 256, 0, s>>>(oc, n, frame);
    return hipGetLastError();
}

hipError_t launch_validate(const cd_elements &el, unsigned long long *first_bad, hipStream_t s)
{
    hipError_t e = launch_fill_u64(first_bad, ~0ull, 1, s);
    if (e != hipSuccess || el.n == 0)
        return e;
    k_validate<<<blocks_for(el.n, 256), 256, 0, s>>>(el, first_bad);
    return hipGetLastError();
}

hipError_t launch_steps(const uint32_t *dt, uint32_t n, uint32_t T, ObjSteps *st, uint32_t *Kc,
                        unsigned long long *total, unsigned int *bad_dt, hipStream_t s)
{
    hipError_t e = launch_fill_u64(total, 0ull, 1, s);
    if (e == hipSuccess)
        e = launch_fill_u32(bad_dt, 0u, 1, s);
    if (e != hipSuccess || n == 0)
        return e;
    k_steps<<<blocks_for(n, 256), 256, 0, s>>>(dt, n, T, st, Kc, total, bad_dt);
    return hipGetLastError();
}

hipError_t launch_dt_heuristic(const cd_elements &el, double mu, double tick_s,
                               double max_disp, uint32_t T, uint32_t *dt_out, hipStream_t s)
{
    if (el.n == 0)
        return hipSuccess;
    k_dt_heuristic<<<blocks_for(el.n, 256), 256, 0, s>>>(el, mu, tick_s, max_disp, T, dt_out);
    return hipGetLastError();
}

template <int PREC, int RULE>
static void boxes_uniform(dim3 grid, hipStream_t s, const ObjConst *oc, const ObjSinus *os,
                          uint32_t n, uint32_t K, uint32_t dt, uint32_t T, double tick_s,
                          double half_thr, uint32_t chunk, bool sorted, const uint32_t *rank_code,
                          const uint32_t *rank_obj, uint32_t res, const BoxOut &out)
{
    k_boxes_uniform<PREC, RULE><<<grid, 128, 0, s>>>(oc, os, n, K, dt, T, tick_s, half_thr,
                                                     chunk, sorted, rank_code, rank_obj, res,
                                                     out);
}

uint32_t uniform_chunk(uint32_t K)
{
    // 8 consecutive intervals per thread (warm-started Kepler solves) measured
    // best: 0.73 ms for the 60.65 M boxes of the tracked hour against 0.79 ms
    // with 16 and 0.82-0.83 ms with 4 or 32
    uint32_t chunk = 8;
    while ((K + chunk - 1) / chunk > 65535u)
        chunk *= 2;
    return chunk;
}

hipError_t launch_boxes_uniform(const ObjConst *oc, const ObjSinus *os, uint32_t n, uint32_t K,
                                uint32_t dt, uint32_t T, double tick_s, double half_thr,
                                int precision, int rule, bool sorted, const BoxOut &out,
                                hipStream_t s)
{
    if (n == 0 || K == 0)
        return hipSuccess;
    uint32_t chunk = uniform_chunk(K);
    dim3 grid(blocks_for(n, 128), (K + chunk - 1) / chunk);
    if (out.rec && !sorted)
        return hipErrorInvalidValue;   // box records come in the sorted layout
    uint32_t *sc = nullptr, *so = nullptr, st = 1;
    if (sorted) {
        // per block of `chunk` slabs: objects' codes at the block's middle,
        // sorted with their ids (rank r's code and id where the box kernel
        // thread of rank r reads them before it rewrites those entries)
        if ((!out.code && !out.rec) || !out.frame || (uint64_t)n * K > out.cap)
            return hipErrorInvalidValue;
        uint32_t *u, *rc = nullptr, *ro = nullptr;
        const uint32_t runs = (uint32_t)((n + kSegCap - 1) / kSegCap);
        const uint64_t last = K - (uint64_t)(grid.y - 1) * chunk;   // slabs of the last block
        if (out.rec && out.code && last >= (runs > 1 ? 5u : 3u)) {
            // contiguous, in the code array's entries of each block's first
            // slabs: sorted codes (slab 0), sorted ids (slab 1), unsorted
            // codes by object (slab 2), the runs' codes and ids (slabs 3, 4)
            sc = out.code;
            so = out.code + n;
            u = out.code + 2 * (uint64_t)n;
            rc = out.code + 3 * (uint64_t)n;
            ro = out.code + 4 * (uint64_t)n;
            st = 1;
        } else if (out.rec) {
            // a short last block: one word per record of the block's first
            // slab (t1: unsorted, code and obj: sorted; words 0 and 1, the
            // first bound, the runs)
            uint32_t *w = (uint32_t *)out.rec;
            u = w + kRecT1;
            sc = w + kRecCode;
            so = w + kRecObj;
            rc = w;
            ro = w + 1;
            st = kRecWords;
        } else {
            if ((int64_t)n > kSegCap)
                return hipErrorInvalidValue;
            u = out.t0;
            sc = out.code;
            so = out.obj;
            st = 1;
        }
        k_block_codes<<<dim3(blocks_for(n, 256), grid.y), 256, 0, s>>>(oc, n, K, dt, T, tick_s,
                                                                        chunk, out.frame, u, st);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess)
            e = launch_block_sort(u, n, grid.y, (uint64_t)chunk * n, st, sc, so, rc, ro, s);
        if (e != hipSuccess)
            return e;
    }
    auto go = [&](auto prec, auto rl) {
        boxes_uniform<decltype(prec)::value, decltype(rl)::value>(grid, s, oc, os, n, K, dt, T,
                                                                  tick_s, half_thr, chunk, sorted,
                                                                  sc, so, st, out);
    };
    dispatch_rule(precision, rule, go);
    return hipGetLastError();
}

template <int PREC, int RULE>
static void boxes_variable(hipStream_t s, const ObjConst *oc, const ObjSinus *os,
                           const ObjSteps *st, uint32_t n, uint32_t T, double tick_s,
                           double half_thr, const BoxOut &out)
{
    k_boxes_variable<PREC, RULE><<<blocks_for(out.cap, 256), 256, 0, s>>>(oc, os, st, n, T,
                                                                         tick_s, half_thr, out);
}

hipError_t launch_boxes_variable(const ObjConst *oc, const ObjSinus *os, const ObjSteps *st,
                                 uint32_t n, uint32_t T, double tick_s, double half_thr,
                                 int precision, int rule, const BoxOut &out, hipStream_t s)
{
    if (n == 0 || out.cap == 0)
        return hipSuccess;
    auto go = [&](auto prec, auto rl) {
        boxes_variable<decltype(prec)::value, decltype(rl)::value>(s, oc, os, st, n, T, tick_s,
                                                                   half_thr, out);
    };
    dispatch_rule(precision, rule, go);
    return hipGetLastError();
}

hipError_t launch_steps_apply_offsets(ObjSteps *st, const uint32_t *box_off, uint32_t n,
                                      hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    k_steps_apply_offsets<<<blocks_for(n, 256), 256, 0, s>>>(st, box_off, n);
    return hipGetLastError();
}

} // namespace cd
