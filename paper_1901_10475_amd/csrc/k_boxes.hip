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
// One thread owns one object and a run of consecutive intervals, so each new
// endpoint's Newton solve starts from the previous one (1-3 iterations) and
// each endpoint is solved once.  With a uniform step the boxes are written
// time-major (box k * n + i), so the lanes of a wave store consecutive boxes.
#include "cd_internal.h"
#include "orbit.h"

namespace cd {

// m0 is advanced to the horizon's start: M(start + t) = m0 + n (start + t).
__global__ void k_object_setup(cd_elements el, double mu, double start_s, ObjConst *oc)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= el.n)
        return;
    oc[i] = object_const(el.a[i], el.e[i], el.inc[i], el.raan[i], el.argp[i], el.m0[i], mu,
                         start_s);
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
            if (o.code) {
                mn[d] = from_ordered_bits(o.frame[d]);
                double ext = from_ordered_bits(o.frame[3 + d]) - mn[d];
                inv[d] = ext > 0.0 ? 1.0 / ext : 0.0;
            }
        }
    }
};

template <int PREC>
__device__ inline void store_box(const BoxOut &o, const CodeFrame &f, uint64_t b,
                                 const double pa[3], const double pb[3], double g, uint32_t t0,
                                 uint32_t t1, uint32_t obj)
{
    if (b >= o.cap)
        return;
    if (o.code)
        o.code[b] = morton30(0.5 * (pa[0] + pb[0]), 0.5 * (pa[1] + pb[1]),
                             0.5 * (pa[2] + pb[2]), f.mn, f.inv);
    for (int d = 0; d < 3; ++d) {
        double lo = fmin(pa[d], pb[d]) - g;
        double hi = fmax(pa[d], pb[d]) + g;
        if (PREC == CD_FP64) {
            ((double *)o.lo[d])[b] = lo;
            ((double *)o.hi[d])[b] = hi;
        } else {
            ((float *)o.lo[d])[b] = __double2float_rd(lo);
            ((float *)o.hi[d])[b] = __double2float_ru(hi);
        }
    }
    o.t0[b] = t0;
    o.t1[b] = t1;
    o.obj[b] = obj;
}

// Intervals [k0, k1) of object i; box of interval k at index base + k * stride.
template <int PREC>
__device__ inline void object_run(const ObjConst &c, uint32_t i, uint64_t k0, uint64_t k1,
                                  uint64_t K, uint64_t dt, uint64_t T, double tick_s,
                                  double half_thr, const BoxOut &out, uint64_t base,
                                  uint64_t stride)
{
    const CodeFrame f(out);
    uint64_t ta = k0 * dt < T ? k0 * dt : T;
    double M = c.m0 + c.n * ((double)ta * tick_s);
    double E = M + c.e * sin(M), sE, cE;
    kepler(M, c.e, E, sE, cE);
    double pa[3];
    position(c, sE, cE, pa);
    for (uint64_t k = k0; k < k1; ++k) {
        uint64_t tb = (k + 1) * dt < T ? (k + 1) * dt : T;
        double Mb = c.m0 + c.n * ((double)tb * tick_s);
        E += (Mb - M) / (1.0 - c.e * cE);
        kepler(Mb, c.e, E, sE, cE);
        double pb[3];
        position(c, sE, cE, pb);
        double g = c.vmax * ((double)(tb - ta) * tick_s) * 0.5 + half_thr;
        uint32_t t1 = (k + 1 == K) ? (uint32_t)(T + 1) : (uint32_t)tb;
        store_box<PREC>(out, f, base + k * stride, pa, pb, g, (uint32_t)ta, t1, i);
        pa[0] = pb[0];
        pa[1] = pb[1];
        pa[2] = pb[2];
        ta = tb;
        M = Mb;
    }
}

template <int PREC>
__global__ void k_boxes_uniform(const ObjConst *__restrict__ oc, uint32_t n, uint32_t K,
                                uint32_t dt, uint32_t T, double tick_s, double half_thr,
                                uint32_t chunk, BoxOut out)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    uint64_t k0 = (uint64_t)blockIdx.y * chunk;
    if (k0 >= K)
        return;
    uint64_t k1 = k0 + chunk < K ? k0 + chunk : K;
    object_run<PREC>(oc[i], i, k0, k1, K, dt, T, tick_s, half_thr, out, i, n);
}

// Per-object steps, object-major output (box off_i + k).  One lane per box, so
// consecutive lanes store consecutive boxes.  Each lane solves Kepler's
// equation for the start of its interval; the end of the interval is the next
// box's start, taken from the next lane by a shuffle (a second solve only for
// the last box of a wave or of an object).
template <int PREC>
__global__ __launch_bounds__(256) void k_boxes_variable(const ObjConst *__restrict__ oc,
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
    double Ma = c.m0 + c.n * ((double)ta * tick_s);
    double E = Ma + c.e * sin(Ma), sE, cE;
    kepler(Ma, c.e, E, sE, cE);
    double pa[3];
    position(c, sE, cE, pa);
    // the next lane holds the start of this box's end, if it is the same object
    int lane = threadIdx.x & 63;
    double nx = __shfl_down(pa[0], 1, 64), ny = __shfl_down(pa[1], 1, 64),
           nz = __shfl_down(pa[2], 1, 64);
    uint32_t ni = __shfl_down(i, 1, 64);
    uint64_t nk = __shfl_down(k, 1, 64);
    double pb[3];
    if (lane < 63 && ni == i && nk == k + 1 && k + 1 < s.K) {
        pb[0] = nx;
        pb[1] = ny;
        pb[2] = nz;
    } else {
        double Mb = c.m0 + c.n * ((double)tb * tick_s);
        E += (Mb - Ma) / (1.0 - c.e * cE);
        kepler(Mb, c.e, E, sE, cE);
        position(c, sE, cE, pb);
    }
    if (!active)
        return;
    double g = c.vmax * ((double)(tb - ta) * tick_s) * 0.5 + half_thr;
    uint32_t t1 = (k + 1 == s.K) ? (uint32_t)(T + 1) : (uint32_t)tb;
    const CodeFrame f(out);
    store_box<PREC>(out, f, b, pa, pb, g, (uint32_t)ta, t1, i);
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

hipError_t launch_object_setup(const cd_elements &el, double mu, double start_s, ObjConst *oc,
                               hipStream_t s)
{
    if (el.n == 0)
        return hipSuccess;
    k_object_setup<<<blocks_for(el.n, 256), 256, 0, s>>>(el, mu, start_s, oc);
    return hipGetLastError();
}

hipError_t launch_orbit_frame(const ObjConst *oc, uint32_t n, unsigned long long *frame,
                              hipStream_t s)
{
    hipError_t e = launch_fill_u64(frame, ~0ull, 3, s);
    if (e == hipSuccess)
        e = launch_fill_u64(frame + 3, 0ull, 3, s);
    if (e != hipSuccess || n == 0)
        return e;
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

hipError_t launch_boxes_uniform(const ObjConst *oc, uint32_t n, uint32_t K, uint32_t dt,
                                uint32_t T, double tick_s, double half_thr, int precision,
                                const BoxOut &out, hipStream_t s)
{
    if (n == 0 || K == 0)
        return hipSuccess;
    uint32_t chunk = 16;
    while ((K + chunk - 1) / chunk > 65535u)
        chunk *= 2;
    dim3 grid(blocks_for(n, 128), (K + chunk - 1) / chunk);
    if (precision == CD_FP64)
        k_boxes_uniform<CD_FP64><<<grid, 128, 0, s>>>(oc, n, K, dt, T, tick_s, half_thr, chunk,
                                                       out);
    else
        k_boxes_uniform<CD_FP32><<<grid, 128, 0, s>>>(oc, n, K, dt, T, tick_s, half_thr, chunk,
                                                       out);
    return hipGetLastError();
}

hipError_t launch_boxes_variable(const ObjConst *oc, const ObjSteps *st, uint32_t n, uint32_t T,
                                 double tick_s, double half_thr, int precision, const BoxOut &out,
                                 hipStream_t s)
{
    if (n == 0 || out.cap == 0)
        return hipSuccess;
    if (precision == CD_FP64)
        k_boxes_variable<CD_FP64><<<blocks_for(out.cap, 256), 256, 0, s>>>(oc, st, n, T, tick_s,
                                                                         half_thr, out);
    else
        k_boxes_variable<CD_FP32><<<blocks_for(out.cap, 256), 256, 0, s>>>(oc, st, n, T, tick_s,
                                                                         half_thr, out);
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
