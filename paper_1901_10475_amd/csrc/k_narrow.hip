// k_narrow.hip -- narrow phase: the first collision instant of every candidate.
//
// Alg. Brute Force tests every pair of objects at every instant 0, delta,
// 2 delta, ..., T and reports the first instant at which two occupancy cubes
// of radius thr / 2 (Def. Occupancy Region) overlap: ||p_i(t) - p_j(t)||_inf
// <= thr.  Every such (t, i, j) lies inside a record of the broad phase,
// because each box holds every position of its interval; testing only the
// records' instants therefore gives the same first collision.
//
// One lane per record walks the record's instants in order.  Each axis of
// p_i - p_j changes by at most (vmax_i + vmax_j) per second, so with the
// inf-norm distance D > thr at instant t no instant before
// t + (D - thr) / (vmax_i + vmax_j) can be a collision: the walk jumps there
// (rounded down to a tick, then up to the instant grid) and never passes a
// witness.  Far-apart stretches cost one position pair each; only the
// approach itself is sampled instant by instant.
#include "cd_internal.h"
#include "orbit.h"

namespace cd {

struct Walker {
    ObjConst c;
    double E = 0.0, M = 0.0;
    bool warm = false;
    __device__ void at(double t_s, double p[3])
    {
        double m = c.m0 + c.n * t_s;
        if (warm && fabs(m - M) < 1.0) {   // short step: extrapolate from the last E
            double sE, cE;
            sincos(E, &sE, &cE);
            E += (m - M) / (1.0 - c.e * cE);
        } else {
            E = m + c.e * sin(m);
            warm = true;
        }
        M = m;
        double sE, cE;
        kepler(m, c.e, E, sE, cE);
        position(c, sE, cE, p);
    }
};

__global__ void k_first_witness(cd_elements el, double mu, double tick_s, uint32_t start,
                                double thr, uint32_t T, uint32_t delta,
                                const cd_pair *__restrict__ pairs, uint64_t count,
                                uint32_t *__restrict__ witness, unsigned long long *first)
{
    uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= count)
        return;
    cd_pair pr = pairs[r];
    uint32_t w = kEnd;
    if (pr.i < (uint64_t)el.n && pr.j < (uint64_t)el.n && pr.t_lo < pr.t_hi) {
        double start_s = (double)start * tick_s;
        Walker a, b;
        a.c = object_const(el.a[pr.i], el.e[pr.i], el.inc[pr.i], el.raan[pr.i], el.argp[pr.i],
                           el.m0[pr.i], mu, start_s);
        b.c = object_const(el.a[pr.j], el.e[pr.j], el.inc[pr.j], el.raan[pr.j], el.argp[pr.j],
                           el.m0[pr.j], mu, start_s);
        const double vrel = (a.c.vmax + b.c.vmax) * tick_s;   // km per tick
        // instants are absolute multiples of delta; t is relative to start
        const uint64_t S = start, D = delta;
        uint64_t t = ((S + pr.t_lo + D - 1) / D) * D - S;
        uint64_t t_end = (uint64_t)pr.t_hi - 1;
        if (t_end > T)
            t_end = T;
        while (t <= t_end) {
            double pa[3], pb[3];
            a.at((double)t * tick_s, pa);
            b.at((double)t * tick_s, pb);
            double dist = fmax(fabs(pa[0] - pb[0]), fmax(fabs(pa[1] - pb[1]), fabs(pa[2] - pb[2])));
            if (dist <= thr) {
                w = (uint32_t)t;
                break;
            }
            double s = (dist - thr) / vrel;   // ticks before the cubes can touch
            uint64_t adv = 0;
            if (s >= 1.0)
                adv = s > 4.0e9 ? (uint64_t)4.0e9 : (uint64_t)floor(s * (1.0 - 1e-12));
            uint64_t nt = t + (adv > 1 ? adv : 1);
            t = ((S + nt + D - 1) / D) * D - S;   // next instant of the grid at or after nt
        }
    }
    witness[r] = w;
    if (w != kEnd && first)
        atomicMin(first, ((unsigned long long)w << 32) | (unsigned long long)r);
}

static inline unsigned blocks_for(uint64_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

hipError_t launch_first_witness(const cd_elements &el, double mu, double tick_s, uint32_t start,
                                double thr, uint32_t T, uint32_t delta, const cd_pair *pairs,
                                uint64_t count, uint32_t *witness, unsigned long long *first,
                                hipStream_t s)
{
    hipError_t e = first ? launch_fill_u64(first, ~0ull, 1, s) : hipSuccess;
    if (e != hipSuccess || count == 0)
        return e;
    k_first_witness<<<blocks_for(count, 64), 64, 0, s>>>(el, mu, tick_s, start, thr, T, delta,
                                                          pairs, count, witness, first);
    return hipGetLastError();
}

} // namespace cd
