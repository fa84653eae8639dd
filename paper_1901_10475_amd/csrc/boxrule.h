// boxrule.h -- the occ-int of one object over one interval under each box
// rule (Def. Interval Occupancy Region; the interval rules of Sec. 4.5),
// shared by the box kernels and the bulk interval refinement.
//
// CD_BOX_SPEED: the hull of the two endpoint positions grown by vmax * span / 2
// and the radius.  CD_BOX_INTERVAL_NU: the orbit equation and the perifocal
// axes evaluated in outward-rounded interval arithmetic over [nu_a, nu_b].
// CD_BOX_INTERVAL_E: the exact range of each coordinate written as one
// sinusoid of the eccentric anomaly over [E_a, E_b].
#pragma once
#include "cd_internal.h"
#include "interval.h"

namespace cd {

// Kepler solution at an interval endpoint.
struct EndPt {
    double M, E, sE, cE;
};

// Bounds of object c (sinusoid constants os[i]) over the interval between the
// Kepler solutions A and B (positions pa, pb; span_s seconds apart) under the
// box rule RULE, the radius half_thr included.
template <int RULE>
__device__ inline void box_bounds(const ObjConst &c, const ObjSinus *os, uint32_t i,
                                  const EndPt &A, const EndPt &B, const double pa[3],
                                  const double pb[3], double span_s, double half_thr,
                                  double lo[3], double hi[3])
{
    if (RULE == CD_BOX_SPEED) {
        double g = c.vmax * span_s * 0.5 + half_thr;
        for (int d = 0; d < 3; ++d) {
            lo[d] = fmin(pa[d], pb[d]) - g;
            hi[d] = fmax(pa[d], pb[d]) + g;
        }
        return;
    }
    const double w = 1e-10;                       // rad, for the endpoint solves' rounding
    const double eps4 = 4.0 * 2.220446049250313e-16;
    bool full = B.M - A.M >= kTwoPi;
    Iv pos[3];
    if (RULE == CD_BOX_INTERVAL_NU) {
        // nu = E + 2 atan(beta sin E / (1 - beta cos E)), beta = e / (1 + sqrt(1 - e^2)):
        // continuous in E, so unwrapped E gives unwrapped nu
        double beta = c.e * c.a / (c.a + c.b);
        double nua = A.E + 2.0 * atan(beta * A.sE / (1.0 - beta * A.cE));
        double nub = B.E + 2.0 * atan(beta * B.sE / (1.0 - beta * B.cE));
        Iv x = full ? iv(0.0, kTwoPi) : iv(nua - w, fmax(nua, nub) + w);
        Iv C = iv_cos(x), S = iv_sin(x);
        Iv one = iv(1.0, 1.0), ee = iv(c.e, c.e);
        Iv r = (iv(c.a, c.a) * (one - ee * ee)) / (one + ee * C);
        Iv X = r * C, Y = r * S;
        for (int d = 0; d < 3; ++d)
            pos[d] = X * iv_around(c.P[d], eps4) + Y * iv_around(c.Q[d], eps4);
    } else {
        // The exact range of ctr_d + R_d cos(E - phi_d) over [E_a - w, E_b + w]:
        // between its critical points the function is monotone, so the range
        // is the two end values -- the endpoint positions, already computed --
        // extended to ctr_d + R_d (E - phi_d an even multiple of pi) or
        // ctr_d - R_d (an odd one) when such a point lies inside; the
        // widening w moves an end value by at most w R_d.
        const ObjSinus &s = os[i];
        double elo = A.E - w, ehi = fmax(A.E, B.E) + w;
        for (int d = 0; d < 3; ++d) {
            double vmin = fmin(pa[d], pb[d]), vmax = fmax(pa[d], pb[d]);
            double top = s.ctr[d] + s.R[d], bot = s.ctr[d] - s.R[d];
            if (full) {
                vmin = bot;
                vmax = top;
            } else {
                double k0 = ceil((elo - s.phi[d]) * kInvPi - 1e-12);
                double k1 = floor((ehi - s.phi[d]) * kInvPi + 1e-12);
                if (k0 <= k1) {
                    if ((((long long)k0) & 1) == 0)
                        vmax = top;
                    else
                        vmin = bot;
                    if (k0 + 1.0 <= k1) {
                        vmin = bot;
                        vmax = top;
                    }
                }
            }
            // range widening plus the rounding of positions and constants
            double pad = w * s.R[d] + 16.0 * 2.220446049250313e-16 * c.a;
            pos[d] = Iv{vmin - pad, vmax + pad};
        }
    }
    for (int d = 0; d < 3; ++d) {
        lo[d] = iv_dn(pos[d].lo - half_thr);
        hi[d] = iv_up(pos[d].hi + half_thr);
    }
}

} // namespace cd
