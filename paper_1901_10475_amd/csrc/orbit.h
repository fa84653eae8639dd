// orbit.h -- Kepler propagation shared by the box and narrow-phase kernels.
//
// An object's position at time t (Sec. 7.1): the mean anomaly advances
// linearly, M = m0 + n t with n = sqrt(mu / a^3); Kepler's equation
// E - e sin E = M gives the eccentric anomaly (the exact solution of the
// true-anomaly ODE, Eq. nu-dot); in the orbit's plane the position is
// (a (cos E - e), b sin E), b = a sqrt(1 - e^2), and the three rotations
// R_z(raan) R_x(i) R_z(argp) take the plane's axes to ECI (vectors P, Q).
#pragma once
#include "cd_internal.h"

namespace cd {

// Per-object constants, with m0 advanced to the horizon's start.
__device__ inline ObjConst object_const(double a, double e, double inc, double raan,
                                        double argp, double m0, double mu, double start_s)
{
    double ci, si, cO, sO, cw, sw;
    sincos(inc, &si, &ci);
    sincos(raan, &sO, &cO);
    sincos(argp, &sw, &cw);
    ObjConst c;
    c.a = a;
    c.e = e;
    c.b = a * sqrt(1.0 - e * e);
    c.n = sqrt(mu / (a * a * a));
    c.m0 = m0 + c.n * start_s;
    c.vmax = sqrt(mu * (1.0 + e) / (a * (1.0 - e)));   // perigee speed, the largest
    // R_z(raan) R_x(inc) R_z(argp) applied to the perifocal x and y axes
    c.P[0] = cO * cw - sO * sw * ci;
    c.P[1] = sO * cw + cO * sw * ci;
    c.P[2] = sw * si;
    c.Q[0] = -cO * sw - sO * cw * ci;
    c.Q[1] = -sO * sw + cO * cw * ci;
    c.Q[2] = cw * si;
    return c;
}

// Newton on Kepler's equation E - e sin E = M from the guess in E.  Returns
// sin E and cos E at the converged E (first-order corrected for the last step).
__device__ inline void kepler(double M, double e, double &E, double &sE, double &cE)
{
    for (int it = 0; it < 40; ++it) {
        sincos(E, &sE, &cE);
        double d = (E - e * sE - M) / (1.0 - e * cE);
        E -= d;
        if (fabs(d) <= 1e-15 * (1.0 + fabs(E))) {
            double s0 = sE;
            sE = sE - cE * d;
            cE = cE + s0 * d;
            return;
        }
    }
    sincos(E, &sE, &cE);
}

__device__ inline void position(const ObjConst &c, double sE, double cE, double p[3])
{
    double u = c.a * (cE - c.e);
    double v = c.b * sE;
    p[0] = u * c.P[0] + v * c.Q[0];
    p[1] = u * c.P[1] + v * c.Q[1];
    p[2] = u * c.P[2] + v * c.Q[2];
}

} // namespace cd
