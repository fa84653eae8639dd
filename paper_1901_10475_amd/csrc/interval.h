// interval.h -- outward-rounded interval arithmetic for the interval-evaluation
// boxes (Sec. 4.5).
//
// Each operation rounds to nearest and then steps each bound one ulp outward
// (nextafter), so the result holds the exact value of the operation for any
// operands inside the operand intervals.  cos and sin take the end values,
// widened by 2^-50 for the library's rounding, and the extremum of every
// multiple of pi (cos) or pi/2 + multiple of pi (sin) inside the interval.
#pragma once
#include <hip/hip_runtime.h>

namespace cd {

struct Iv {
    double lo, hi;
};

__device__ inline double iv_dn(double x) { return nextafter(x, -INFINITY); }
__device__ inline double iv_up(double x) { return nextafter(x, INFINITY); }
__device__ inline Iv iv(double lo, double hi) { return Iv{lo, hi}; }
// x +- u, for a constant known to u
__device__ inline Iv iv_around(double x, double u) { return Iv{x - u, x + u}; }

__device__ inline Iv operator+(Iv a, Iv b) { return Iv{iv_dn(a.lo + b.lo), iv_up(a.hi + b.hi)}; }
__device__ inline Iv operator-(Iv a, Iv b) { return Iv{iv_dn(a.lo - b.hi), iv_up(a.hi - b.lo)}; }

__device__ inline Iv operator*(Iv a, Iv b)
{
    double p0 = a.lo * b.lo, p1 = a.lo * b.hi, p2 = a.hi * b.lo, p3 = a.hi * b.hi;
    return Iv{iv_dn(fmin(fmin(p0, p1), fmin(p2, p3))), iv_up(fmax(fmax(p0, p1), fmax(p2, p3)))};
}

// b must not contain 0
__device__ inline Iv operator/(Iv a, Iv b)
{
    double q0 = a.lo / b.lo, q1 = a.lo / b.hi, q2 = a.hi / b.lo, q3 = a.hi / b.hi;
    return Iv{iv_dn(fmin(fmin(q0, q1), fmin(q2, q3))), iv_up(fmax(fmax(q0, q1), fmax(q2, q3)))};
}

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kInvPi = 0.31830988618379067153776752674503;

// Range of cos(x + shift * pi / 2 ... ) helper: extrema of cos at k pi (shift
// 0) or of sin at pi/2 + k pi (shift 0.5); even k is the maximum 1, odd k the
// minimum -1.
__device__ inline Iv trig_range(Iv x, double va, double vb, double shift)
{
    if (!(x.hi - x.lo < kTwoPi))
        return Iv{-1.0, 1.0};
    const double u = 0x1p-50;
    double mn = fmin(va, vb) - u, mx = fmax(va, vb) + u;
    double k0 = ceil(x.lo * kInvPi - shift - 1e-12), k1 = floor(x.hi * kInvPi - shift + 1e-12);
    if (k0 <= k1) {
        if ((((long long)k0) & 1) == 0)
            mx = 1.0;
        else
            mn = -1.0;
        if (k0 + 1.0 <= k1) {
            mx = 1.0;
            mn = -1.0;
        }
    }
    return Iv{fmax(mn, -1.0), fmin(mx, 1.0)};
}

__device__ inline Iv iv_cos(Iv x) { return trig_range(x, cos(x.lo), cos(x.hi), 0.0); }
__device__ inline Iv iv_sin(Iv x) { return trig_range(x, sin(x.lo), sin(x.hi), 0.5); }

} // namespace cd
