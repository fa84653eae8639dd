/*
 * cd_oracle.c -- CPU oracle for the 4D-AABB broad phase (test infrastructure).
 *
 * THIS IS TEST INFRASTRUCTURE.  Only tests, the smoke check and the benchmark's
 * CPU-baseline leg may call it.  It is deliberately plain: no blocking, no
 * fusion, no reordering beyond what each definition states, so that it can be
 * read against the paper line by line.  OpenMP only splits the outermost loop
 * of the literal pair test; the result is sorted afterwards, so it does not
 * depend on the thread count.
 *
 * Readings of the paper this file takes (each one is listed in the design
 * notes as well):
 *   - The single-variable ODE of Eq. (nu-dot) is solved exactly through
 *     Kepler's equation instead of by Runge-Kutta; its solution nu(t) is the
 *     function g of Sec. 4.5.  The element set carries the mean anomaly at
 *     t = 0 (m0), from which nu follows.
 *   - The map of Sec. 7.1 from the orbit plane to space (rotations by the
 *     inclination, the node and the argument of perigee) is
 *     R_z(Omega) R_x(i) R_z(omega) applied to the perifocal position.
 *   - occ-int over [t_a, t_b] is the axis-aligned hull of the two endpoint
 *     positions grown by vmax*(t_b - t_a)/2 plus the radius r = thr/2, with
 *     vmax the perigee speed.  It contains every position in the interval
 *     (the speed bound) and equals occ at a single instant (Property 1).
 *     The alternative occ-int of Sec. 4.5, an interval evaluation of h over
 *     the range of the single variable (nu, or the eccentric anomaly), is
 *     or_box_interval; or_boxes takes either by its rule argument.
 *   - Time tags are half-open on the integer tick grid, [t_k, t_{k+1}); the
 *     last interval is clamped at T as advanceTime does and its tag is closed
 *     at T, stored as [t_{K-1}, T + 1).
 *   - Box comparisons are closed (<=), as the occupancy cube is closed.
 *   - A record never pairs an object with itself (queryObject excludes the
 *     queried object; the brute-force inner loop is read as j > i).
 */
#include "cd_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double OR_TWO_PI = 6.283185307179586476925286766559;
static const double OR_PI = 3.1415926535897932384626433832795;

/* ------------------------------------------------------------------------ */
/* Dynamics                                                                  */
/* ------------------------------------------------------------------------ */

/* Kepler's equation E - e sin E = M by Newton's method.  For e < 1 the
 * function is monotone; starting from M + e sin M it converges in a handful of
 * steps for the eccentricities used here. */
double or_eccentric_anomaly(double M, double e)
{
    double E = M + e * sin(M);
    for (int it = 0; it < 60; ++it) {
        double f = E - e * sin(E) - M;
        double fp = 1.0 - e * cos(E);
        double d = f / fp;
        E -= d;
        if (fabs(d) <= 1e-15 * (1.0 + fabs(E)))
            break;
    }
    return E;
}

/* nu(t): the solution g of the single-variable ODE nu' = f(nu) of Eq.
 * (nu-dot).  Mean anomaly grows linearly at n = sqrt(mu / a^3); the eccentric
 * anomaly follows from Kepler's equation and the true anomaly from the
 * half-angle relation. */
double or_true_anomaly(const double el[6], double t_s, double mu)
{
    double a = el[0], e = el[1], m0 = el[5];
    double n_mean = sqrt(mu / (a * a * a));
    double M = fmod(m0 + n_mean * t_s, OR_TWO_PI);
    if (M < 0.0)
        M += OR_TWO_PI;
    double E = or_eccentric_anomaly(M, e);
    return 2.0 * atan2(sqrt(1.0 + e) * sin(0.5 * E), sqrt(1.0 - e) * cos(0.5 * E));
}

/* h(nu): the orbit equation gives the radius, the perifocal position is
 * (r cos nu, r sin nu, 0), and three rotations (by omega about z, by i about
 * x, by Omega about z) take it to the ECI frame (Sec. 7.1). */
void or_position_from_nu(const double el[6], double nu, double pos[3])
{
    double a = el[0], e = el[1], inc = el[2], raan = el[3], argp = el[4];
    double r = a * (1.0 - e * e) / (1.0 + e * cos(nu));
    double v[3] = { r * cos(nu), r * sin(nu), 0.0 };
    double w[3];
    /* R_z(omega) */
    w[0] = cos(argp) * v[0] - sin(argp) * v[1];
    w[1] = sin(argp) * v[0] + cos(argp) * v[1];
    w[2] = v[2];
    /* R_x(i) */
    v[0] = w[0];
    v[1] = cos(inc) * w[1] - sin(inc) * w[2];
    v[2] = sin(inc) * w[1] + cos(inc) * w[2];
    /* R_z(Omega) */
    pos[0] = cos(raan) * v[0] - sin(raan) * v[1];
    pos[1] = sin(raan) * v[0] + cos(raan) * v[1];
    pos[2] = v[2];
}

void or_position(const double el[6], double t_s, double mu, double pos[3])
{
    or_position_from_nu(el, or_true_anomaly(el, t_s, mu), pos);
}

/* Largest speed on a Kepler ellipse, reached at perigee (vis-viva at
 * r = a(1 - e)). */
double or_vmax(double a, double e, double mu)
{
    return sqrt(mu * (1.0 + e) / (a * (1.0 - e)));
}

/* ------------------------------------------------------------------------ */
/* Interval arithmetic (Sec. 4.5)                                            */
/* ------------------------------------------------------------------------ */

/* Every operation rounds to nearest and then moves each bound one ulp
 * outward, so the true result of the operation on any points of the operand
 * intervals lies inside the returned interval. */
static double iv_dn(double x) { return nextafter(x, -INFINITY); }
static double iv_up(double x) { return nextafter(x, INFINITY); }

or_iv or_iv_make(double lo, double hi)
{
    or_iv r = { lo, hi };
    return r;
}

or_iv or_iv_add(or_iv a, or_iv b)
{
    return or_iv_make(iv_dn(a.lo + b.lo), iv_up(a.hi + b.hi));
}

or_iv or_iv_sub(or_iv a, or_iv b)
{
    return or_iv_make(iv_dn(a.lo - b.hi), iv_up(a.hi - b.lo));
}

or_iv or_iv_mul(or_iv a, or_iv b)
{
    double p[4] = { a.lo * b.lo, a.lo * b.hi, a.hi * b.lo, a.hi * b.hi };
    double mn = p[0], mx = p[0];
    for (int k = 1; k < 4; ++k) {
        mn = fmin(mn, p[k]);
        mx = fmax(mx, p[k]);
    }
    return or_iv_make(iv_dn(mn), iv_up(mx));
}

/* b must not contain 0 */
or_iv or_iv_div(or_iv a, or_iv b)
{
    double p[4] = { a.lo / b.lo, a.lo / b.hi, a.hi / b.lo, a.hi / b.hi };
    double mn = p[0], mx = p[0];
    for (int k = 1; k < 4; ++k) {
        mn = fmin(mn, p[k]);
        mx = fmax(mx, p[k]);
    }
    return or_iv_make(iv_dn(mn), iv_up(mx));
}

/* x * x as one operation (the tight square, free of the dependency problem) */
or_iv or_iv_sqr(or_iv a)
{
    double l2 = a.lo * a.lo, h2 = a.hi * a.hi;
    if (a.lo >= 0.0)
        return or_iv_make(iv_dn(l2), iv_up(h2));
    if (a.hi <= 0.0)
        return or_iv_make(iv_dn(h2), iv_up(l2));
    return or_iv_make(0.0, iv_up(fmax(l2, h2)));
}

/* cos over [lo, hi]: the end values, widened by two ulps for the library's
 * rounding, and 1 or -1 where an even or odd multiple of pi lies inside (with
 * a relative slack of 1e-12, so an extremum at an end is never missed). */
or_iv or_iv_cos(or_iv x)
{
    if (!(x.hi - x.lo < OR_TWO_PI))
        return or_iv_make(-1.0, 1.0);
    double ca = cos(x.lo), cb = cos(x.hi);
    double mn = iv_dn(iv_dn(fmin(ca, cb))), mx = iv_up(iv_up(fmax(ca, cb)));
    double k0 = ceil(x.lo / OR_PI - 1e-12), k1 = floor(x.hi / OR_PI + 1e-12);
    for (double k = k0; k <= k1; k += 1.0) {
        if (fmod(fabs(k), 2.0) == 0.0)
            mx = 1.0;
        else
            mn = -1.0;
    }
    return or_iv_make(fmax(mn, -1.0), fmin(mx, 1.0));
}

/* sin over [lo, hi]: likewise, with the extrema at pi/2 + k pi (1 for even
 * k, -1 for odd k). */
or_iv or_iv_sin(or_iv x)
{
    if (!(x.hi - x.lo < OR_TWO_PI))
        return or_iv_make(-1.0, 1.0);
    double sa = sin(x.lo), sb = sin(x.hi);
    double mn = iv_dn(iv_dn(fmin(sa, sb))), mx = iv_up(iv_up(fmax(sa, sb)));
    double k0 = ceil(x.lo / OR_PI - 0.5 - 1e-12), k1 = floor(x.hi / OR_PI - 0.5 + 1e-12);
    for (double k = k0; k <= k1; k += 1.0) {
        if (fmod(fabs(k), 2.0) == 0.0)
            mx = 1.0;
        else
            mn = -1.0;
    }
    return or_iv_make(fmax(mn, -1.0), fmin(mx, 1.0));
}

/* Eccentric anomaly of object el at time t_s, in [0, 2 pi). */
static double or_ecc_at(const double el[6], double t_s, double mu)
{
    double a = el[0], e = el[1], m0 = el[5];
    double M = fmod(m0 + sqrt(mu / (a * a * a)) * t_s, OR_TWO_PI);
    if (M < 0.0)
        M += OR_TWO_PI;
    return or_eccentric_anomaly(M, e);
}

/* occ-int by interval evaluation (Sec. 4.5): simulate the single variable x
 * at both ends of [t_a, t_b], then evaluate h over [x(t_a), x(t_b)] in
 * interval arithmetic and add the radius thr / 2.  P and Q are the perifocal
 * axes in ECI (the three rotations of Sec. 7.1 applied to the plane's x and y
 * axes).
 *
 * var = 1: x is the true anomaly nu (the variable Sec. 7.1 names) and h is
 *   the orbit equation r = p / (1 + e cos nu), p = a (1 - e^2), followed by
 *   (r cos nu) P + (r sin nu) Q.
 * var = 2: x is the eccentric anomaly E (it too solves a single-variable ODE,
 *   E' = n / (1 - e cos E)); coordinate d of a (cos E - e) P + b sin E Q,
 *   b = a sqrt(1 - e^2), is written as the one sinusoid
 *   -a e P_d + R_d cos(E - phi_d), R_d = sqrt((a P_d)^2 + (b Q_d)^2),
 *   phi_d = atan2(b Q_d, a P_d), in which E occurs once, so the interval
 *   evaluation has no dependency overestimate.
 * Both variables increase with t, so over [t_a, t_b] x stays between its end
 * values, taken unwrapped (the forward difference mod 2 pi), and covers the
 * whole turn when the mean anomaly advances 2 pi or more.  The range is
 * widened by 1e-10 rad for the rounding of the two end solutions, each
 * coefficient of P and Q by 4 DBL_EPSILON, and R_d, phi_d and the centre
 * term by 4 ulps. */
void or_box_interval(const double el[6], double ta_s, double tb_s, double mu, double thr_km,
                     int var, double lo[3], double hi[3])
{
    double a = el[0], e = el[1], inc = el[2], raan = el[3], argp = el[4];
    double n_mean = sqrt(mu / (a * a * a));
    double dM = n_mean * (tb_s - ta_s);
    const double w = 1e-10;
    or_iv x;
    if (dM >= OR_TWO_PI) {
        x = or_iv_make(0.0, OR_TWO_PI);
    } else {
        double xa, xb, rate;
        if (var == 1) {
            xa = or_true_anomaly(el, ta_s, mu);
            xb = or_true_anomaly(el, tb_s, mu);
            rate = sqrt((1.0 + e) / ((1.0 - e) * (1.0 - e) * (1.0 - e)));   /* max dnu/dM */
        } else {
            xa = or_ecc_at(el, ta_s, mu);
            xb = or_ecc_at(el, tb_s, mu);
            rate = 1.0 / (1.0 - e);                                         /* max dE/dM */
        }
        double d = xb - xa;
        while (d < 0.0)
            d += OR_TWO_PI;
        /* an advance beyond the largest possible one is a rounding wrap of a
         * tiny step */
        if (d > dM * rate * (1.0 + 1e-9) + 1e-9)
            d = 0.0;
        x = or_iv_make(xa - w, xa + d + w);
    }
    double ci = cos(inc), si = sin(inc), cO = cos(raan), sO = sin(raan), cw = cos(argp),
           sw = sin(argp);
    double P[3] = { cO * cw - sO * sw * ci, sO * cw + cO * sw * ci, sw * si };
    double Q[3] = { -cO * sw - sO * cw * ci, -sO * sw + cO * cw * ci, cw * si };
    or_iv pos[3];
    if (var == 1) {
        or_iv C = or_iv_cos(x), S = or_iv_sin(x);
        or_iv one = or_iv_make(1.0, 1.0), ee = or_iv_make(e, e);
        or_iv p = or_iv_mul(or_iv_make(a, a), or_iv_sub(one, or_iv_sqr(ee)));
        or_iv r = or_iv_div(p, or_iv_add(one, or_iv_mul(ee, C)));
        or_iv X = or_iv_mul(r, C), Y = or_iv_mul(r, S);
        for (int d = 0; d < 3; ++d) {
            or_iv Pd = or_iv_make(P[d] - 4.0 * DBL_EPSILON, P[d] + 4.0 * DBL_EPSILON);
            or_iv Qd = or_iv_make(Q[d] - 4.0 * DBL_EPSILON, Q[d] + 4.0 * DBL_EPSILON);
            pos[d] = or_iv_add(or_iv_mul(X, Pd), or_iv_mul(Y, Qd));
        }
    } else {
        double b = a * sqrt(1.0 - e * e);
        for (int d = 0; d < 3; ++d) {
            double A = a * P[d], B = b * Q[d];
            double R = sqrt(A * A + B * B), phi = atan2(B, A), c = -a * e * P[d];
            double ur = 4.0 * DBL_EPSILON * R + 4.0 * DBL_EPSILON * a;
            double uc = 4.0 * DBL_EPSILON * a;
            or_iv arg = or_iv_sub(x, or_iv_make(phi - 4.0 * DBL_EPSILON * (1.0 + fabs(phi)),
                                                phi + 4.0 * DBL_EPSILON * (1.0 + fabs(phi))));
            pos[d] = or_iv_add(or_iv_make(c - uc, c + uc),
                               or_iv_mul(or_iv_make(R - ur, R + ur), or_iv_cos(arg)));
        }
    }
    for (int d = 0; d < 3; ++d) {
        lo[d] = iv_dn(pos[d].lo - 0.5 * thr_km);
        hi[d] = iv_up(pos[d].hi + 0.5 * thr_km);
    }
}

/* ------------------------------------------------------------------------ */
/* 4D boxes                                                                  */
/* ------------------------------------------------------------------------ */

uint64_t or_intervals(uint32_t dt, uint32_t T)
{
    if (T == 0)
        return 1;
    return ((uint64_t)T + dt - 1) / dt;
}

int64_t or_box_count(int64_t n, const uint32_t *dt, uint32_t T)
{
    int64_t N = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (dt[i] == 0)
            return -1;
        N += (int64_t)or_intervals(dt[i], T);
    }
    return N;
}

/* Each object's horizon [0, T] is cut into intervals of dt ticks, the last
 * one clamped at T (advanceTime's clamp).  Interval k spans the continuous
 * times [t_k, t_{k+1}] with t_k = min(k dt, T).  Its box is occ-int over that
 * interval (the reading in the file header) and its tag is [t_k, t_{k+1}),
 * with the last tag closed at T.  That gives the 4D occupancy region
 * occ-int x interval of Def. 4D Occupancy Region. */
int or_boxes(int64_t n, const double *el, const uint32_t *dt, uint32_t T, uint32_t start,
             double tick_s, double mu, double thr_km, int rule,
             double *lo, double *hi, uint32_t *t0, uint32_t *t1, uint32_t *obj)
{
    if (T == UINT32_MAX || rule < 0 || rule > 2)
        return -1;
    int64_t b = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (dt[i] == 0)
            return -1;
        const double *e6 = el + 6 * i;
        double vmax = or_vmax(e6[0], e6[1], mu);
        uint64_t K = or_intervals(dt[i], T);
        for (uint64_t k = 0; k < K; ++k, ++b) {
            uint64_t ta = k * dt[i] < T ? k * dt[i] : T;
            uint64_t tb = (k + 1) * dt[i] < T ? (k + 1) * dt[i] : T;
            if (rule == 1 || rule == 2) {
                or_box_interval(e6, (double)(start + ta) * tick_s,
                                (double)(start + tb) * tick_s, mu, thr_km, rule, lo + 3 * b,
                                hi + 3 * b);
            } else {
                double pa[3], pb[3];
                or_position(e6, (double)(start + ta) * tick_s, mu, pa);
                or_position(e6, (double)(start + tb) * tick_s, mu, pb);
                double g = vmax * ((double)(tb - ta) * tick_s) / 2.0 + thr_km / 2.0;
                for (int d = 0; d < 3; ++d) {
                    lo[3 * b + d] = fmin(pa[d], pb[d]) - g;
                    hi[3 * b + d] = fmax(pa[d], pb[d]) + g;
                }
            }
            t0[b] = (uint32_t)ta;
            t1[b] = (k + 1 == K) ? T + 1 : (uint32_t)tb;
            obj[b] = (uint32_t)i;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Pair sets                                                                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint32_t *v;
    int64_t n, cap;
} or_vec;

static void vec_push(or_vec *s, uint32_t i, uint32_t j, uint32_t a, uint32_t b)
{
    if (s->n == s->cap) {
        s->cap = s->cap ? 2 * s->cap : 1024;
        s->v = (uint32_t *)realloc(s->v, (size_t)s->cap * 4 * sizeof(uint32_t));
    }
    uint32_t *r = s->v + 4 * s->n++;
    r[0] = i;
    r[1] = j;
    r[2] = a;
    r[3] = b;
}

static int rec_cmp(const void *pa, const void *pb)
{
    const uint32_t *a = (const uint32_t *)pa, *b = (const uint32_t *)pb;
    for (int k = 0; k < 4; ++k) {
        if (a[k] < b[k])
            return -1;
        if (a[k] > b[k])
            return 1;
    }
    return 0;
}

/* Concatenate per-thread record lists, sort lexicographically and drop
 * repeated records: the canonical form of a pair set. */
static int64_t canonical(or_vec *parts, int nparts, uint32_t **out)
{
    int64_t total = 0;
    for (int t = 0; t < nparts; ++t)
        total += parts[t].n;
    uint32_t *all = (uint32_t *)malloc((size_t)(total > 0 ? total : 1) * 4 * sizeof(uint32_t));
    int64_t at = 0;
    for (int t = 0; t < nparts; ++t) {
        if (parts[t].n)
            memcpy(all + 4 * at, parts[t].v, (size_t)parts[t].n * 4 * sizeof(uint32_t));
        at += parts[t].n;
        free(parts[t].v);
    }
    qsort(all, (size_t)total, 4 * sizeof(uint32_t), rec_cmp);
    int64_t m = 0;
    for (int64_t r = 0; r < total; ++r)
        if (m == 0 || rec_cmp(all + 4 * (m - 1), all + 4 * r) != 0) {
            if (m != r)
                memcpy(all + 4 * m, all + 4 * r, 4 * sizeof(uint32_t));
            ++m;
        }
    *out = all;
    return m;
}

/* Two 4D boxes intersect when their time tags overlap and, on every spatial
 * axis, their closed extents overlap (Def. Collision applied to occ-4d). */
static int boxes_overlap(const double *lo, const double *hi, const uint32_t *t0,
                         const uint32_t *t1, int64_t a, int64_t b)
{
    if (!(t0[a] < t1[b] && t0[b] < t1[a]))
        return 0;
    for (int d = 0; d < 3; ++d)
        if (!(lo[3 * a + d] <= hi[3 * b + d] && lo[3 * b + d] <= hi[3 * a + d]))
            return 0;
    return 1;
}

static void emit(or_vec *s, const uint32_t *t0, const uint32_t *t1,
                 const uint32_t *obj, int64_t a, int64_t b)
{
    uint32_t i = obj[a] < obj[b] ? obj[a] : obj[b];
    uint32_t j = obj[a] < obj[b] ? obj[b] : obj[a];
    uint32_t tl = t0[a] > t0[b] ? t0[a] : t0[b];
    uint32_t th = t1[a] < t1[b] ? t1[a] : t1[b];
    vec_push(s, i, j, tl, th);
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int64_t or_pairs(int64_t N, const double *lo, const double *hi,
                 const uint32_t *t0, const uint32_t *t1, const uint32_t *obj,
                 uint32_t **out)
{
    int nt = or_num_threads();
    or_vec *parts = (or_vec *)calloc((size_t)nt, sizeof(or_vec));
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t a = 0; a < N; ++a) {
#ifdef _OPENMP
        or_vec *mine = &parts[omp_get_thread_num()];
#else
        or_vec *mine = &parts[0];
#endif
        for (int64_t b = a + 1; b < N; ++b)
            if (obj[a] != obj[b] && boxes_overlap(lo, hi, t0, t1, a, b))
                emit(mine, t0, t1, obj, a, b);
    }
    int64_t m = canonical(parts, nt, out);
    free(parts);
    return m;
}

int64_t or_pairs_of(int64_t N, const double *lo, const double *hi,
                    const uint32_t *t0, const uint32_t *t1, const uint32_t *obj,
                    int64_t ns, const int64_t *sample, uint32_t **out)
{
    int nt = or_num_threads();
    or_vec *parts = (or_vec *)calloc((size_t)nt, sizeof(or_vec));
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < N; ++b) {
#ifdef _OPENMP
        or_vec *mine = &parts[omp_get_thread_num()];
#else
        or_vec *mine = &parts[0];
#endif
        for (int64_t s = 0; s < ns; ++s) {
            int64_t a = sample[s];
            if (a != b && obj[a] != obj[b] && boxes_overlap(lo, hi, t0, t1, a, b))
                emit(mine, t0, t1, obj, a, b);
        }
    }
    int64_t m = canonical(parts, nt, out);
    free(parts);
    return m;
}

int64_t or_time_overlapping_pairs(int64_t N, const uint32_t *t0,
                                  const uint32_t *t1, const uint32_t *obj)
{
    int64_t c = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : c)
    for (int64_t a = 0; a < N; ++a)
        for (int64_t b = a + 1; b < N; ++b)
            if (obj[a] != obj[b] && t0[a] < t1[b] && t0[b] < t1[a])
                ++c;
    return c;
}

/* ---- the bucketed driver: same set, time-overlapping pairs only ---------- */

/* The pair test above fails at once for two boxes whose time tags do not
 * overlap, so leaving those pairs out cannot change the set.  The sweep
 * below visits the boxes in order of t0 (ties by index).  A box can overlap
 * in time only boxes visited before it whose t1 exceeds its t0, or boxes
 * visited after it (which find it the same way), so each overlapping pair is
 * tested once, by its later box.  The earlier boxes that may still overlap
 * form the active list, kept in a binary heap ordered by t1: before a block
 * of visits the boxes whose t1 is at most the block's first t0 leave it, and
 * they can never overlap a later box (later boxes start no earlier).
 *
 * Visits are taken in blocks of consecutive boxes (a block ends where t0
 * changes, once it holds at least OR_BLOCK_MIN boxes).  Within a block each
 * box is tested against the active list at the block's start and against the
 * boxes of the block visited before it.  With a uniform step (every box of
 * time slab k tagged [k dt, (k + 1) dt)) every slab is one block whose active
 * list is empty, so the driver is "all pairs within each slab"; with
 * per-object steps it is a sweep in t0 order over an active list in t1
 * order.  The full pair test is still applied to every tested pair. */
#define OR_BLOCK_MIN 1024

static int cmp_u64(const void *pa, const void *pb)
{
    uint64_t a = *(const uint64_t *)pa, b = *(const uint64_t *)pb;
    return a < b ? -1 : (a > b ? 1 : 0);
}

typedef struct {
    uint32_t *box; /* box indices; heap order by t1 */
    int64_t n, cap;
} or_heap;

static void heap_push(or_heap *h, const uint32_t *t1, uint32_t b)
{
    if (h->n == h->cap) {
        h->cap = h->cap ? 2 * h->cap : 1024;
        h->box = (uint32_t *)realloc(h->box, (size_t)h->cap * sizeof(uint32_t));
    }
    int64_t c = h->n++;
    h->box[c] = b;
    while (c > 0) {
        int64_t p = (c - 1) / 2;
        if (t1[h->box[p]] <= t1[h->box[c]])
            break;
        uint32_t tmp = h->box[p];
        h->box[p] = h->box[c];
        h->box[c] = tmp;
        c = p;
    }
}

static void heap_pop(or_heap *h, const uint32_t *t1)
{
    h->box[0] = h->box[--h->n];
    int64_t c = 0;
    for (;;) {
        int64_t l = 2 * c + 1, r = l + 1, m = c;
        if (l < h->n && t1[h->box[l]] < t1[h->box[m]])
            m = l;
        if (r < h->n && t1[h->box[r]] < t1[h->box[m]])
            m = r;
        if (m == c)
            break;
        uint32_t tmp = h->box[m];
        h->box[m] = h->box[c];
        h->box[c] = tmp;
        c = m;
    }
}

/* One box, copied into visiting order so that the tests of a block read
 * consecutive memory. */
typedef struct {
    double lo[3], hi[3];
    uint32_t t0, t1, obj, pad;
} or_box;

/* The test of boxes_overlap plus the different-object condition, on copies.
 * The conditions are taken in the order that rejects most pairs soonest
 * (first axis, then time, object, other axes); they are all required, so the
 * order does not change the result. */
static void test_and_emit(or_vec *out, const or_box *a, const or_box *b)
{
    if (!(a->lo[0] <= b->hi[0] && b->lo[0] <= a->hi[0]))
        return;
    if (!(a->t0 < b->t1 && b->t0 < a->t1) || a->obj == b->obj)
        return;
    for (int d = 1; d < 3; ++d)
        if (!(a->lo[d] <= b->hi[d] && b->lo[d] <= a->hi[d]))
            return;
    vec_push(out, a->obj < b->obj ? a->obj : b->obj, a->obj < b->obj ? b->obj : a->obj,
             a->t0 > b->t0 ? a->t0 : b->t0, a->t1 < b->t1 ? a->t1 : b->t1);
}

int64_t or_pairs_bucketed(int64_t N, const double *lo, const double *hi,
                          const uint32_t *t0, const uint32_t *t1, const uint32_t *obj,
                          uint32_t **out)
{
    int nt = or_num_threads();
    or_vec *parts = (or_vec *)calloc((size_t)nt, sizeof(or_vec));
    /* visiting order: (t0, index) ascending */
    uint64_t *order = (uint64_t *)malloc((size_t)(N > 0 ? N : 1) * sizeof(uint64_t));
    for (int64_t b = 0; b < N; ++b)
        order[b] = ((uint64_t)t0[b] << 32) | (uint64_t)b;
    qsort(order, (size_t)N, sizeof(uint64_t), cmp_u64);
    or_box *v = (or_box *)malloc((size_t)(N > 0 ? N : 1) * sizeof(or_box));
    uint32_t *t1v = (uint32_t *)malloc((size_t)(N > 0 ? N : 1) * sizeof(uint32_t));
    for (int64_t k = 0; k < N; ++k) {
        int64_t b = (int64_t)(order[k] & 0xFFFFFFFFu);
        for (int d = 0; d < 3; ++d) {
            v[k].lo[d] = lo[3 * b + d];
            v[k].hi[d] = hi[3 * b + d];
        }
        v[k].t0 = t0[b];
        v[k].t1 = t1v[k] = t1[b];
        v[k].obj = obj[b];
        v[k].pad = 0;
    }
    free(order);

    or_heap active = { 0, 0, 0 }; /* visiting positions, heap order by t1 */
    or_box *act = NULL;
    int64_t act_cap = 0;
    int64_t begin = 0;
    while (begin < N) {
        int64_t end = begin + 1;
        while (end < N && (end - begin < OR_BLOCK_MIN || v[end].t0 == v[end - 1].t0))
            ++end;
        while (active.n > 0 && t1v[active.box[0]] <= v[begin].t0)
            heap_pop(&active, t1v);
        int64_t nact = active.n;
        if (nact > act_cap) {
            act_cap = 2 * nact;
            act = (or_box *)realloc(act, (size_t)act_cap * sizeof(or_box));
        }
        for (int64_t q = 0; q < nact; ++q)
            act[q] = v[active.box[q]];
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t k = begin; k < end; ++k) {
#ifdef _OPENMP
            or_vec *mine = &parts[omp_get_thread_num()];
#else
            or_vec *mine = &parts[0];
#endif
            for (int64_t q = 0; q < nact; ++q)
                test_and_emit(mine, &v[k], &act[q]);
            for (int64_t q = begin; q < k; ++q)
                test_and_emit(mine, &v[k], &v[q]);
        }
        for (int64_t k = begin; k < end; ++k)
            heap_push(&active, t1v, (uint32_t)k);
        begin = end;
    }
    free(active.box);
    free(act);
    free(t1v);
    free(v);
    int64_t m = canonical(parts, nt, out);
    free(parts);
    return m;
}

void or_set_num_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/* ------------------------------------------------------------------------ */
/* Alg. Brute Force                                                          */
/* ------------------------------------------------------------------------ */

/* For every multiple t of delta in [0, T], every pair i < j is tested for
 * intersecting occupancy cubes: the closed cubes of radii r_i and r_j about
 * the two positions meet exactly when the inf-norm distance of the centres is
 * at most r_i + r_j.  The algorithm as printed stops at the first witness; it
 * is run to the end here so that recall can be checked, and the first row of
 * the output is its answer. */
int64_t or_brute_force(int64_t n, const double *el, const double *r,
                       uint32_t T, uint32_t delta, double tick_s, double mu,
                       uint32_t **out)
{
    or_vec acc = { 0, 0, 0 };
    double *p = (double *)malloc((size_t)(n > 0 ? n : 1) * 3 * sizeof(double));
    if (delta == 0)
        delta = 1;
    for (uint64_t t = 0; t <= T; t += delta) {
        for (int64_t i = 0; i < n; ++i)
            or_position(el + 6 * i, (double)t * tick_s, mu, p + 3 * i);
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = i + 1; j < n; ++j) {
                double dmax = 0.0;
                for (int d = 0; d < 3; ++d) {
                    double dd = fabs(p[3 * i + d] - p[3 * j + d]);
                    if (dd > dmax)
                        dmax = dd;
                }
                if (dmax <= r[i] + r[j])
                    vec_push(&acc, (uint32_t)t, (uint32_t)i, (uint32_t)j, 0);
            }
    }
    free(p);
    /* repack the 4-wide rows as 3-wide (t, i, j) */
    uint32_t *res = (uint32_t *)malloc((size_t)(acc.n > 0 ? acc.n : 1) * 3 * sizeof(uint32_t));
    for (int64_t k = 0; k < acc.n; ++k) {
        res[3 * k + 0] = acc.v[4 * k + 0];
        res[3 * k + 1] = acc.v[4 * k + 1];
        res[3 * k + 2] = acc.v[4 * k + 2];
    }
    free(acc.v);
    *out = res;
    return acc.n;
}

/* ------------------------------------------------------------------------ */
/* Bulk interval refinement                                                  */
/* ------------------------------------------------------------------------ */

/* occ-int of one object over the continuous times [ta_s, tb_s] by the given
 * rule: 0 the speed-bound box (endpoint hull grown by vmax * span / 2 and the
 * radius), 1 or 2 the interval evaluation over the true or eccentric anomaly. */
static void occ_int(const double e6[6], double ta_s, double tb_s, double mu, double thr_km,
                    int rule, double lo[3], double hi[3])
{
    if (rule == 1 || rule == 2) {
        or_box_interval(e6, ta_s, tb_s, mu, thr_km, rule, lo, hi);
        return;
    }
    double pa[3], pb[3];
    or_position(e6, ta_s, mu, pa);
    or_position(e6, tb_s, mu, pb);
    double g = or_vmax(e6[0], e6[1], mu) * (tb_s - ta_s) / 2.0 + thr_km / 2.0;
    for (int d = 0; d < 3; ++d) {
        lo[d] = fmin(pa[d], pb[d]) - g;
        hi[d] = fmax(pa[d], pb[d]) + g;
    }
}

typedef struct {
    const double *el;
    double tick_s, mu, thr;
    int rule;
    uint64_t delta, start, min_steps;
    or_vec *acc;
} refine_ctx;

/* Grid instants u..v (absolute tick u * delta .. v * delta) of objects i, j:
 * dropped when their occ-int boxes over that span do not meet (no instant in
 * it can collide); kept as one leaf once it holds at most min_steps instants;
 * otherwise halved, the first half taking floor of half the steps as
 * resolveCollisions does. */
static void refine_span(const refine_ctx *c, uint32_t i, uint32_t j, uint64_t u, uint64_t v)
{
    double li[3], hi_[3], lj[3], hj[3];
    double ta = (double)(u * c->delta) * c->tick_s, tb = (double)(v * c->delta) * c->tick_s;
    occ_int(c->el + 6 * i, ta, tb, c->mu, c->thr, c->rule, li, hi_);
    occ_int(c->el + 6 * j, ta, tb, c->mu, c->thr, c->rule, lj, hj);
    for (int d = 0; d < 3; ++d)
        if (li[d] > hj[d] || lj[d] > hi_[d])
            return;
    if (v - u + 1 <= c->min_steps) {
        vec_push(c->acc, i, j, (uint32_t)(u * c->delta - c->start),
                 (uint32_t)(v * c->delta - c->start + 1));
        return;
    }
    uint64_t m = u + (v - u) / 2;
    refine_span(c, i, j, u, m);
    refine_span(c, i, j, m + 1, v);
}

/* The data-parallel form of the time halving of Procedure resolveCollisions:
 * every candidate record (i, j, t_lo, t_hi) -- times relative to start, the
 * last instant T -- covers the grid instants t with start + t a multiple of
 * delta in [t_lo, min(t_hi - 1, T)]; their span is halved while the two
 * objects' boxes over it meet.  Output: the canonical list of kept leaves
 * (i, j, first instant, last instant + 1).  With min_steps = 1 and the speed
 * box the leaves are exactly the instants at which the pair collides (a box
 * over one instant is the occupancy cube, Property 1). */
int64_t or_refine(int64_t n, const double *el, uint32_t T, uint32_t start, double tick_s,
                  double mu, double thr_km, int rule, uint32_t delta, uint32_t min_steps,
                  int64_t R, const uint32_t *rec, uint32_t **out)
{
    if (delta == 0 || min_steps == 0 || rule < 0 || rule > 2)
        return -1;
    or_vec acc = { 0, 0, 0 };
    refine_ctx c = { el, tick_s, mu, thr_km, rule, delta, start, min_steps, &acc };
    for (int64_t r = 0; r < R; ++r) {
        uint32_t i = rec[4 * r], j = rec[4 * r + 1], tlo = rec[4 * r + 2], thi = rec[4 * r + 3];
        if (i >= (uint64_t)n || j >= (uint64_t)n || thi <= tlo)
            continue;
        uint64_t last = (uint64_t)thi - 1 < (uint64_t)T ? (uint64_t)thi - 1 : (uint64_t)T;
        if ((uint64_t)tlo > last)
            continue;
        uint64_t u = ((uint64_t)start + tlo + delta - 1) / delta;
        uint64_t v = ((uint64_t)start + last) / delta;
        if (u > v)
            continue;
        refine_span(&c, i, j, u, v);
    }
    return canonical(&acc, 1, out);
}

/* ------------------------------------------------------------------------ */
/* Potential-collision graph by altitude bands                               */
/* ------------------------------------------------------------------------ */

/* Radial band of an object (Def. Potential-Collision Graph with the perigee
 * and apogee test of the orbit evaluation): every position lies between the
 * perigee a(1 - e) and the apogee a(1 + e) from the Earth's centre, and every
 * point of its occupancy cube within sqrt(3) r of the position (the cube's
 * circumscribed sphere), r = thr / 2. */
void or_band(const double el6[6], double thr_km, double *lo, double *hi)
{
    double a = el6[0], e = el6[1];
    double pad = sqrt(3.0) * 0.5 * thr_km;
    *lo = a * (1.0 - e) - pad;
    *hi = a * (1.0 + e) + pad;
}

/* Two objects can collide only if their bands meet: a common point of the two
 * cubes has one distance from the centre, inside both bands. */
int or_band_compatible(const double el_i[6], const double el_j[6], double thr_km)
{
    double li, hi, lj, hj;
    or_band(el_i, thr_km, &li, &hi);
    or_band(el_j, thr_km, &lj, &hj);
    return li <= hj && lj <= hi;
}

/* The records (i, j, t_lo, t_hi) whose objects are band-compatible, in input
 * order; returns their count (rows of 4 in *out). */
int64_t or_band_filter(int64_t n, const double *el, double thr_km, int64_t R,
                       const uint32_t *rec, uint32_t **out)
{
    uint32_t *res = (uint32_t *)malloc((size_t)(R > 0 ? R : 1) * 4 * sizeof(uint32_t));
    int64_t m = 0;
    for (int64_t r = 0; r < R; ++r) {
        uint32_t i = rec[4 * r], j = rec[4 * r + 1];
        if (i >= (uint64_t)n || j >= (uint64_t)n)
            continue;
        if (or_band_compatible(el + 6 * i, el + 6 * j, thr_km)) {
            memcpy(res + 4 * m, rec + 4 * r, 4 * sizeof(uint32_t));
            ++m;
        }
    }
    *out = res;
    return m;
}

static int cmp_double(const void *pa, const void *pb)
{
    double a = *(const double *)pa, b = *(const double *)pb;
    return a < b ? -1 : (a > b ? 1 : 0);
}

/* Edge partitioning into p altitude bands (Sec. 7, orbital decomposition):
 * the semi-major axes sorted, every d-th one (d = floor(n / p), at least 1)
 * marks an edge, edges[0] = -inf and edges[p] = +inf; object i joins every
 * band [edges[k], edges[k+1]) that its radial band [lo_i, hi_i] meets.
 * Writes edges[p + 1] and count[p] (objects per band); if members is not NULL
 * it receives the bands' object ids, band by band, ascending within a band
 * (sum of count entries).  Returns that sum. */
int64_t or_band_partition(int64_t n, const double *el, double thr_km, int p, double *edges,
                          int64_t *count, uint32_t *members)
{
    if (p < 1)
        return -1;
    double *a = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    for (int64_t i = 0; i < n; ++i)
        a[i] = el[6 * i];
    qsort(a, (size_t)n, sizeof(double), cmp_double);
    int64_t d = n / p > 0 ? n / p : 1;
    edges[0] = -INFINITY;
    edges[p] = INFINITY;
    for (int k = 1; k < p; ++k) {
        int64_t at = (int64_t)k * d;
        edges[k] = n > 0 ? a[at < n ? at : n - 1] : 0.0;
    }
    free(a);
    int64_t total = 0;
    for (int k = 0; k < p; ++k) {
        count[k] = 0;
        for (int64_t i = 0; i < n; ++i) {
            double lo, hi;
            or_band(el + 6 * i, thr_km, &lo, &hi);
            if (lo < edges[k + 1] && hi >= edges[k]) {
                if (members)
                    members[total] = (uint32_t)i;
                ++count[k];
                ++total;
            }
        }
    }
    return total;
}

/* ------------------------------------------------------------------------ */
/* Growth pieces                                                             */
/* ------------------------------------------------------------------------ */

/* Largest float not above x: round to nearest, then step down once if that
 * landed above. */
float or_round_down_f32(double x)
{
    float f = (float)x;
    if ((double)f > x)
        f = nextafterf(f, -INFINITY);
    return f;
}

/* Smallest float not below x. */
float or_round_up_f32(double x)
{
    float f = (float)x;
    if ((double)f < x)
        f = nextafterf(f, INFINITY);
    return f;
}

/* Per-object step: the largest whole number of ticks over which the object
 * cannot move more than max_disp (speed bound vmax).  Any step gives
 * conservative boxes; this one keeps every box's motion term near a fixed
 * length. */
void or_dt_heuristic(int64_t n, const double *el, double mu, double tick_s,
                     double max_disp_km, uint32_t T, uint32_t *dt_out)
{
    double cap = T > 0 ? (double)T : 1.0;
    for (int64_t i = 0; i < n; ++i) {
        double v = or_vmax(el[6 * i], el[6 * i + 1], mu);
        double d = floor(max_disp_km / (v * tick_s));
        if (!(d >= 1.0))
            d = 1.0;
        if (d > cap)
            d = cap;
        dt_out[i] = (uint32_t)d;
    }
}

void or_outward_f32(int64_t m, const double *lo, const double *hi, float *lo32,
                    float *hi32)
{
    for (int64_t k = 0; k < m; ++k) {
        lo32[k] = or_round_down_f32(lo[k]);
        hi32[k] = or_round_up_f32(hi[k]);
    }
}

void or_free(void *p)
{
    free(p);
}
