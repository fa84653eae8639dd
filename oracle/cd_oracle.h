/*
 * cd_oracle.h -- CPU oracle for the 4D-AABB broad phase (test infrastructure).
 *
 * THIS IS TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It shares
 * no code, header, constant or helper with the HIP library; the two meet only
 * through the seeded input catalogs.
 *
 * Everything is plain IEEE FP64 C, written to be read against Bak & Hobbs,
 * "Efficient n-to-n Collision Detection for Space Debris using 4D AABB Trees":
 *   - Def. "World Object", "Occupancy Region", "Collision" (Sec. 2)
 *   - Alg. "Brute Force Method" (Sec. 3.1)
 *   - Def. "Interval Occupancy Region" with Properties 1-2, Def. "4D Occupancy
 *     Region" (Sec. 4), the clamp of procedure advanceTime (Sec. 4.3)
 *   - Eq. (nu-dot) and the three-rotation map to ECI (Sec. 7.1)
 *
 * Units: km, s, rad; time on the integer tick grid (tick_s seconds per tick).
 * Element rows are {a, e, i, raan, argp, m0} (m0 = mean anomaly at t = 0).
 * Box arrays are AoS: lo[N][3], hi[N][3].  Pair records are uint32[4]
 * {i, j, t_lo, t_hi} with i < j, meaning the two 4D boxes overlap during the
 * integer ticks [t_lo, t_hi).
 */
#ifndef CD_ORACLE_H
#define CD_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- dynamics: g(t) = nu(t) and h(nu) of Sec. 4.5 / 7.1 ------------------ */
double or_eccentric_anomaly(double M, double e);
double or_true_anomaly(const double el[6], double t_s, double mu);
void or_position_from_nu(const double el[6], double nu, double pos[3]);
void or_position(const double el[6], double t_s, double mu, double pos[3]);
double or_vmax(double a, double e, double mu);

/* ---- 4D boxes (Def. Interval Occupancy Region / 4D Occupancy Region) ----- */
/* number of intervals of one object: max(1, ceil(T / dt)) */
uint64_t or_intervals(uint32_t dt, uint32_t T);
int64_t or_box_count(int64_t n, const uint32_t *dt, uint32_t T);
/* Object-major boxes: box (i, k) is at off_i + k, off_i = sum_{i'<i} K_i'.
 * The horizon covers absolute ticks [start, start + T]: positions are taken
 * at start + t_k, tags are relative to start (a window of a longer horizon
 * is the same problem over a shifted time interval).
 * Returns 0, or -1 on invalid input (dt = 0, T + 1 overflow). */
int or_boxes(int64_t n, const double *el, const uint32_t *dt, uint32_t T, uint32_t start,
             double tick_s, double mu, double thr_km, int rule,
             double *lo, double *hi, uint32_t *t0, uint32_t *t1, uint32_t *obj);

/* ---- interval arithmetic and the interval-evaluation box (Sec. 4.5) ---- */
/* rule of or_boxes: 0 the speed-bound box; 1 or 2 or_box_interval over the
 * true (1) or eccentric (2) anomaly */
typedef struct {
    double lo, hi;
} or_iv;
or_iv or_iv_make(double lo, double hi);
or_iv or_iv_add(or_iv a, or_iv b);
or_iv or_iv_sub(or_iv a, or_iv b);
or_iv or_iv_mul(or_iv a, or_iv b);
or_iv or_iv_div(or_iv a, or_iv b);
or_iv or_iv_sqr(or_iv a);
or_iv or_iv_cos(or_iv x);
or_iv or_iv_sin(or_iv x);
void or_box_interval(const double el[6], double ta_s, double tb_s, double mu, double thr_km,
                     int var, double lo[3], double hi[3]);

/* ---- pair sets: the plain definition, all box pairs tested -------------- */
/* Literal all-pairs over N boxes.  *out receives a malloc'd, canonical
 * (sorted by i, j, t_lo, t_hi; duplicate-free) record array; free with
 * or_free.  Returns the record count. */
int64_t or_pairs(int64_t N, const double *lo, const double *hi,
                 const uint32_t *t0, const uint32_t *t1, const uint32_t *obj,
                 uint32_t **out);
/* All records that involve at least one of the ns sampled boxes. */
int64_t or_pairs_of(int64_t N, const double *lo, const double *hi,
                    const uint32_t *t0, const uint32_t *t1, const uint32_t *obj,
                    int64_t ns, const int64_t *sample, uint32_t **out);
/* The same canonical set as or_pairs, testing only box pairs whose time tags
 * overlap: a sweep in t0 order with an active list in t1 order (with a
 * uniform step, all pairs within each time slab).  N < 2^32. */
int64_t or_pairs_bucketed(int64_t N, const double *lo, const double *hi,
                          const uint32_t *t0, const uint32_t *t1, const uint32_t *obj,
                          uint32_t **out);
/* Brute-force-equivalent test count: different-object box pairs whose time
 * tags overlap (the work the plain definition cannot skip). */
int64_t or_time_overlapping_pairs(int64_t N, const uint32_t *t0,
                                  const uint32_t *t1, const uint32_t *obj);

/* ---- Alg. Brute Force on the occupancy regions -------------------------- */
/* All witnesses (i < j, t) with occ(w_i,t) and occ(w_j,t) intersecting, at
 * t = 0, delta, 2 delta, ... <= T ticks; radius r[i] per object.  Output is
 * a malloc'd uint32[count][3] in (t, i, j) order.  The first row is the
 * algorithm's own answer (its first witness). */
int64_t or_brute_force(int64_t n, const double *el, const double *r,
                       uint32_t T, uint32_t delta, double tick_s, double mu,
                       uint32_t **out);

/* ---- growth pieces ------------------------------------------------------ */
float or_round_down_f32(double x);
float or_round_up_f32(double x);
/* elementwise RD(lo), RU(hi) over m values */
void or_outward_f32(int64_t m, const double *lo, const double *hi, float *lo32,
                    float *hi32);
/* dt_i = clamp(floor(max_disp / (vmax_i * tick_s)), 1, max(T, 1)) ticks */
void or_dt_heuristic(int64_t n, const double *el, double mu, double tick_s,
                     double max_disp_km, uint32_t T, uint32_t *dt_out);

void or_free(void *p);
int or_num_threads(void);
/* OpenMP threads of the later calls (<= 0 leaves the setting unchanged) */
void or_set_num_threads(int nthreads);

/* ---- bulk interval refinement (resolveCollisions' halving, in bulk) ---- */
/* rec: R records (i, j, t_lo, t_hi) relative to start; rule as or_boxes;
 * returns the canonical leaf count (rows of 4 in *out, free with or_free),
 * -1 on bad arguments. */
int64_t or_refine(int64_t n, const double *el, uint32_t T, uint32_t start, double tick_s,
                  double mu, double thr_km, int rule, uint32_t delta, uint32_t min_steps,
                  int64_t R, const uint32_t *rec, uint32_t **out);

/* ---- potential-collision graph by altitude bands ---- */
void or_band(const double el6[6], double thr_km, double *lo, double *hi);
int or_band_compatible(const double el_i[6], const double el_j[6], double thr_km);
int64_t or_band_filter(int64_t n, const double *el, double thr_km, int64_t R,
                       const uint32_t *rec, uint32_t **out);
int64_t or_band_partition(int64_t n, const double *el, double thr_km, int p, double *edges,
                          int64_t *count, uint32_t *members);

#ifdef __cplusplus
}
#endif
#endif
