/*
 * cd4d.h -- C ABI of the MI355X (gfx950) 4D-AABB broad phase.
 *
 * Bak & Hobbs, "Efficient n-to-n Collision Detection for Space Debris using 4D
 * AABB Trees".  The library answers the broad-phase half of the paper's
 * problem (Def. Continuous / Discrete-Time n-to-n Collision Detection
 * Problem, Sec. 2): given n world objects (Def. World Object) moving on Kepler
 * orbits (Sec. 7.1) and a horizon T, it returns every candidate
 *     (i, j, [t_lo, t_hi))   i < j
 * whose 4D occupancy regions (Def. 4D Occupancy Region, Sec. 4) intersect.
 * The paper's sequential tree (Alg. 4D AABB Tree Collision Detection) tests
 * these box intersections one query at a time; here all of them are found in
 * one bulk pass: boxes -> sorted Morton keys -> LBVH -> self-traversal ->
 * canonical list.
 *
 * Conventions shared by every entry point:
 *   - Units: km, s, rad.  Time is counted in integer ticks of tick_s seconds.
 *   - Every pointer is a DEVICE pointer unless its name ends in _host.
 *   - The caller allocates and owns all memory: elements, boxes, tree,
 *     workspace and output.  The library allocates no device memory.  Its
 *     only state is: the thread-local error string (cd_last_error); the
 *     thread-local launch shapes of the traversal (cd_set_tuning), read by
 *     the calling thread's later queries; the process-wide stage profiler
 *     (cd_profile_*, guarded by a mutex); and a process-wide hint, kept in an
 *     atomic, of how many node-pair levels the last drained synchronous query
 *     needed, which sets how many levels the next one launches before its
 *     first host check; and, per thread, the last synchronous query's level
 *     count (cd_last_query_levels) and raw record count (when that fitted the
 *     one-workgroup canonical list, the next query forms its list before the
 *     first host check, on the device's count).  None of them changes a
 *     result: records depend only on the arguments of the call.
 *   - Streams are hipStream_t values passed as void* (NULL = default stream).
 *     Work is enqueued on that stream; functions marked "syncs" wait for it.
 *   - Every function returns a status code; no exception crosses the ABI.
 *     cd_last_error() gives a thread-local message for the last failure.
 *   - Workspace sizes come from the matching *_ws query; passing less returns
 *     CD_E_WORKSPACE before anything is enqueued.
 *   - CD_DEBUG_SYNC=1 in the environment (read once per process): every call
 *     that enqueues work also waits for it and returns at once what would
 *     otherwise surface at a later synchronising call: CD_E_DEVICE for a HIP
 *     error, CD_E_INVALID from cd_build_tree when the build flagged its
 *     input (keys out of order, a box outside its slab) and from
 *     cd_query_pairs_async for status bit 2, CD_E_CAPACITY from
 *     cd_query_pairs_async for status bit 1.  Skipped while the stream
 *     records a graph.
 */
#ifndef CD4D_H
#define CD4D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define CD_OK 0
#define CD_E_INVALID 1   /* bad argument: null pointer, n < 0, dt = 0, e outside [0,1), ... */
#define CD_E_WORKSPACE 2 /* workspace (or tree buffer) smaller than required */
#define CD_E_CAPACITY 3  /* more records than `capacity`; *count_host holds the need */
#define CD_E_OVERFLOW 4  /* n, box count or T + 1 does not fit 32 bits */
#define CD_E_DEVICE 5    /* HIP runtime error; see cd_last_error() */

/* ---- precisions of boxes and trees ------------------------------------- */
#define CD_FP64 0
#define CD_FP32 1 /* outward-rounded: lo rounded down, hi rounded up */

typedef void *cd_stream_t; /* a hipStream_t */

/* Orbital elements of n objects, structure of arrays, FP64, device memory.
 * a: semi-major axis (km, > 0); e: eccentricity in [0, 1); inc, raan, argp:
 * inclination, right ascension of the ascending node, argument of perigee
 * (rad); m0: mean anomaly at t = 0 (rad).  (Sec. 7.1 lists the true anomaly;
 * the mean anomaly at epoch fixes it.) */
typedef struct {
    const double *a, *e, *inc, *raan, *argp, *m0;
    int64_t n;
} cd_elements;

/* Run parameters.  threshold_km is the collision distance thr = 2r: every
 * object is a world object with inf-norm radius r = thr / 2 (Def. World
 * Object, Def. Occupancy Region).  horizon_ticks is T; its last tick is
 * included, so T + 1 must fit 32 bits.  dt_ticks is the uniform time step,
 * used when no per-object step array is given.  start_ticks places the
 * horizon at absolute ticks [start, start + T] after the elements' epoch
 * (positions are taken at start + t); tags and records stay relative to
 * start, so a long horizon can be run as consecutive windows.  box_rule
 * chooses how cd_build_boxes bounds an object over an interval (the occ-int
 * of Def. Interval Occupancy Region): CD_BOX_SPEED (0) or one of the two
 * interval evaluations of Sec. 4.5; other values are CD_E_INVALID. */
enum {
    CD_BOX_SPEED = 0,       /* endpoint hull grown by vmax * dt / 2 */
    CD_BOX_INTERVAL_NU = 1, /* interval evaluation over the true anomaly */
    CD_BOX_INTERVAL_E = 2   /* interval evaluation over the eccentric anomaly */
};
typedef struct {
    double tick_s;          /* seconds per tick, e.g. 1e-3 */
    double mu;              /* gravitational parameter, km^3/s^2 (398600.4418) */
    double threshold_km;    /* thr >= 0 */
    uint32_t horizon_ticks; /* T */
    uint32_t dt_ticks;      /* uniform step (>= 1) when no dt array is given */
    uint32_t start_ticks;   /* absolute tick of the horizon's t = 0 (0: the epoch) */
    uint32_t box_rule;      /* CD_BOX_* (0: the speed bound) */
} cd_params;

/* A set of 4D boxes, structure of arrays, caller-owned device memory.
 * Box b covers lo[d][b] <= x_d <= hi[d][b] (closed) during ticks
 * t0[b] <= t < t1[b] and belongs to object obj[b].  lo/hi point to double
 * (CD_FP64) or float (CD_FP32) arrays.
 *
 * Layout hints, written by cd_build_boxes and optional for caller-built boxes:
 *   slab_ticks, slab_size: if slab_size > 0, boxes [s*slab_size,
 *     (s+1)*slab_size) all have t0 / slab_ticks == s (time-major slabs);
 *     the tree builder then sorts each slab inside one workgroup.
 *   horizon_ticks: an upper bound on every t0 (used to size sort keys).
 *   obj_count: an upper bound on obj + 1 (used to size sort keys); 0 means
 *     "up to 2^32".
 *   code, code_valid: optional per-box 30-bit Morton code (the tree's
 *     spatial sort key).  If code is not NULL, cd_build_boxes writes it (in
 *     the frame of the orbits' bounding boxes, so no code is clamped) and sets
 *     code_valid = 1; cd_build_tree then sorts by these codes instead of
 *     re-reading every box to form them.  Codes only shape the tree: any codes
 *     give the same records.  code_valid = 0 (or code NULL) makes
 *     cd_build_tree compute codes from the boxes.
 *   layout: the order of a uniform step's boxes inside each time slab.
 *     CD_LAYOUT_OBJECT: box (i, k) at k * n + i, code = that of the box
 *     centre.  CD_LAYOUT_SORTED: the slabs are taken in blocks of 8
 *     consecutive slabs (more when K / 8 exceeds 65 535), and inside every
 *     slab of a block the boxes follow the Morton order of their objects'
 *     positions at the block's middle instant; code holds that order's key
 *     (non-decreasing along each slab) and obj[b] names the object of box b.
 *     cd_build_boxes reads the requested layout (CD_LAYOUT_SORTED needs code
 *     != NULL and n <= CD_SORTED_MAX_ARRAYS, or n <= CD_SORTED_MAX_RECORDS
 *     when writing records; otherwise, and for per-object steps, it writes
 *     CD_LAYOUT_OBJECT) and leaves the layout it wrote.  cd_build_tree
 *     needs no key sort for CD_LAYOUT_SORTED boxes with valid codes and slab
 *     hints; it checks that each slab's codes are non-decreasing (error bit
 *     as for a box outside its slab, reported by the query).
 *   records: NULL, or FP64 box records written instead of the lo, hi, t0,
 *     t1 and obj arrays: 64 bytes per box, {double lo[3], hi[3]; uint32_t
 *     t0, t1, obj, code}, the layout of an FP64 tree's leaf records (the code
 *     array is still written as well).  cd_build_boxes writes them for a
 *     uniform step in the sorted layout (FP64 boxes, n <=
 *     CD_SORTED_MAX_RECORDS; otherwise CD_E_INVALID).  With records =
 *     cd_tree_leaf_records(tree) and CD_LAYOUT_SORTED, cd_build_tree takes
 *     them as the tree's leaves where they are: no sort and no copy. */
typedef struct {
    int64_t count;
    int precision;
    void *lo[3], *hi[3];
    uint32_t *t0, *t1, *obj;
    uint32_t slab_ticks;
    int64_t slab_size;
    uint32_t horizon_ticks;
    uint32_t obj_count;
    uint32_t *code;
    int code_valid;
    int layout;   /* CD_LAYOUT_OBJECT or CD_LAYOUT_SORTED */
    void *records;
} cd_boxes;
#define CD_LAYOUT_OBJECT 0
#define CD_LAYOUT_SORTED 1
/* object counts up to which cd_build_boxes writes CD_LAYOUT_SORTED boxes */
#define CD_SORTED_MAX_ARRAYS 17408
#define CD_SORTED_MAX_RECORDS 278528

/* A linear BVH over a box set.  mem is a caller-owned device buffer of
 * cd_tree_bytes(count, precision) bytes; cd_build_tree fills it and the
 * remaining descriptor fields. */
typedef struct {
    void *mem;
    size_t bytes;
    int64_t count;      /* leaves */
    int precision;
    uint32_t slab_ticks;
    uint32_t horizon_ticks;
    uint32_t obj_count;
} cd_tree;

/* One candidate: objects i < j, whose boxes overlap during ticks
 * [t_lo, t_hi) (t_hi = T + 1 marks an interval that ends at T inclusive). */
typedef struct {
    uint32_t i, j, t_lo, t_hi;
} cd_pair;

/* ---- diagnostics -------------------------------------------------------- */
const char *cd_status_string(int status);
const char *cd_last_error(void);
int cd_version(void);

/* A plain streaming copy of `bytes` bytes from src to dst (device memory):
 * 16-byte loads, non-temporal 16-byte stores, grid-stride.  It is the
 * measured achievable HBM bandwidth (read + write bytes over its time) that
 * the kernels' roofline fractions are read against, beside the 8 TB/s
 * specification, and a kernel of known byte count for calibrating HBM byte
 * counters.  bytes and both addresses must be multiples of 16 and the ranges
 * must not overlap (else CD_E_INVALID).  Async. */
int cd_stream_copy(void *dst, const void *src, size_t bytes, cd_stream_t stream);

/* Per-stage device time.  While enabled, every call records a hipEvent pair
 * on its stream around each kernel stage ("boxes", "keys", "sort", "karras",
 * "refit", "traverse", "canon").  cd_profile_read waits for the recorded
 * events, accumulates elapsed milliseconds and launch counts per stage name,
 * copies up to `max` entries (names are static strings) and returns how many
 * stages exist; reset != 0 clears the totals.  Process-wide, guarded by a
 * mutex; the events are created lazily and reused. */
int cd_profile_enable(int on);
int cd_profile_read(const char **names, double *ms_total, int64_t *launches, int max,
                    int reset);

/* ---- step 1: per-object time steps and box counts ----------------------- */

/* Number of boxes the given steps produce: sum over objects of
 * K_i = max(1, ceil(T / dt_i)).  Each object's interval sequence follows
 * procedure advanceTime (Sec. 4.3): consecutive intervals on the tick grid,
 * the last one clamped at T.  dt_ticks may be NULL (uniform params->dt_ticks;
 * no device work) or a device array of n steps (syncs; CD_E_INVALID if any
 * step is 0).  ws must hold cd_box_count_ws(n) bytes. */
size_t cd_box_count_ws(int64_t n);
int cd_box_count(const uint32_t *dt_ticks, int64_t n, const cd_params *p,
                 int64_t *count_host, void *ws, size_t ws_bytes, cd_stream_t stream);

/* Checks every element (finite; a > 0; 0 <= e < 1).  Syncs.  On failure
 * returns CD_E_INVALID and *bad_index_host = first offending object. */
size_t cd_validate_ws(int64_t n);
int cd_validate_elements(const cd_elements *el, int64_t *bad_index_host, void *ws,
                         size_t ws_bytes, cd_stream_t stream);

/* Per-object step from the speed bound.  The paper keeps one time interval
 * per object (Sec. 4: each object's t_min, t_max) and leaves its length to a
 * rule (Procedure advanceTime, Sec. 4.3, doubles it while the object meets
 * nobody); this call fixes the length per object so that each interval's
 * displacement is at most max_disp_km:
 *   dt_i = clamp(floor(max_disp_km / (vmax_i * tick_s)), 1, max(T, 1)) ticks,
 * vmax_i the perigee speed.  Any step keeps the boxes conservative; this one
 * bounds each box's motion term.  Async. */
int cd_dt_heuristic(const cd_elements *el, const cd_params *p, double max_disp_km,
                    uint32_t *dt_out, cd_stream_t stream);

/* ---- step 2: 4D boxes (Def. Interval Occupancy Region, 4D Occupancy) ----- */

/* Builds every box.  For object i and interval k, with t_k = min(k dt_i, T),
 * Kepler propagation (the exact solution of Eq. nu-dot, mapped to ECI by the
 * three rotations of Sec. 7.1) gives, in FP64, the positions p_a = pos(t_k),
 * p_b = pos(t_{k+1}) and the eccentric anomalies E_a, E_b.  The box is
 *   CD_BOX_SPEED: g = vmax_i (t_{k+1} - t_k) tick_s / 2 + thr / 2,
 *     lo = min(p_a, p_b) - g, hi = max(p_a, p_b) + g per axis;
 *   CD_BOX_INTERVAL_NU (Sec. 4.5 with the variable of Sec. 7.1): h evaluated
 *     in outward-rounded interval arithmetic over [nu_a, nu_b] (the whole
 *     turn when the mean anomaly advances 2 pi or more), h being
 *     r = a (1 - e^2) / (1 + e cos nu), then (r cos nu) P + (r sin nu) Q;
 *   CD_BOX_INTERVAL_E: the same over [E_a, E_b] with coordinate d written
 *     as ctr_d + R_d cos(E - phi_d), in which E occurs once, so the box is
 *     the hull of the path itself (the endpoint hull, extended to
 *     ctr_d +- R_d where E - phi_d crosses a multiple of pi);
 *   the interval rules widen the variable's range by 1e-10 rad and add
 *   thr / 2;
 *   tag [t_k, t_{k+1}), the last one [t_{K-1}, T + 1).
 * Every rule holds each position in the interval and equals the occupancy
 * cube at a single instant (Property 1).  With a CD_FP32 output the FP64
 * bounds are rounded outward.
 * Order: uniform step (dt_ticks NULL) -> time-major, slab k at [k n, (k + 1) n)
 * in the order out->layout asks for (box (i,k) at k*n + i for
 * CD_LAYOUT_OBJECT; by the objects' Morton order for CD_LAYOUT_SORTED), and
 * out->slab_size = n, out->slab_ticks = dt.  Per-object steps -> object-major,
 * box (i,k) at off_i + k.  out->count must equal cd_box_count's result and
 * out's arrays must hold that many entries.  Async; element validity is not
 * rechecked here (see cd_validate_elements). */
size_t cd_build_boxes_ws(int64_t n);
int cd_build_boxes(const cd_elements *el, const uint32_t *dt_ticks, const cd_params *p,
                   cd_boxes *out, void *ws, size_t ws_bytes, cd_stream_t stream);

/* ---- step 3: the tree (Morton keys, LDS radix sort, Karras LBVH, refit) -- */

/* Builds an LBVH over the boxes (the AABB tree of Sec. 3.2, built in bulk):
 * each box gets a time-major key [t0 / slab_ticks | 30-bit Morton code of its
 * centre (of a given code, its low 30 bits)]; keys are radix-sorted (inside one workgroup's LDS per slab when
 * the slab hint is set, device-wide otherwise); the binary radix (Karras)
 * hierarchy over the sorted keys has every inner box equal to the exact union
 * of its children, so an inner node overlaps whatever its leaves overlap.  It
 * is formed top-down with an atomic refit for slab-hinted box arrays, and
 * from the leaves up in one pass (hierarchy and unions together) for box
 * records in place and for box sets without a slab hint (after the
 * device-wide key sort).  precision CD_FP32 is allowed for FP64 boxes (outward
 * rounding at the leaves).  slab_ticks = 0 takes boxes->slab_ticks if set,
 * else horizon / 64 (at least 1).  Box records in the tree's own leaf-record
 * area (cd_boxes.records) are used in place.
 * Async. */
size_t cd_tree_bytes(int64_t count, int precision);
/* The leaf-record area of an FP64 tree buffer of count leaves (host pointer
 * arithmetic on tree_mem; NULL if count < 1): where cd_build_boxes can write
 * box records for cd_build_tree to use in place (see cd_boxes.records). */
void *cd_tree_leaf_records(void *tree_mem, int64_t count);
size_t cd_build_tree_ws(int64_t count);
int cd_build_tree(const cd_boxes *boxes, int precision, uint32_t slab_ticks, cd_tree *tree,
                  void *ws, size_t ws_bytes, cd_stream_t stream);

/* ---- step 4: the n-to-n query ------------------------------------------- */

/* Self-traversal of the tree.  Two objects' 4D occupancy regions intersect
 * when their time intervals overlap and their 3D boxes do (Def. 4D Occupancy
 * Region, Sec. 4); a box is never paired with another box of its own object,
 * as queryObject excludes the queried object (Procedure resolveCollisions,
 * Sec. 4.4) and Alg. Brute Force pairs distinct objects only (Sec. 3.1).
 * Every pair of boxes of different objects whose time tags overlap
 * (t0_a < t1_b and t0_b < t1_a) and whose closed 3D extents overlap on every
 * axis gives one record
 *   (min(obj), max(obj), max(t0_a, t0_b), min(t1_a, t1_b)).
 * The list written to out is sorted by (i, j, t_lo, t_hi) and free of
 * repeats.  Syncs (it reads the record count).  If more than `capacity`
 * records exist, returns CD_E_CAPACITY with *count_host = the number needed;
 * out is then unspecified, the tree is untouched and the call can be repeated
 * with a larger buffer and workspace. */
size_t cd_query_pairs_ws(int64_t count, int64_t capacity);
int cd_query_pairs(const cd_tree *tree, cd_pair *out, int64_t capacity, int64_t *count_host,
                   void *ws, size_t ws_bytes, cd_stream_t stream);

/* Graph-capturable form of cd_query_pairs: the same records in the same
 * order, with no host synchronisation and no host reads, so the call can be
 * recorded into a hipGraph (cd_graph_*) and replayed.  Results stay on the
 * device:
 *   *count_dev  (uint64): records written to out; when status bit 1 is set,
 *                         the number of raw records found instead (an upper
 *                         bound of what a repeat with more capacity needs);
 *   *status_dev (uint32): 0, or bit 1 = capacity exceeded (out incomplete),
 *                         bit 2 = tree inconsistent (as CD_E_INVALID above).
 * The node-pair traversal runs for the tuning's max_levels levels, each
 * level ending at once when the previous queue is empty; if its queue
 * overflows or is not drained by then, the per-leaf walk redoes the
 * traversal, decided on the device.  The canonical sort runs over all
 * `capacity` slots (unused slots hold a filler record that sorts last), so
 * its cost follows the capacity, not the count.  Workspace as for
 * cd_query_pairs.  Returns CD_OK once everything is enqueued. */
int cd_query_pairs_async(const cd_tree *tree, cd_pair *out, int64_t capacity,
                         unsigned long long *count_dev, unsigned int *status_dev, void *ws,
                         size_t ws_bytes, cd_stream_t stream);

/* The same query as cd_query_pairs_async, for callers that cannot allocate
 * memory (code under hipGraph capture, tight serving loops, harnesses that
 * forbid allocation): the workspace is a fixed device array inside the
 * library, cd_noalloc_scratch_bytes() bytes (64 MiB) per device, held by
 * every device the library runs on until the process ends.  The caller still
 * passes the tree and the outputs.  A query whose workspace
 * (cd_query_pairs_ws(tree->count, capacity)) exceeds the array returns
 * CD_E_WORKSPACE before anything is enqueued.  Call with the stream's device
 * current.  All calls on one device share its array: calls that overlap in
 * time on one device (several streams, several host threads) race and give
 * undefined results; calls ordered on one stream are safe, since each call
 * clears what it reads before use.  Allocates nothing; the first call on a
 * device looks up the array's device address.  Async. */
size_t cd_noalloc_scratch_bytes(void);
int cd_query_pairs_async_noalloc(const cd_tree *tree, cd_pair *out, int64_t capacity,
                                 unsigned long long *count_dev, unsigned int *status_dev,
                                 cd_stream_t stream);

/* ---- launch shapes of the traversal -------------------------------------- */

/* Launch shapes of the calling thread, read by that thread's later query
 * calls (a captured graph keeps the shapes in force at capture time).  Zero
 * fields take the defaults in brackets.  Shapes change timing only, never the
 * records. */
typedef struct {
    uint32_t expand_blocks;   /* workgroups per node-pair level, 64..65536 [2048]; mode 2:
                                 at most this many, and no more than the device holds
                                 at once */
    uint32_t expand_threads;  /* lanes per node-pair workgroup: 64 .. 1024, a power of 2
                                 [256]; mode 2 always takes 1024 */
    uint32_t walk_threads;    /* lanes per per-leaf-walk workgroup: 64, 128 or 256 [256] */
    uint32_t mode;            /* 0 = node pairs, one launch per level, per-leaf walk as
                                 fallback; 1 = per-leaf walk only; 2 = node pairs, every
                                 level in one launch of a resident grid (levels separated
                                 by a device-wide wait bounded at 2 s, after which the
                                 per-leaf walk takes over), per-leaf walk as fallback [0] */
    uint32_t max_levels;      /* node-pair levels of cd_query_pairs_async in mode 0,
                                 1..400 [96] */
} cd_tuning;

/* NULL restores the defaults; out-of-range fields give CD_E_INVALID and
 * change nothing. */
int cd_set_tuning(const cd_tuning *t);
int cd_get_tuning(cd_tuning *t);
/* Node-pair levels the calling thread's last cd_query_pairs ran until its
 * queue was empty (0 when that query used the per-leaf walk, or none ran):
 * on the same tree, a max_levels with which cd_query_pairs_async needs no
 * walk. */
int cd_last_query_levels(void);

/* ---- executed-work counters (diagnostic build) --------------------------- */

/* The library built with CD_COUNTERS defined (libcd4d_counters.so, the same
 * calls and results as libcd4d.so) counts the work the traversal executes:
 * the brute force of Alg. Brute Force tests every pair of boxes, the tree
 * tests far fewer, and these counters say how many.  Totals since the last
 * cd_counters_reset, summed over every query of every thread of the process:
 *   tests        4D box-box tests executed by the traversal (node pairs: the
 *                child pairs of every expanded pair; per-leaf walk: one per
 *                visited node).  The build adds one sibling test per inner
 *                node (the traversal's seeds), not counted here.
 *   leaf_tests   of those, tests between two leaf boxes;
 *   mixed_tests  tests between a leaf box and an inner node;
 *   leaf_hits    tests of two overlapping leaf boxes of different objects
 *                (each one appended record, before repeats are removed);
 *   pairs        node pairs expanded (seeds and queued pairs);
 *   walk_steps   tests made by per-leaf walks.
 * visits (optional, a device array of n counts that the caller zeroes): entry
 * i is incremented for every counted test with a leaf box of object i on one
 * side (twice for a test of two leaves of object i), so the entries sum to
 * 2 leaf_tests + mixed_tests. */
typedef struct {
    uint64_t tests, leaf_tests, mixed_tests, leaf_hits, pairs, walk_steps;
} cd_counters;

/* 1 in the CD_COUNTERS build, 0 otherwise (then reset and read return
 * CD_E_INVALID). */
int cd_counters_available(void);
/* Zeroes the totals and binds visits (NULL: none; n < 2^32).  Syncs. */
int cd_counters_reset(uint32_t *visits, int64_t n, cd_stream_t stream);
/* Totals so far.  Syncs. */
int cd_counters_read(cd_counters *out_host, cd_stream_t stream);

/* ---- graphs ------------------------------------------------------------- */

/* Record the work the calling thread enqueues on `stream` (any of the calls
 * above except those that synchronise: cd_box_count, cd_validate_elements,
 * cd_query_pairs) and replay it with one launch.  The stream must not be the
 * legacy default stream.  Buffers named by the recorded calls must stay
 * allocated while the graph exists; a replay rereads their current contents. */
typedef struct cd_graph_s *cd_graph;
int cd_graph_begin(cd_stream_t stream);
int cd_graph_end(cd_stream_t stream, cd_graph *graph_out);
int cd_graph_launch(cd_graph graph, cd_stream_t stream);
int cd_graph_destroy(cd_graph graph);

/* ---- narrow phase: the first collision (Alg. Brute Force over candidates) */

/* For record r of pairs[0..count) (as returned by cd_query_pairs for the same
 * elements and params): witness_out[r] = the first instant t, in ticks
 * relative to the horizon's start like the records, with t_lo <= t < t_hi,
 * t <= T and start_ticks + t a multiple of delta_ticks (the instants 0,
 * delta, 2 delta, ... of Alg. Brute Force), at which
 * ||p_i(t) - p_j(t)||_inf <= threshold_km (the occupancy cubes of radius
 * thr / 2 touch or overlap, Def. Occupancy Region); CD_NO_WITNESS if none.
 * first_out (device uint64, nullable) receives min over records of
 * (t << 32 | r): the earliest collision and, among equal instants, the first
 * record in canonical order, i.e. the smallest (i, j); ~0 if no record has
 * one.  Positions are those of cd_build_boxes (FP64 Kepler propagation).
 * Because every collision instant lies inside some record (the boxes are
 * conservative), the result equals Alg. Brute Force's first collision.
 * delta_ticks >= 1.  Async. */
#define CD_NO_WITNESS 0xFFFFFFFFu
int cd_first_witness(const cd_elements *el, const cd_params *p, uint32_t delta_ticks,
                     const cd_pair *pairs, int64_t count, uint32_t *witness_out,
                     unsigned long long *first_out, cd_stream_t stream);

/* ---- bulk interval refinement (Procedure resolveCollisions, in bulk) ----- */

/* The time halving of Procedure resolveCollisions applied to every candidate
 * record at once.  Record r = (i, j, t_lo, t_hi) of pairs[0..count) covers
 * the grid instants t (relative ticks, start_ticks + t a multiple of
 * delta_ticks) with t_lo <= t <= min(t_hi - 1, T).  Their span is dropped when
 * the two objects' occ-int boxes over it (p->box_rule, as cd_build_boxes
 * forms them, over the continuous time between its first and last instant)
 * do not meet; kept as a leaf once it holds at most min_steps instants;
 * otherwise halved, the first half taking half of the remaining steps rounded
 * down, and each half tested again.  out receives the canonical list (sorted
 * by i, j, t_lo, t_hi; repeats removed) of leaves (i, j, first instant, last
 * instant + 1).  With min_steps = 1 and CD_BOX_SPEED the leaves are exactly
 * the instants at which the pair collides (a box over one instant is the
 * occupancy cube, Property 1); the interval rules add only instants within
 * their 1e-10 rad widening of the threshold.
 * *count_host = leaves written.  CD_E_CAPACITY: more leaves than capacity
 * (*count_host = the leaf count), or a level's work queue, max(2 count,
 * capacity, 65536) items, overflowed (*count_host = twice that); retry with
 * capacity >= *count_host.  Synchronises. */
size_t cd_refine_records_ws(int64_t n, int64_t count, int64_t capacity);
int cd_refine_records(const cd_elements *el, const cd_params *p, uint32_t delta_ticks,
                      uint32_t min_steps, const cd_pair *pairs, int64_t count, cd_pair *out,
                      int64_t capacity, int64_t *count_host, void *ws, size_t ws_bytes,
                      cd_stream_t stream);

/* ---- potential-collision graph by altitude bands ------------------------ */

/* Def. Potential-Collision Graph, with the perigee/apogee test of the orbit
 * evaluation: object i lies at distances from the Earth's centre in its radial
 * band [a_i(1 - e_i) - sqrt(3) r, a_i(1 + e_i) + sqrt(3) r], r = thr / 2 (a
 * point of its occupancy cube is within sqrt(3) r of the position, the cube's
 * circumscribed sphere), so objects with disjoint bands never collide.
 *
 * cd_band_filter: out[0..*count_host) = the records of pairs[0..count) whose
 * objects' bands meet, in input order (a canonical input stays canonical).
 * out may not alias pairs.  Synchronises. */
size_t cd_band_filter_ws(int64_t count);
int cd_band_filter(const cd_elements *el, const cd_params *p, const cd_pair *pairs,
                   int64_t count, cd_pair *out, int64_t *count_host, void *ws, size_t ws_bytes,
                   cd_stream_t stream);

/* Edge partitioning into nbands altitude bands (Sec. 6 and the orbit
 * evaluation's decomposition): edges[0] = -inf, edges[nbands] = +inf and
 * edges[k] = the (k * max(1, n / nbands))-th smallest semi-major axis; object
 * i joins every band k with lo_i < edges[k + 1] and hi_i >= edges[k] (its
 * radial band meets [edges[k], edges[k + 1])).  Every band-compatible pair
 * shares a band, so the bands are independent problems whose records, mapped
 * back (cd_remap_records) and filtered (cd_band_filter), make up the filtered
 * records of the whole catalog.  Outputs (device): edges[nbands + 1] (double),
 * offsets[nbands + 1] (uint32: band k's objects are members[offsets[k] ..
 * offsets[k + 1]), ascending ids), members[capacity].  *count_host = the
 * number of memberships; CD_E_CAPACITY if it exceeds capacity.
 * 1 <= nbands <= 4096, n * nbands < 2^32.  Synchronises. */
size_t cd_band_partition_ws(int64_t n, int32_t nbands);
int cd_band_partition(const cd_elements *el, const cd_params *p, int32_t nbands, double *edges,
                      uint32_t *offsets, uint32_t *members, int64_t capacity,
                      int64_t *count_host, void *ws, size_t ws_bytes, cd_stream_t stream);

/* out (device, 6 * count doubles): row d = element d (a, e, inc, raan, argp,
 * m0) of objects ids[0..count), at out + d * count.  Ids >= el->n leave their
 * column untouched.  Async. */
int cd_gather_elements(const cd_elements *el, const uint32_t *ids, int64_t count, double *out,
                       cd_stream_t stream);

/* out[r] = (min(ids[i], ids[j]), max(ids[i], ids[j]), t_lo, t_hi) for record
 * r = (i, j, t_lo, t_hi) of in (local ids < nids; others map to 0xFFFFFFFF).
 * out may alias in.  Async. */
int cd_remap_records(const cd_pair *in, int64_t count, const uint32_t *ids, int64_t nids,
                     cd_pair *out, cd_stream_t stream);

/* The canonical list of any records (sorted by i, j, t_lo, t_hi; repeats
 * removed), e.g. the bands' records merged: out[0..*count_host).  t_lo must
 * be at most horizon_ticks + 1 and ids below obj_count (both size the sort
 * keys); t_hi may take any value.  Synchronises. */
size_t cd_canonical_records_ws(int64_t count);
int cd_canonical_records(const cd_pair *in, int64_t count, uint32_t horizon_ticks,
                         uint32_t obj_count, cd_pair *out, int64_t *count_host, void *ws,
                         size_t ws_bytes, cd_stream_t stream);

/* ---- learned per-object step ------------------------------------------- */

/* The paper keeps a time interval per object so that objects far from all
 * others take long intervals (Sec. Collision Detection with 4D AABB Trees;
 * Procedure advanceTime) and leaves the step rule open.  These calls run a
 * 5 -> 64 -> 64 -> 1 ReLU network that predicts y = log2(step in seconds)
 * from x = (a/42164, e, i/pi, r_p/42164, vmax/8), r_p = a(1 - e), vmax the
 * perigee speed:
 *   h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = w3 . h2 + b3,
 *   dt = clamp(floor(2^y / tick_s), 1, max(T, 1)) ticks.
 * Parameters: one flat vector of CD_MLP_PARAMS values in the order W1 (64x5,
 * row-major), b1 (64), W2 (64x64, row-major), b2 (64), w3 (64), b3 (1).  Any
 * step keeps the boxes conservative, so the network affects cost only.
 * All pointers are device pointers unless named _host. */
#define CD_MLP_PARAMS 4609

/* x_out[i*5 + f] (FP32) = feature f of object i, computed in FP64.  Async. */
int cd_mlp_features(const cd_elements *el, const cd_params *p, float *x_out,
                    cd_stream_t stream);

/* BF16 inference: w_bf16 holds the parameters as bfloat16 bit patterns;
 * inputs and hidden activations are rounded to bfloat16, sums are FP32.
 * dt_out[i] = the decoded step; where y is not finite, or w_bf16 is NULL, the
 * cd_dt_heuristic step for fallback_disp_km is used.  y_out (nullable)
 * receives y (NaN for every object when w_bf16 is NULL).  Async. */
int cd_dt_mlp(const cd_elements *el, const uint16_t *w_bf16, double fallback_disp_km,
              const cd_params *p, uint32_t *dt_out, float *y_out, cd_stream_t stream);

/* FP32 forward pass: y_out[b] for x[b*5 .. b*5+4], w FP32 parameters.  Async. */
int cd_mlp_forward(const float *w, const float *x, int64_t batch, float *y_out,
                   cd_stream_t stream);

/* FP32 loss L = mean_b (y_b - target_b)^2 and its gradient with respect to
 * every parameter (grad_out[CD_MLP_PARAMS], same order as w); *loss_out is a
 * device float (nullable).  The batch sum is taken per block of samples and
 * the block partials are added in a fixed order: results are deterministic.
 * 1 <= batch < 2^31.  Async. */
size_t cd_mlp_grad_ws(int64_t batch);
int cd_mlp_grad(const float *w, const float *x, const float *target, int64_t batch,
                float *grad_out, float *loss_out, void *ws, size_t ws_bytes, cd_stream_t stream);

/* One Adam step (Kingma & Ba, bias-corrected moments) in place on w, m, v
 * (FP32, CD_MLP_PARAMS each) for gradient g; step >= 1 counts from 1.  If
 * w_bf16_out is not NULL it receives the updated weights rounded to bfloat16
 * (nearest, ties to even).  Async. */
int cd_mlp_adam(float *w, float *m, float *v, const float *g, int64_t step, float lr,
                float beta1, float beta2, float eps, uint16_t *w_bf16_out, cd_stream_t stream);

/* counts_out[o] = number of records of pairs[0..count) naming object o (as i
 * or j), o < n; names >= n are ignored.  Async. */
int cd_pair_object_counts(const cd_pair *pairs, int64_t count, int64_t n, uint32_t *counts_out,
                          cd_stream_t stream);

#ifdef __cplusplus
}
#endif
#endif
