// cd_api.cpp -- the C ABI of include/cd4d.h: argument checks, workspace
// layout and the order of launches.  All arithmetic runs in the kernels.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <mutex>
#include <new>
#include <vector>

#include "cd_internal.h"

using namespace cd;

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

}  // namespace

namespace cd {
// The thread-local error message, for the entry points defined in other
// translation units.
int set_error(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}
}  // namespace cd

namespace {

#define CD_HIP(x)                                                                          \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess)                                                              \
            return fail(CD_E_DEVICE, "%s failed: %s", #x, hipGetErrorString(e_));           \
    } while (0)

// CD_DEBUG_SYNC=1 (read once): every call that enqueues work waits for it and
// reports at once what would otherwise surface at a later synchronising call
// -- a HIP error, the build's error bits in a tree header, the status word of
// a device-count query.  Nothing is checked while the stream records a graph.
bool debug_sync_on()
{
    static const bool on = [] {
        const char *v = getenv("CD_DEBUG_SYNC");
        return v && *v && strcmp(v, "0") != 0;
    }();
    return on;
}

int debug_sync(hipStream_t s, const char *what, const unsigned int *tree_err = nullptr,
               const unsigned int *status_dev = nullptr)
{
    if (!debug_sync_on())
        return CD_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
        return CD_OK;
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess)
        e = hipGetLastError();
    if (e != hipSuccess)
        return fail(CD_E_DEVICE, "%s: %s (CD_DEBUG_SYNC)", what, hipGetErrorString(e));
    unsigned int v[2] = {0, 0};
    if (tree_err && (e = hipMemcpy(&v[0], tree_err, sizeof v[0], hipMemcpyDeviceToHost)) != hipSuccess)
        return fail(CD_E_DEVICE, "%s: reading the tree header: %s", what, hipGetErrorString(e));
    if (status_dev &&
        (e = hipMemcpy(&v[1], status_dev, sizeof v[1], hipMemcpyDeviceToHost)) != hipSuccess)
        return fail(CD_E_DEVICE, "%s: reading the status: %s", what, hipGetErrorString(e));
    if (v[0] || (v[1] & 2u))
        return fail(CD_E_INVALID, "%s: tree inconsistent (error bits 0x%x) (CD_DEBUG_SYNC)", what,
                    v[0] ? v[0] : v[1]);
    if (v[1] & 1u)
        return fail(CD_E_CAPACITY, "%s: more records than the capacity (CD_DEBUG_SYNC)", what);
    return CD_OK;
}

// ---- stage timing (cd_profile_*) ----
struct ProfPending {
    const char *name;
    hipEvent_t a, b;
};
struct ProfTotal {
    const char *name;
    double ms;
    int64_t launches;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfPending> g_prof_pending;
std::vector<hipEvent_t> g_prof_pool;
std::vector<ProfTotal> g_prof_totals;

hipEvent_t prof_event()
{
    if (!g_prof_pool.empty()) {
        hipEvent_t e = g_prof_pool.back();
        g_prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess)
        return nullptr;
    return e;
}

// Records an event pair around a stage when profiling is on.
struct Stage {
    const char *name;
    hipStream_t s;
    hipEvent_t a = nullptr;
    Stage(const char *n, hipStream_t st) : name(n), s(st)
    {
        std::lock_guard<std::mutex> g(g_prof_mu);
        if (!g_prof_on)
            return;
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
            return;   // no timing inside a graph
        a = prof_event();
        if (a && hipEventRecord(a, s) != hipSuccess) {
            g_prof_pool.push_back(a);
            a = nullptr;
        }
    }
    ~Stage()
    {
        if (!a)
            return;
        std::lock_guard<std::mutex> g(g_prof_mu);
        hipEvent_t b = prof_event();
        if (b && hipEventRecord(b, s) == hipSuccess)
            g_prof_pending.push_back({name, a, b});
        else {
            g_prof_pool.push_back(a);
            if (b)
                g_prof_pool.push_back(b);
        }
    }
};

// ---- launch shapes (cd_set_tuning): per calling thread ----
constexpr cd_tuning kDefaultTuning = {2048, 256, 256, 0, 96};
thread_local cd_tuning g_tune = kDefaultTuning;

cd_tuning tuning() { return g_tune; }

constexpr int64_t kMaxBoxes = (1ll << 30) - 1;  // node ids of 2N - 1 nodes below 2^31
constexpr size_t kTreeHeader = sizeof(TreeHeader);
constexpr int kExpandBatch = 12;                 // levels launched between count checks
constexpr int kExpandMaxLevels = 400;            // > 2 x the deepest possible tree
// Query control block (32-bit words): [l] queue count after level l - 1
// ([0] stays zero), then the per-leaf-walk flag, the level flags, the
// one-launch traversal's arrival counter, a status copy (record count
// low/high, tree error) at an 8-byte-aligned word, and the result of a small
// canonical list formed before the host read the count.
constexpr int kCtlWalk = kExpandMaxLevels + 1;
constexpr int kCtlFlags = kExpandMaxLevels + 2;
constexpr int kCtlBarrier = kExpandMaxLevels + 3;
constexpr int kCtlStatus = kExpandMaxLevels + 4;
constexpr int kCtlCanon = kCtlStatus + 3;   // small canonical list done: records + 1
constexpr int kCtlWords = kCtlStatus + 4;
// Node-pair levels the last drained traversal needed: the next synchronous
// query launches that many before its first count check.
std::atomic<int> g_expand_levels{kExpandBatch};
// Node-pair levels the calling thread's last synchronous query needed to
// drain its queue (0: the per-leaf walk ran, or no query yet).
thread_local int g_last_levels = 0;
// Raw record count of the calling thread's last synchronous query: when it
// fits the one-workgroup canonical list (or the tile-and-merge path, with a
// quarter to spare), the next query forms that list right after its
// node-pair levels, before the host reads the count, which saves a round
// trip to the host.
thread_local unsigned long long g_last_records = 0;

int check_params(const cd_params *p)
{
    if (!p)
        return fail(CD_E_INVALID, "params is NULL");
    if (!(p->tick_s > 0.0) || !isfinite(p->tick_s))
        return fail(CD_E_INVALID, "tick_s must be finite and > 0");
    if (!(p->mu > 0.0) || !isfinite(p->mu))
        return fail(CD_E_INVALID, "mu must be finite and > 0");
    if (!(p->threshold_km >= 0.0) || !isfinite(p->threshold_km))
        return fail(CD_E_INVALID, "threshold_km must be finite and >= 0");
    if (p->horizon_ticks == 0xFFFFFFFFu)
        return fail(CD_E_OVERFLOW, "horizon_ticks + 1 must fit 32 bits");
    if (p->box_rule > CD_BOX_INTERVAL_E)
        return fail(CD_E_INVALID, "unknown box_rule %u", p->box_rule);
    return CD_OK;
}

int check_elements(const cd_elements *el)
{
    if (!el)
        return fail(CD_E_INVALID, "elements is NULL");
    if (el->n < 0)
        return fail(CD_E_INVALID, "n < 0");
    if (el->n >= (1ll << 31))
        return fail(CD_E_OVERFLOW, "n must be < 2^31");
    if (el->n > 0 && (!el->a || !el->e || !el->inc || !el->raan || !el->argp || !el->m0))
        return fail(CD_E_INVALID, "element array is NULL");
    return CD_OK;
}

uint64_t intervals(uint32_t dt, uint32_t T) { return T == 0 ? 1 : ((uint64_t)T + dt - 1) / dt; }

int bits_for(uint64_t v)  // bits needed to hold values 0..v
{
    int b = 0;
    while (b < 64 && (v >> b) != 0)
        ++b;
    return b;
}

BoxView view_of(const cd_boxes *b)
{
    BoxView v;
    for (int d = 0; d < 3; ++d) {
        v.lo[d] = b->lo[d];
        v.hi[d] = b->hi[d];
    }
    v.t0 = b->t0;
    v.t1 = b->t1;
    v.obj = b->obj;
    v.code = (b->code && b->code_valid) ? b->code : nullptr;
    return v;
}

// Time field of the key when the boxes carry no slab hint (per-object steps,
// caller-built boxes): 64 slabs over the horizon.  Narrow slabs leave nearly
// every box straddling a slab edge, and the traversal then joins neighbouring
// slabs through union boxes that span all of space; measured on the tracked
// hour with 5 km steps, T/4096 -> T/64 cut the query from 34.6 to 20.1 ms.
uint32_t default_slab(uint32_t horizon) { return horizon / 64u > 0 ? horizon / 64u : 1u; }

// ---- workspace layouts (shared by the *_ws queries and the calls) ----

struct CountWS {
    ObjSteps *st;
    uint32_t *Kc;
    unsigned long long *total;
    unsigned int *bad;
};
size_t layout_count(void *base, size_t bytes, int64_t n, CountWS *w)
{
    Carve c(base, bytes);
    w->st = c.take<ObjSteps>(n);
    w->Kc = c.take<uint32_t>(n);
    w->total = c.take<unsigned long long>(1);
    w->bad = c.take<unsigned int>(1);
    return c.off;
}

struct BoxWS {
    CountWS cnt;
    ObjConst *oc;
    ObjSinus *os;
    uint32_t *box_off;
    unsigned long long *frame;
    void *scan;
};
size_t layout_boxes(void *base, size_t bytes, int64_t n, BoxWS *w)
{
    size_t off = layout_count(base, bytes, n, &w->cnt);
    Carve c(base, bytes);
    c.off = off;
    w->oc = c.take<ObjConst>(n);
    w->os = c.take<ObjSinus>(n);
    w->box_off = c.take<uint32_t>(n);
    w->frame = c.take<unsigned long long>(6);
    w->scan = c.take_bytes(scan_ws_bytes((size_t)n));
    return c.off;
}

struct TreeWS {
    KV *kva, *kvb;          // key sort items (16-byte pairs or 8-byte words)
    uint64_t *keys;         // slab build: sorted codes
    uint32_t *parent, *arrive, *list_items, *list_count;
    uint8_t *clev;
    void *agglo;            // bottom-up build
    uint32_t *esc;   // escapes of an FP64 tree's nodes, for the refit
    unsigned long long *bounds;
    void *radix;
};
size_t layout_tree(void *base, size_t bytes, int64_t N, TreeWS *w)
{
    Carve c(base, bytes);
    size_t n = (size_t)(N > 0 ? N : 1);
    w->kva = c.take<KV>(n);
    w->kvb = c.take<KV>(n);
    w->keys = c.take<uint64_t>(n);
    w->parent = c.take<uint32_t>(2 * n);
    w->arrive = c.take<uint32_t>(n);
    size_t slots = refit_list_slots((uint32_t)n, nullptr) + 1;
    w->list_items = c.take<uint32_t>(slots * kRefitListCap);
    w->list_count = c.take<uint32_t>(slots);
    w->clev = c.take<uint8_t>(n);
    w->agglo = c.take_bytes(agglo_ws_bytes((uint32_t)n));
    w->esc = c.take<uint32_t>(2 * n);
    w->bounds = c.take<unsigned long long>(6);
    w->radix = c.take_bytes(radix_ws_bytes(n));
    return c.off;
}

struct QueryWS {
    Rec *raw, *alt;
    unsigned long long *counter;
    uint32_t *flags, *pos;
    void *scan, *radix;
    uint2 *qa, *qb;
    unsigned int *qcount, *qflags;
    uint32_t qcap;
};
// Radix passes of the canonical order (i, j, t_lo, t_hi), least significant
// field first, over the bits each field can use.
DigitPlan record_plan_bits(uint32_t horizon_ticks, uint32_t obj_count)
{
    int tb = bits_for((uint64_t)horizon_ticks + 1);
    int ob = obj_count ? bits_for((uint64_t)obj_count - 1) : 32;
    DigitPlan plan;
    memset(&plan, 0, sizeof plan);
    const int fields[4] = {3, 2, 1, 0};  // t_hi, t_lo, j, i
    // t_lo is some box's t0 (at most the horizon); t_hi some box's t1, which
    // caller-built boxes may put past it: all 32 bits
    const int widths[4] = {32, tb, ob, ob};
    for (int f = 0; f < 4; ++f)
        for (int sh = 0; sh < widths[f]; sh += 8) {
            plan.field[plan.npass] = (uint8_t)fields[f];
            plan.shift[plan.npass] = (uint8_t)sh;
            ++plan.npass;
        }
    return plan;
}

DigitPlan record_plan(const cd_tree *tree)
{
    return record_plan_bits(tree->horizon_ticks, tree->obj_count);
}

// node pairs per traversal level: N covers every case seen short of boxes that
// overlap nearly everything (those overflow into the per-leaf walk)
uint32_t queue_cap(int64_t N) { return (uint32_t)(N > 65536 ? N : 65536); }
size_t layout_query(void *base, size_t bytes, int64_t N, int64_t cap, QueryWS *w)
{
    Carve c(base, bytes);
    size_t m = (size_t)(cap > 0 ? cap : 1);
    w->qcap = queue_cap(N);
    w->qa = c.take<uint2>(w->qcap);
    w->qb = c.take<uint2>(w->qcap);
    w->qcount = c.take<unsigned int>(kCtlWords);
    w->qflags = w->qcount + kCtlFlags;
    w->raw = c.take<Rec>(m);
    w->alt = c.take<Rec>(m);
    w->counter = c.take<unsigned long long>(1);
    w->flags = c.take<uint32_t>(m);
    w->pos = c.take<uint32_t>(m + 1);
    w->scan = c.take_bytes(scan_ws_bytes(m));
    w->radix = c.take_bytes(radix_ws_bytes(m));
    return c.off;
}

// Bulk interval refinement: control words [l] = queue count before level l,
// then the level flags and a status copy (leaf count low/high, flags, last
// queue count).
constexpr int kRefineMaxLevels = 40;      // > log2(2^32 instants) + 2
constexpr int kRefCtlFlags = kRefineMaxLevels + 1;
constexpr int kRefCtlStatus = kRefineMaxLevels + 4;
constexpr int kRefCtlWords = kRefCtlStatus + 4;

struct RefineWS {
    ObjConst *oc;
    ObjSinus *os;
    uint4 *qa, *qb;
    unsigned int *ctl;
    Rec *raw, *alt;
    unsigned long long *counter;
    uint32_t *flags, *pos;
    void *scan, *radix;
    uint32_t qcap;
};
// work items per level: the records twice over, the output capacity, or 2^16
uint32_t refine_queue_cap(int64_t count, int64_t capacity)
{
    uint64_t q = (uint64_t)(count > 0 ? count : 0) * 2;
    if ((uint64_t)capacity > q)
        q = (uint64_t)capacity;
    if (q < 65536)
        q = 65536;
    return (uint32_t)(q < 0xFFFFFFF0ull ? q : 0xFFFFFFF0ull);
}
size_t layout_refine(void *base, size_t bytes, int64_t n, int64_t count, int64_t cap,
                     RefineWS *w)
{
    Carve c(base, bytes);
    size_t m = (size_t)(cap > 0 ? cap : 1);
    size_t no = (size_t)(n > 0 ? n : 1);
    w->qcap = refine_queue_cap(count, cap);
    w->oc = c.take<ObjConst>(no);
    w->os = c.take<ObjSinus>(no);
    w->qa = c.take<uint4>(w->qcap);
    w->qb = c.take<uint4>(w->qcap);
    w->ctl = c.take<unsigned int>(kRefCtlWords);
    w->raw = c.take<Rec>(m);
    w->alt = c.take<Rec>(m);
    w->counter = c.take<unsigned long long>(1);
    w->flags = c.take<uint32_t>(m);
    w->pos = c.take<uint32_t>(m + 1);
    w->scan = c.take_bytes(scan_ws_bytes(m));
    w->radix = c.take_bytes(radix_ws_bytes(m));
    return c.off;
}

// Potential-collision graph by altitude bands.
constexpr int kMaxBands = 4096;
double band_pad(const cd_params *p) { return sqrt(3.0) * 0.5 * p->threshold_km; }

struct BandWS {
    KV *ka, *kb;
    uint32_t *cnt, *off;
    void *scan, *radix;
};
size_t layout_bands(void *base, size_t bytes, int64_t n, int64_t nbands, BandWS *w)
{
    Carve c(base, bytes);
    size_t no = (size_t)(n > 0 ? n : 1);
    size_t m = no * (size_t)(nbands > 0 ? nbands : 1);   // memberships: at most n per band
    w->ka = c.take<KV>(m);
    w->kb = c.take<KV>(m);
    w->cnt = c.take<uint32_t>(no + 1);
    w->off = c.take<uint32_t>(no + 1);
    w->scan = c.take_bytes(scan_ws_bytes(no + 1));
    w->radix = c.take_bytes(radix_ws_bytes(m));
    return c.off;
}

struct RecWS {
    Rec *raw, *alt;
    uint32_t *flags, *pos;
    void *scan, *radix;
};
size_t layout_records(void *base, size_t bytes, int64_t count, RecWS *w)
{
    Carve c(base, bytes);
    size_t m = (size_t)(count > 0 ? count : 1);
    w->raw = c.take<Rec>(m);
    w->alt = c.take<Rec>(m);
    w->flags = c.take<uint32_t>(m + 1);
    w->pos = c.take<uint32_t>(m + 1);
    w->scan = c.take_bytes(scan_ws_bytes(m + 1));
    w->radix = c.take_bytes(radix_ws_bytes(m));
    return c.off;
}

} // namespace

extern "C" {

const char *cd_status_string(int status)
{
    switch (status) {
    case CD_OK: return "ok";
    case CD_E_INVALID: return "invalid argument";
    case CD_E_WORKSPACE: return "workspace too small";
    case CD_E_CAPACITY: return "output capacity too small";
    case CD_E_OVERFLOW: return "size does not fit 32 bits";
    case CD_E_DEVICE: return "HIP runtime error";
    default: return "unknown status";
    }
}

const char *cd_last_error(void) { return g_err; }

int cd_version(void) { return 1; }

int cd_stream_copy(void *dst, const void *src, size_t bytes, cd_stream_t stream)
{
    if (bytes == 0)
        return CD_OK;
    if (!dst || !src)
        return fail(CD_E_INVALID, "dst or src is NULL");
    if ((bytes & 15u) || ((uintptr_t)dst & 15u) || ((uintptr_t)src & 15u))
        return fail(CD_E_INVALID, "copy size and addresses must be multiples of 16 bytes");
    const char *a = (const char *)src, *b = (const char *)dst;
    if (a < b + bytes && b < a + bytes)
        return fail(CD_E_INVALID, "source and destination overlap");
    CD_HIP(launch_stream_copy(src, dst, (uint64_t)(bytes / 16), (hipStream_t)stream));
    return debug_sync((hipStream_t)stream, "cd_stream_copy");
}

int cd_profile_enable(int on)
{
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof_on = on != 0;
    return CD_OK;
}

int cd_profile_read(const char **names, double *ms_total, int64_t *launches, int max, int reset)
{
    std::lock_guard<std::mutex> g(g_prof_mu);
    for (auto &p : g_prof_pending) {
        float ms = 0.0f;
        if (hipEventSynchronize(p.b) != hipSuccess || hipEventElapsedTime(&ms, p.a, p.b) !=
                                                          hipSuccess)
            return fail(CD_E_DEVICE, "reading stage events failed");
        bool found = false;
        for (auto &t : g_prof_totals)
            if (strcmp(t.name, p.name) == 0) {
                t.ms += ms;
                t.launches += 1;
                found = true;
            }
        if (!found)
            g_prof_totals.push_back({p.name, (double)ms, 1});
        g_prof_pool.push_back(p.a);
        g_prof_pool.push_back(p.b);
    }
    g_prof_pending.clear();
    int n = (int)g_prof_totals.size();
    for (int k = 0; k < n && k < max; ++k) {
        if (names)
            names[k] = g_prof_totals[k].name;
        if (ms_total)
            ms_total[k] = g_prof_totals[k].ms;
        if (launches)
            launches[k] = g_prof_totals[k].launches;
    }
    if (reset)
        g_prof_totals.clear();
    return n;
}

// ---- step 1 -----------------------------------------------------------------------------

size_t cd_box_count_ws(int64_t n)
{
    CountWS w;
    return layout_count(nullptr, 0, n > 0 ? n : 0, &w);
}

int cd_box_count(const uint32_t *dt_ticks, int64_t n, const cd_params *p, int64_t *count_host,
                 void *ws, size_t ws_bytes, cd_stream_t stream)
{
    int rc = check_params(p);
    if (rc)
        return rc;
    if (!count_host)
        return fail(CD_E_INVALID, "count_host is NULL");
    if (n < 0)
        return fail(CD_E_INVALID, "n < 0");
    if (n >= (1ll << 31))
        return fail(CD_E_OVERFLOW, "n must be < 2^31");
    *count_host = 0;
    if (n == 0)
        return CD_OK;
    uint64_t total;
    if (!dt_ticks) {
        if (p->dt_ticks == 0)
            return fail(CD_E_INVALID, "dt_ticks must be >= 1");
        total = (uint64_t)n * intervals(p->dt_ticks, p->horizon_ticks);
    } else {
        if (ws_bytes < cd_box_count_ws(n) || !ws)
            return fail(CD_E_WORKSPACE, "box-count workspace too small");
        hipStream_t s = (hipStream_t)stream;
        CountWS w;
        layout_count(ws, ws_bytes, n, &w);
        CD_HIP(launch_steps(dt_ticks, (uint32_t)n, p->horizon_ticks, w.st, w.Kc, w.total, w.bad,
                            s));
        unsigned long long h[1];
        unsigned int bad = 0;
        CD_HIP(hipMemcpyAsync(h, w.total, sizeof h, hipMemcpyDeviceToHost, s));
        CD_HIP(hipMemcpyAsync(&bad, w.bad, sizeof bad, hipMemcpyDeviceToHost, s));
        CD_HIP(hipStreamSynchronize(s));
        if (bad)
            return fail(CD_E_INVALID, "a per-object dt_ticks is 0");
        total = h[0];
    }
    if (total > (uint64_t)kMaxBoxes)
        return fail(CD_E_OVERFLOW, "box count %llu exceeds 2^31 - 1",
                    (unsigned long long)total);
    *count_host = (int64_t)total;
    return CD_OK;
}

size_t cd_validate_ws(int64_t n) { return 256; }

int cd_validate_elements(const cd_elements *el, int64_t *bad_index_host, void *ws,
                         size_t ws_bytes, cd_stream_t stream)
{
    int rc = check_elements(el);
    if (rc)
        return rc;
    if (!bad_index_host)
        return fail(CD_E_INVALID, "bad_index_host is NULL");
    *bad_index_host = -1;
    if (el->n == 0)
        return CD_OK;
    if (!ws || ws_bytes < cd_validate_ws(el->n))
        return fail(CD_E_WORKSPACE, "validate workspace too small");
    hipStream_t s = (hipStream_t)stream;
    unsigned long long *first = (unsigned long long *)ws;
    CD_HIP(launch_validate(*el, first, s));
    unsigned long long h = 0;
    CD_HIP(hipMemcpyAsync(&h, first, sizeof h, hipMemcpyDeviceToHost, s));
    CD_HIP(hipStreamSynchronize(s));
    if (h != ~0ull) {
        *bad_index_host = (int64_t)h;
        return fail(CD_E_INVALID, "object %llu has invalid elements (need finite, a > 0, "
                                  "0 <= e < 1)", h);
    }
    return CD_OK;
}

int cd_dt_heuristic(const cd_elements *el, const cd_params *p, double max_disp_km,
                    uint32_t *dt_out, cd_stream_t stream)
{
    int rc = check_elements(el);
    if (!rc)
        rc = check_params(p);
    if (rc)
        return rc;
    if (!(max_disp_km > 0.0) || !isfinite(max_disp_km))
        return fail(CD_E_INVALID, "max_disp_km must be finite and > 0");
    if (el->n > 0 && !dt_out)
        return fail(CD_E_INVALID, "dt_out is NULL");
    CD_HIP(launch_dt_heuristic(*el, p->mu, p->tick_s, max_disp_km, p->horizon_ticks, dt_out,
                               (hipStream_t)stream));
    return debug_sync((hipStream_t)stream, "cd_dt_heuristic");
}

// ---- step 2 -----------------------------------------------------------------------------

size_t cd_build_boxes_ws(int64_t n)
{
    BoxWS w;
    return layout_boxes(nullptr, 0, n > 0 ? n : 0, &w);
}

int cd_build_boxes(const cd_elements *el, const uint32_t *dt_ticks, const cd_params *p,
                   cd_boxes *out, void *ws, size_t ws_bytes, cd_stream_t stream)
{
    int rc = check_elements(el);
    if (!rc)
        rc = check_params(p);
    if (rc)
        return rc;
    if (!out)
        return fail(CD_E_INVALID, "out is NULL");
    if (out->precision != CD_FP64 && out->precision != CD_FP32)
        return fail(CD_E_INVALID, "unknown box precision %d", out->precision);
    if (out->count < 0 || out->count > kMaxBoxes)
        return fail(CD_E_OVERFLOW, "box count out of range");
    int64_t n = el->n;
    uint32_t T = p->horizon_ticks;
    out->horizon_ticks = T;
    out->obj_count = (uint32_t)n;
    out->slab_size = 0;
    out->slab_ticks = 0;
    if (out->layout != CD_LAYOUT_OBJECT && out->layout != CD_LAYOUT_SORTED)
        return fail(CD_E_INVALID, "unknown box layout %d", out->layout);
    if (n == 0) {
        if (out->count != 0)
            return fail(CD_E_INVALID, "out->count must be 0 for n = 0");
        out->layout = CD_LAYOUT_OBJECT;
        return CD_OK;
    }
    if (out->records) {
        if (out->precision != CD_FP64)
            return fail(CD_E_INVALID, "box records are FP64");
        if (!out->code)
            return fail(CD_E_INVALID, "box records need the packed code array too");
        if (dt_ticks)
            return fail(CD_E_INVALID, "box records need a uniform step");
        if ((uintptr_t)out->records & 15u)
            return fail(CD_E_INVALID, "box records must be 16-byte aligned");
    } else if (out->count > 0) {
        for (int d = 0; d < 3; ++d)
            if (!out->lo[d] || !out->hi[d])
                return fail(CD_E_INVALID, "box array is NULL");
        if (!out->t0 || !out->t1 || !out->obj)
            return fail(CD_E_INVALID, "box tag array is NULL");
    }
    if (!ws || ws_bytes < cd_build_boxes_ws(n))
        return fail(CD_E_WORKSPACE, "build-boxes workspace too small");
    hipStream_t s = (hipStream_t)stream;
    BoxWS w;
    layout_boxes(ws, ws_bytes, n, &w);
    BoxOut bo;
    for (int d = 0; d < 3; ++d) {
        bo.lo[d] = out->lo[d];
        bo.hi[d] = out->hi[d];
    }
    bo.t0 = out->t0;
    bo.t1 = out->t1;
    bo.obj = out->obj;
    bo.code = out->code;
    bo.frame = w.frame;
    bo.cap = (uint64_t)out->count;
    bo.rec = (Node64 *)out->records;
    out->code_valid = 0;
    Stage st_boxes("boxes", s);
    const bool frame = bo.code || bo.rec;
    CD_HIP(launch_object_setup(*el, p->mu, (double)p->start_ticks * p->tick_s, w.oc, w.os,
                               frame ? w.frame : nullptr, s));
    if (frame)
        CD_HIP(launch_orbit_frame(w.oc, (uint32_t)n, w.frame, s));
    double half_thr = 0.5 * p->threshold_km;
    if (!dt_ticks) {
        if (p->dt_ticks == 0)
            return fail(CD_E_INVALID, "dt_ticks must be >= 1");
        uint64_t K = intervals(p->dt_ticks, T);
        if ((uint64_t)n * K != (uint64_t)out->count)
            return fail(CD_E_INVALID, "out->count %lld != n * K = %llu", (long long)out->count,
                        (unsigned long long)((uint64_t)n * K));
        bool sorted = out->layout == CD_LAYOUT_SORTED && (bo.code || bo.rec) &&
                      (n <= kSegCap || (bo.rec && n <= kSortedMaxObjects));
        if (bo.rec && !sorted)
            return fail(CD_E_INVALID, "box records need the sorted layout (CD_LAYOUT_SORTED, "
                                      "n <= %lld)", (long long)kSortedMaxObjects);
        CD_HIP(launch_boxes_uniform(w.oc, w.os, (uint32_t)n, (uint32_t)K, p->dt_ticks, T,
                                    p->tick_s, half_thr, out->precision, (int)p->box_rule,
                                    sorted, bo, s));
        out->slab_ticks = p->dt_ticks;
        out->slab_size = n;
        out->layout = sorted ? CD_LAYOUT_SORTED : CD_LAYOUT_OBJECT;
    } else {
        CD_HIP(launch_steps(dt_ticks, (uint32_t)n, T, w.cnt.st, w.cnt.Kc, w.cnt.total, w.cnt.bad,
                            s));
        CD_HIP(scan_exclusive_u32(w.cnt.Kc, w.box_off, (size_t)n, w.scan, s));
        CD_HIP(launch_steps_apply_offsets(w.cnt.st, w.box_off, (uint32_t)n, s));
        // out->count is the caller's box count; lanes past the real total return
        CD_HIP(launch_boxes_variable(w.oc, w.os, w.cnt.st, (uint32_t)n, T, p->tick_s, half_thr,
                                     out->precision, (int)p->box_rule, bo, s));
        out->layout = CD_LAYOUT_OBJECT;
    }
    out->code_valid = (bo.code || bo.rec) ? 1 : 0;
    return debug_sync((hipStream_t)stream, "cd_build_boxes");
}

// ---- step 3 -----------------------------------------------------------------------------

size_t cd_tree_bytes(int64_t count, int precision)
{
    if (count <= 0)
        return kTreeHeader;
    return tree_leaf_esc_offset((uint64_t)count, precision) +
           (precision == CD_FP64 ? (size_t)count * sizeof(uint32_t) : 0);
}

void *cd_tree_leaf_records(void *tree_mem, int64_t count)
{
    if (!tree_mem || count < 1)
        return nullptr;
    return (char *)tree_mem + kTreeHeader + (size_t)(count - 1) * sizeof(Node64);
}

size_t cd_build_tree_ws(int64_t count)
{
    TreeWS w;
    return layout_tree(nullptr, 0, count > 0 ? count : 0, &w);
}

int cd_build_tree(const cd_boxes *boxes, int precision, uint32_t slab_ticks, cd_tree *tree,
                  void *ws, size_t ws_bytes, cd_stream_t stream)
{
    if (!boxes || !tree)
        return fail(CD_E_INVALID, "boxes or tree is NULL");
    if (precision != CD_FP64 && precision != CD_FP32)
        return fail(CD_E_INVALID, "unknown tree precision %d", precision);
    if (boxes->precision != CD_FP64 && boxes->precision != CD_FP32)
        return fail(CD_E_INVALID, "unknown box precision %d", boxes->precision);
    if (boxes->precision == CD_FP32 && precision == CD_FP64)
        return fail(CD_E_INVALID, "an FP64 tree needs FP64 boxes");
    int64_t N = boxes->count;
    if (N < 0)
        return fail(CD_E_INVALID, "box count < 0");
    if (N > kMaxBoxes)
        return fail(CD_E_OVERFLOW, "box count exceeds 2^31 - 1");
    if (!tree->mem || tree->bytes < cd_tree_bytes(N, precision))
        return fail(CD_E_WORKSPACE, "tree buffer too small (%zu < %zu)", tree->bytes,
                    cd_tree_bytes(N, precision));
    if (boxes->records) {
        // box records written into this tree's leaf-record area
        if (boxes->records != cd_tree_leaf_records(tree->mem, N))
            return fail(CD_E_INVALID, "box records must be the tree's own leaf records");
        if (boxes->precision != CD_FP64 || precision != CD_FP64)
            return fail(CD_E_INVALID, "box records need FP64 boxes and an FP64 tree");
        if (!boxes->code)
            return fail(CD_E_INVALID, "box records need the packed code array too");
        if (boxes->layout != CD_LAYOUT_SORTED || !boxes->code_valid || boxes->slab_size <= 0 ||
            boxes->slab_size > kSortedMaxObjects || N % boxes->slab_size != 0 ||
            (slab_ticks && slab_ticks != boxes->slab_ticks))
            return fail(CD_E_INVALID, "box records need the sorted layout of a uniform step");
    } else if (N > 0) {
        for (int d = 0; d < 3; ++d)
            if (!boxes->lo[d] || !boxes->hi[d])
                return fail(CD_E_INVALID, "box array is NULL");
        if (!boxes->t0 || !boxes->t1 || !boxes->obj)
            return fail(CD_E_INVALID, "box tag array is NULL");
    }
    if (N > 0 && (!ws || ws_bytes < cd_build_tree_ws(N)))
        return fail(CD_E_WORKSPACE, "build-tree workspace too small");
    uint32_t horizon = boxes->horizon_ticks ? boxes->horizon_ticks : 0xFFFFFFFEu;
    uint32_t w = slab_ticks ? slab_ticks
                            : (boxes->slab_ticks ? boxes->slab_ticks : default_slab(horizon));
    hipStream_t s = (hipStream_t)stream;
    unsigned int *err = (unsigned int *)tree->mem;
    void *nodes = (char *)tree->mem + kTreeHeader;
    CD_HIP(launch_fill_u32(err, 0u, kTreeHeader / 4, s));
    tree->count = N;
    tree->precision = precision;
    tree->slab_ticks = w;
    tree->horizon_ticks = horizon;
    tree->obj_count = boxes->obj_count;
    if (N == 0)
        return CD_OK;
    TreeWS tw;
    layout_tree(ws, ws_bytes, N, &tw);
    BoxView bv = view_of(boxes);
    uint32_t max_slab = horizon / w;
    bool seg = boxes->slab_size > 0 && boxes->slab_size <= kSegCap && boxes->slab_ticks == w &&
               N % boxes->slab_size == 0;
    uint2 *kids = (uint2 *)((char *)tree->mem + tree_kids_offset((uint64_t)N, precision));
    SeedSink sink;
    sink.items = (uint2 *)((char *)tree->mem + tree_seeds_offset((uint64_t)N, precision));
    sink.cap = (uint32_t)seed_cap((uint64_t)N);
    sink.hdr = (TreeHeader *)tree->mem;
    const bool in_place = boxes->records != nullptr;
    // boxes sorted within their slabs by their codes (cd_build_boxes with
    // CD_LAYOUT_SORTED) as arrays: box j is leaf j, no key sort
    const bool presorted = seg && boxes->layout == CD_LAYOUT_SORTED && bv.code;
    if (seg && !in_place && !presorted) {
        // object-order slabs: each slab sorted in one workgroup's LDS with its
        // leaf records written in sorted order, then the top-down Karras pass
        // and the refit.  FP32 trees keep their link records in the tree
        // itself; FP64 records carry them inline and take the escapes from the
        // workspace during the refit (their link word is the left child).
        LinkSink links;
        links.rec = precision == CD_FP32 ? (Link *)((Box32 *)nodes + (2 * (size_t)N - 1))
                                         : nullptr;
        links.esc = precision == CD_FP32 ? nullptr : tw.esc;
        uint32_t m = (uint32_t)boxes->slab_size;
        if (!bv.code) {
            Stage st("keys", s);
            CD_HIP(launch_bounds(bv, boxes->precision, (uint32_t)N, tw.bounds, s));
        }
        {
            Stage st("sort", s);
            CD_HIP(launch_slab_build(bv, boxes->precision, precision, (uint32_t)(N / m), m,
                                     (uint32_t)N, w, tw.bounds, (uint32_t *)tw.keys, nodes, err,
                                     s));
        }
        {
            Stage st("karras", s);
            CD_HIP(launch_karras_slabs((const uint32_t *)tw.keys, (uint32_t)N, m, kids, links,
                                       tw.parent, tw.clev, s));
        }
        {
            Stage st("refit", s);
            CD_HIP(launch_refit(precision, (uint32_t)N, tw.parent, kids, links, tw.clev,
                                tw.arrive, tw.list_items, tw.list_count, nodes, sink, err, s));
        }
        return debug_sync((hipStream_t)stream, "cd_build_tree", (const unsigned int *)tree->mem);
    }
    // every other box set: hierarchy, inner boxes and skip links in one
    // bottom-up pass; an FP64 tree's leaf skip links go to the side array
    uint32_t *side = nullptr;
    if (precision == CD_FP64) {
        side = (uint32_t *)((char *)tree->mem + tree_leaf_esc_offset((uint64_t)N, precision));
        CD_HIP(launch_fill_u32(&((TreeHeader *)tree->mem)->leaf_esc_side, 1u, 1, s));
    }
    if (in_place) {
        // the leaf records are in place (the records' code words keep the
        // codes); keys from the packed codes
        Stage st("hierarchy", s);
        CD_HIP(launch_agglo(bv.code, (uint32_t)boxes->slab_size, w, (uint32_t)N, nodes, kids,
                            side, tw.agglo, sink, err, s));
        return debug_sync((hipStream_t)stream, "cd_build_tree", (const unsigned int *)tree->mem);
    }
    AggLeafSource src{};
    if (presorted) {
        // keys from the slab of each position and the codes
        src.code = bv.code;
        src.slab_size = (uint32_t)boxes->slab_size;
        src.slab_ticks = w;
    } else {
        // per-object steps and other unsorted box sets: one key sort, the
        // boxes then read through the sorted items.  When slab, code and box
        // index fit one 64-bit word the sort moves 8-byte items instead of
        // 16-byte (key, index) pairs; box sets too large for the whole code
        // keep its top bits (at least kMinPackedCodeBits of 30)
        const int sb = bits_for(max_slab), ib = N > 1 ? bits_for((uint64_t)N - 1) : 1;
        const int room = 64 - sb - ib;
        const int cb = room < (int)kKeyCodeBits ? room : (int)kKeyCodeBits;
        const bool packed = cb >= (int)kMinPackedCodeBits;
        {
            Stage st("keys", s);
            if (!bv.code)
                CD_HIP(launch_bounds(bv, boxes->precision, (uint32_t)N, tw.bounds, s));
            CD_HIP(launch_keys(bv, boxes->precision, (uint32_t)N, w, max_slab, 0, tw.bounds,
                               nullptr, packed ? nullptr : tw.kva, err, s,
                               packed ? (uint64_t *)tw.kva : nullptr, (uint32_t)ib,
                               packed ? (uint32_t)cb : kKeyCodeBits));
        }
        void *res = nullptr;
        {
            Stage st("sort", s);
            DigitPlan plan;
            memset(&plan, 0, sizeof plan);
            if (packed) {   // code bits, then slab bits, above the box index
                for (int sh = 0; sh < cb + sb; sh += 8)
                    plan.shift[plan.npass++] = (uint8_t)(ib + sh);
            } else {        // code (low word), then slab (high word) of the key
                for (int sh = 0; sh < (int)kKeyCodeBits; sh += 8)
                    plan.shift[plan.npass++] = (uint8_t)sh;
                for (int sh = 0; sh < sb; sh += 8)
                    plan.shift[plan.npass++] = (uint8_t)(32 + sh);
            }
            if (packed)
                CD_HIP(radix_sort8(tw.kva, tw.kvb, (size_t)N, plan, tw.radix, &res, s));
            else
                CD_HIP(radix_sort16(SORT_KV, tw.kva, tw.kvb, (size_t)N, plan, tw.radix, &res,
                                    s));
        }
        src.kv = packed ? nullptr : (const KV *)res;
        src.packed = packed ? (const uint64_t *)res : nullptr;
        src.ib = (uint32_t)ib;
        src.cb = (uint32_t)(packed ? cb : kKeyCodeBits);
    }
    Stage st("hierarchy", s);
    CD_HIP(launch_agglo_gather(src, bv, boxes->precision, precision, (uint32_t)N, nodes, kids,
                               side, tw.agglo, sink, err, s));
    return debug_sync((hipStream_t)stream, "cd_build_tree", (const unsigned int *)tree->mem);
}

// ---- step 4 -----------------------------------------------------------------------------

size_t cd_query_pairs_ws(int64_t count, int64_t capacity)
{
    QueryWS w;
    return layout_query(nullptr, 0, count, capacity > 0 ? capacity : 0, &w);
}

int cd_query_pairs(const cd_tree *tree, cd_pair *out, int64_t capacity, int64_t *count_host,
                   void *ws, size_t ws_bytes, cd_stream_t stream)
{
    if (!tree || !count_host)
        return fail(CD_E_INVALID, "tree or count_host is NULL");
    if (!tree->mem || tree->count < 0)
        return fail(CD_E_INVALID, "tree is not built");
    if (tree->bytes < cd_tree_bytes(tree->count, tree->precision))
        return fail(CD_E_INVALID, "tree buffer smaller than its node count needs");
    if (capacity < 0 || capacity > 0xFFFFFFFEll)
        return fail(CD_E_INVALID, "capacity out of range");
    if (capacity > 0 && !out)
        return fail(CD_E_INVALID, "out is NULL");
    if (!ws || ws_bytes < cd_query_pairs_ws(tree->count, capacity))
        return fail(CD_E_WORKSPACE, "query workspace too small");
    *count_host = 0;
    hipStream_t s = (hipStream_t)stream;
    int64_t N = tree->count;
    unsigned int *err = (unsigned int *)tree->mem;
    const void *nodes = (const char *)tree->mem + kTreeHeader;
    QueryWS w;
    layout_query(ws, ws_bytes, N, capacity, &w);
    TreeHeader *hdr = (TreeHeader *)tree->mem;
    const unsigned int *side_on = &hdr->leaf_esc_side;
    const uint32_t *side = (const uint32_t *)((const char *)tree->mem +
                                              tree_leaf_esc_offset((uint64_t)N, tree->precision));
    const uint2 *seeds =
        (const uint2 *)((const char *)tree->mem + tree_seeds_offset((uint64_t)N, tree->precision));
    const uint2 *kids =
        (const uint2 *)((const char *)tree->mem + tree_kids_offset((uint64_t)N, tree->precision));
    const cd_tuning tu = tuning();
    unsigned int stw[3];        // record count low/high, tree error
    bool status_read = false;   // stw already read with the last control block
    unsigned int canon_done = 0;   // records + 1 of a list formed before the count was read
    {
        // the stage ends early when the small canonical list is formed with
        // the first control-block read (its own stage)
        Stage *trav = new Stage("traverse", s);
        struct StageEnd {
            Stage *&p;
            ~StageEnd() { delete p; }
        } trav_end{trav};
        // node-pair traversal from the refit's overlapping sibling pairs; a
        // build error or lost seeds (k_query_begin), a queue overflow or a bad
        // node hand the query to the per-leaf walk, decided from one read of
        // the control block per batch of levels
        bool walk = true;
        const unsigned int *run_walk = nullptr;
        status_read = false;
        g_last_levels = 0;
        if (N > 1 && tu.mode == 2) {
            // every level in one launch; the walk decided on the device
            CD_HIP(launch_fill_u32(w.qcount, 0u, kCtlWords, s));
            CD_HIP(launch_fill_u64(w.counter, 0ull, 1, s));
            CD_HIP(launch_query_begin(hdr, w.qflags, s));
            CD_HIP(launch_expand_all(nodes, kids, tree->precision, (uint32_t)N, seeds,
                                     &hdr->nseeds, (uint32_t)seed_cap((uint64_t)N), w.qa, w.qb,
                                     w.qcount, w.qcap, kExpandMaxLevels, w.raw,
                                     (unsigned long long)capacity, w.counter, w.qflags,
                                     w.qcount + kCtlBarrier, tu.expand_blocks, s));
            CD_HIP(launch_query_decide(w.qcount, w.qflags, w.counter, w.qcount + kCtlWalk, s));
            run_walk = w.qcount + kCtlWalk;
        } else if (N > 1 && tu.mode == 0) {
            CD_HIP(launch_fill_u32(w.qcount, 0u, kCtlWords, s));
            CD_HIP(launch_fill_u64(w.counter, 0ull, 1, s));
            CD_HIP(launch_query_begin(hdr, w.qflags, s));
            const uint2 *in = seeds;
            const unsigned int *n_in = &hdr->nseeds;
            uint32_t in_cap = (uint32_t)seed_cap((uint64_t)N);
            // the control block with the status copy behind it: a drained
            // traversal needs no second read
            unsigned int ctl[kCtlWords];
            int lev = 0;
            int batch = g_expand_levels.load(std::memory_order_relaxed);
            batch = batch < 1 ? 1 : (batch > kExpandMaxLevels ? kExpandMaxLevels : batch);
            unsigned int qf = 0;
            bool try_canon = true;
            const unsigned long long last = g_last_records;
            uint32_t plan = 0;   // bound of a tile-and-merge list formed early
            if (last > (unsigned long long)kSmallCanon && last <= (unsigned long long)kMediumCanon) {
                unsigned long long b = (last + last / 4 + kSmallCanon) / kSmallCanon * kSmallCanon;
                b = b < (unsigned long long)kMediumCanon ? b : (unsigned long long)kMediumCanon;
                b = b < (unsigned long long)capacity ? b : (unsigned long long)capacity;
                plan = b > (unsigned long long)kSmallCanon ? (uint32_t)b : 0u;
                try_canon = plan != 0;
            } else if (last > (unsigned long long)kSmallCanon) {
                try_canon = false;
            }
            while (lev < kExpandMaxLevels) {
                if (!trav)
                    trav = new Stage("traverse", s);
                int end = lev + batch < kExpandMaxLevels ? lev + batch : kExpandMaxLevels;
                for (; lev < end; ++lev) {
                    uint2 *outq = (lev & 1) ? w.qb : w.qa;
                    CD_HIP(launch_expand(nodes, kids, tree->precision, (uint32_t)N, in, n_in,
                                         in_cap, outq, w.qcount + lev + 1, w.qcap, w.raw,
                                         (unsigned long long)capacity, w.counter, w.qflags, 1,
                                         tu.expand_blocks, tu.expand_threads, s));
                    in = outq;
                    n_in = w.qcount + lev + 1;
                    in_cap = w.qcap;
                }
                CD_HIP(launch_query_status(w.counter, err, w.qcount + kCtlStatus, s));
                if (try_canon) {
                    // the list, if the levels drained and the count fits
                    delete trav;
                    trav = nullptr;
                    Stage c("canon", s);
                    if (plan) {
                        const DevCount g{w.counter, w.qflags, err, (uint32_t)kSmallCanon, plan};
                        CD_HIP(launch_medium_canon(w.raw, w.alt, plan, w.flags, w.pos, w.scan,
                                                   (Rec *)out, s, g, w.qcount + kCtlCanon, 1u));
                    } else {
                        CD_HIP(launch_small_canon_gated(w.raw, w.counter, w.qflags, err,
                                                        (uint32_t)capacity, (Rec *)out,
                                                        w.qcount + kCtlCanon, s));
                    }
                    try_canon = false;
                }
                CD_HIP(hipMemcpyAsync(ctl, w.qcount, sizeof ctl, hipMemcpyDeviceToHost, s));
                CD_HIP(hipStreamSynchronize(s));
                qf = ctl[kCtlFlags];
                if (qf)
                    break;
                batch = kExpandBatch;
            }
            // drained (flag 8) with no overflow, bad node or handover: done
            walk = (qf & 7u) != 0 || (qf & 8u) == 0;
            if (!walk) {
                // levels needed: the last non-empty queue's reader and the one
                // that found the queue empty
                int last = 0;
                for (int l = 1; l <= lev && l <= kExpandMaxLevels; ++l)
                    if (ctl[l])
                        last = l;
                g_expand_levels.store(last + 2, std::memory_order_relaxed);
                g_last_levels = last + 1;
                for (int k = 0; k < 3; ++k)
                    stw[k] = ctl[kCtlStatus + k];
                status_read = true;
                canon_done = ctl[kCtlCanon];
            }
        }
        if (walk) {
            if (!trav)
                trav = new Stage("traverse", s);
            // bounded fallback: one stackless walk per leaf (in mode 2 only if
            // the device decided so, from a count it cleared itself)
            if (!run_walk)
                CD_HIP(launch_fill_u64(w.counter, 0ull, 1, s));
            CD_HIP(launch_traverse(nodes, tree->precision, (uint32_t)N, tree->slab_ticks, w.raw,
                                   (unsigned long long)capacity, w.counter, err, run_walk,
                                   tu.walk_threads, side_on, side, s));
        }
    }
    if (!status_read) {
        CD_HIP(launch_query_status(w.counter, err, w.qcount + kCtlStatus, s));
        CD_HIP(hipMemcpyAsync(stw, w.qcount + kCtlStatus, sizeof stw, hipMemcpyDeviceToHost, s));
        CD_HIP(hipStreamSynchronize(s));
    }
    unsigned long long cnt = (unsigned long long)stw[0] | ((unsigned long long)stw[1] << 32);
    unsigned int e = stw[2];
    g_last_records = cnt;
    if (e)
        return fail(CD_E_INVALID, "tree inconsistent (error bits 0x%x): boxes disagree with "
                                  "their slab hint or horizon, or the build failed", e);
    *count_host = (int64_t)cnt;
    if (cnt > (unsigned long long)capacity)
        return fail(CD_E_CAPACITY, "%llu records exceed capacity %lld", cnt,
                    (long long)capacity);
    if (canon_done) {   // formed with the control block just read
        *count_host = (int64_t)(canon_done - 1);
        return CD_OK;
    }
    if (cnt == 0)
        return CD_OK;
    uint32_t count = (uint32_t)cnt;
    {
        Stage st("canon", s);
        if (count <= (uint32_t)kSmallCanon) {
            CD_HIP(launch_small_canon(w.raw, count, (Rec *)out, w.pos + count, s));
        } else if (count <= (uint32_t)kMediumCanon) {
            CD_HIP(launch_medium_canon(w.raw, w.alt, count, w.flags, w.pos, w.scan, (Rec *)out,
                                       s));
        } else {
            DigitPlan plan = record_plan(tree);
            void *res = nullptr;
            CD_HIP(radix_sort16(SORT_REC, w.raw, w.alt, count, plan, w.radix, &res, s));
            CD_HIP(launch_unique((const Rec *)res, count, w.flags, w.pos, w.scan, (Rec *)out,
                                 s));
        }
    }
    uint32_t uniq = 0;
    CD_HIP(hipMemcpyAsync(&uniq, w.pos + count, sizeof uniq, hipMemcpyDeviceToHost, s));
    CD_HIP(hipStreamSynchronize(s));
    *count_host = uniq;
    return CD_OK;
}

int cd_query_pairs_async(const cd_tree *tree, cd_pair *out, int64_t capacity,
                         unsigned long long *count_dev, unsigned int *status_dev, void *ws,
                         size_t ws_bytes, cd_stream_t stream)
{
    if (!tree || !count_dev || !status_dev)
        return fail(CD_E_INVALID, "tree, count_dev or status_dev is NULL");
    if (!tree->mem || tree->count < 0)
        return fail(CD_E_INVALID, "tree is not built");
    if (tree->bytes < cd_tree_bytes(tree->count, tree->precision))
        return fail(CD_E_INVALID, "tree buffer smaller than its node count needs");
    if (capacity < 1 || capacity > 0xFFFFFFFEll)
        return fail(CD_E_INVALID, "capacity must be in [1, 2^32 - 2]");
    if (!out)
        return fail(CD_E_INVALID, "out is NULL");
    if (!ws || ws_bytes < cd_query_pairs_ws(tree->count, capacity))
        return fail(CD_E_WORKSPACE, "query workspace too small");
    hipStream_t s = (hipStream_t)stream;
    int64_t N = tree->count;
    unsigned int *err = (unsigned int *)tree->mem;
    const void *nodes = (const char *)tree->mem + kTreeHeader;
    QueryWS w;
    layout_query(ws, ws_bytes, N, capacity, &w);
    const TreeHeader *hdr = (const TreeHeader *)tree->mem;
    const unsigned int *side_on = &hdr->leaf_esc_side;
    const uint32_t *side = (const uint32_t *)((const char *)tree->mem +
                                              tree_leaf_esc_offset((uint64_t)N, tree->precision));
    const uint2 *seeds =
        (const uint2 *)((const char *)tree->mem + tree_seeds_offset((uint64_t)N, tree->precision));
    const uint2 *kids =
        (const uint2 *)((const char *)tree->mem + tree_kids_offset((uint64_t)N, tree->precision));
    const cd_tuning tu = tuning();
    const uint32_t cap = (uint32_t)capacity;
    unsigned int *walk = w.qcount + kCtlWalk;
    CD_HIP(launch_fill_u64(w.counter, 0ull, 1, s));
    {
        Stage st("traverse", s);
        CD_HIP(launch_fill_u32(w.qcount, 0u, kCtlWords, s));
        CD_HIP(launch_fill_u32(w.qflags, tu.mode == 1 ? 4u : 0u, 1, s));
        if (N > 1 && tu.mode == 2) {
            CD_HIP(launch_query_begin(hdr, w.qflags, s));
            CD_HIP(launch_expand_all(nodes, kids, tree->precision, (uint32_t)N, seeds,
                                     &hdr->nseeds, (uint32_t)seed_cap((uint64_t)N), w.qa, w.qb,
                                     w.qcount, w.qcap, kExpandMaxLevels, w.raw, cap, w.counter,
                                     w.qflags, w.qcount + kCtlBarrier, tu.expand_blocks, s));
            // qcount[0] is never written: the flags alone decide
            CD_HIP(launch_query_decide(w.qcount, w.qflags, w.counter, walk, s));
            CD_HIP(launch_traverse(nodes, tree->precision, (uint32_t)N, tree->slab_ticks, w.raw,
                                   cap, w.counter, err, walk, tu.walk_threads, side_on, side, s));
        } else if (N > 1) {
            CD_HIP(launch_query_begin(hdr, w.qflags, s));
            const uint2 *in = seeds;
            const unsigned int *n_in = &hdr->nseeds;
            uint32_t in_cap = (uint32_t)seed_cap((uint64_t)N);
            uint32_t levels = tu.mode == 0 ? tu.max_levels : 0;
            for (uint32_t lev = 0; lev < levels; ++lev) {
                uint2 *outq = (lev & 1) ? w.qb : w.qa;
                CD_HIP(launch_expand(nodes, kids, tree->precision, (uint32_t)N, in, n_in, in_cap,
                                     outq, w.qcount + lev + 1, w.qcap, w.raw, cap, w.counter,
                                     w.qflags, 1, tu.expand_blocks, tu.expand_threads, s));
                in = outq;
                n_in = w.qcount + lev + 1;
                in_cap = w.qcap;
            }
            CD_HIP(launch_query_decide(n_in, w.qflags, w.counter, walk, s));
            CD_HIP(launch_traverse(nodes, tree->precision, (uint32_t)N, tree->slab_ticks, w.raw,
                                   cap, w.counter, err, walk, tu.walk_threads, side_on, side, s));
        }
    }
    {
        Stage st("canon", s);
        CD_HIP(launch_pad_records(w.raw, w.counter, cap, s));
        if (cap <= (uint32_t)kSmallCanon) {
            CD_HIP(launch_small_canon(w.raw, cap, (Rec *)out, w.pos + cap, s));
        } else if (cap <= (uint32_t)kMediumCanon) {
            CD_HIP(launch_medium_canon(w.raw, w.alt, cap, w.flags, w.pos, w.scan, (Rec *)out,
                                       s));
        } else {
            DigitPlan plan = record_plan(tree);
            void *res = nullptr;
            CD_HIP(radix_sort16(SORT_REC, w.raw, w.alt, cap, plan, w.radix, &res, s));
            CD_HIP(launch_unique((const Rec *)res, cap, w.flags, w.pos, w.scan, (Rec *)out, s));
        }
        CD_HIP(launch_query_finish(w.counter, err, w.pos + cap, cap, count_dev, status_dev, s));
    }
    return debug_sync((hipStream_t)stream, "cd_query_pairs_async", nullptr, status_dev);
}

int cd_last_query_levels(void) { return g_last_levels; }

int cd_counters_available(void)
{
#ifdef CD_COUNTERS
    return 1;
#else
    return 0;
#endif
}

int cd_counters_reset(uint32_t *visits, int64_t n, cd_stream_t stream)
{
#ifdef CD_COUNTERS
    if (n < 0 || n > 0xFFFFFFFFll)
        return fail(CD_E_INVALID, "n out of range");
    CD_HIP(counters_reset(visits, visits ? (uint32_t)n : 0u, (hipStream_t)stream));
    return CD_OK;
#else
    (void)visits;
    (void)n;
    (void)stream;
    return fail(CD_E_INVALID, "this library was built without CD_COUNTERS");
#endif
}

int cd_counters_read(cd_counters *out, cd_stream_t stream)
{
#ifdef CD_COUNTERS
    if (!out)
        return fail(CD_E_INVALID, "out is NULL");
    unsigned long long v[kCounterWords];
    CD_HIP(counters_read(v, (hipStream_t)stream));
    out->tests = v[0];
    out->leaf_tests = v[1];
    out->mixed_tests = v[2];
    out->leaf_hits = v[3];
    out->pairs = v[4];
    out->walk_steps = v[5];
    return CD_OK;
#else
    (void)out;
    (void)stream;
    return fail(CD_E_INVALID, "this library was built without CD_COUNTERS");
#endif
}

int cd_set_tuning(const cd_tuning *t)
{
    cd_tuning v = kDefaultTuning;
    if (t) {
        auto lanes_ok = [](uint32_t x) { return x == 0 || x == 64 || x == 128 || x == 256; };
        auto expand_ok = [&](uint32_t x) { return lanes_ok(x) || x == 512 || x == 1024; };
        if ((t->expand_blocks && (t->expand_blocks < 64 || t->expand_blocks > 65536)) ||
            !expand_ok(t->expand_threads) || !lanes_ok(t->walk_threads) || t->mode > 2 ||
            t->max_levels > (uint32_t)kExpandMaxLevels)
            return fail(CD_E_INVALID, "tuning field out of range");
        if (t->expand_blocks)
            v.expand_blocks = t->expand_blocks;
        if (t->expand_threads)
            v.expand_threads = t->expand_threads;
        if (t->walk_threads)
            v.walk_threads = t->walk_threads;
        v.mode = t->mode;
        if (t->max_levels)
            v.max_levels = t->max_levels;
    }
    g_tune = v;
    return CD_OK;
}

int cd_get_tuning(cd_tuning *t)
{
    if (!t)
        return fail(CD_E_INVALID, "t is NULL");
    *t = tuning();
    return CD_OK;
}

struct cd_graph_s {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

int cd_graph_begin(cd_stream_t stream)
{
    if (!stream)
        return fail(CD_E_INVALID, "the legacy default stream cannot be captured");
    CD_HIP(hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal));
    return CD_OK;
}

int cd_graph_end(cd_stream_t stream, cd_graph *graph_out)
{
    if (!stream || !graph_out)
        return fail(CD_E_INVALID, "stream or graph_out is NULL");
    *graph_out = nullptr;
    hipGraph_t g = nullptr;
    CD_HIP(hipStreamEndCapture((hipStream_t)stream, &g));
    hipGraphExec_t x = nullptr;
    hipError_t e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);   // the instantiate error is the one reported
        return fail(CD_E_DEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
    }
    cd_graph h = new (std::nothrow) cd_graph_s;
    if (!h) {
        (void)hipGraphExecDestroy(x);
        (void)hipGraphDestroy(g);
        return fail(CD_E_DEVICE, "out of host memory");
    }
    h->graph = g;
    h->exec = x;
    *graph_out = h;
    return CD_OK;
}

int cd_graph_launch(cd_graph graph, cd_stream_t stream)
{
    if (!graph)
        return fail(CD_E_INVALID, "graph is NULL");
    CD_HIP(hipGraphLaunch(graph->exec, (hipStream_t)stream));
    return debug_sync((hipStream_t)stream, "cd_graph_launch");
}

int cd_graph_destroy(cd_graph graph)
{
    if (!graph)
        return CD_OK;
    hipError_t a = hipGraphExecDestroy(graph->exec);
    hipError_t b = hipGraphDestroy(graph->graph);
    delete graph;
    if (a != hipSuccess || b != hipSuccess)
        return fail(CD_E_DEVICE, "graph destroy failed");
    return CD_OK;
}

int cd_first_witness(const cd_elements *el, const cd_params *p, uint32_t delta_ticks,
                     const cd_pair *pairs, int64_t count, uint32_t *witness_out,
                     unsigned long long *first_out, cd_stream_t stream)
{
    int rc = check_elements(el);
    if (!rc)
        rc = check_params(p);
    if (rc)
        return rc;
    if (delta_ticks == 0)
        return fail(CD_E_INVALID, "delta_ticks must be >= 1");
    if (count < 0)
        return fail(CD_E_INVALID, "count < 0");
    if (count > 0 && (!pairs || !witness_out))
        return fail(CD_E_INVALID, "pairs or witness_out is NULL");
    CD_HIP(launch_first_witness(*el, p->mu, p->tick_s, p->start_ticks, p->threshold_km,
                                p->horizon_ticks, delta_ticks, pairs, (uint64_t)count,
                                witness_out, first_out, (hipStream_t)stream));
    return debug_sync((hipStream_t)stream, "cd_first_witness");
}

// ---- bulk interval refinement -----------------------------------------------------------

size_t cd_refine_records_ws(int64_t n, int64_t count, int64_t capacity)
{
    RefineWS w;
    return layout_refine(nullptr, 0, n, count, capacity, &w);
}

int cd_refine_records(const cd_elements *el, const cd_params *p, uint32_t delta_ticks,
                      uint32_t min_steps, const cd_pair *pairs, int64_t count, cd_pair *out,
                      int64_t capacity, int64_t *count_host, void *ws, size_t ws_bytes,
                      cd_stream_t stream)
{
    int rc = check_elements(el);
    if (!rc)
        rc = check_params(p);
    if (rc)
        return rc;
    if (!count_host)
        return fail(CD_E_INVALID, "count_host is NULL");
    *count_host = 0;
    if (delta_ticks == 0 || min_steps == 0)
        return fail(CD_E_INVALID, "delta_ticks and min_steps must be >= 1");
    if (count < 0 || count > 0x7FFFFFFFll)
        return fail(CD_E_INVALID, "count out of range");
    if (capacity < 0 || capacity > 0xFFFFFFFEll)
        return fail(CD_E_INVALID, "capacity out of range");
    if (count > 0 && !pairs)
        return fail(CD_E_INVALID, "pairs is NULL");
    if (capacity > 0 && !out)
        return fail(CD_E_INVALID, "out is NULL");
    if (!ws || ws_bytes < cd_refine_records_ws(el->n, count, capacity))
        return fail(CD_E_WORKSPACE, "refine workspace too small");
    if (count == 0 || el->n == 0)
        return CD_OK;
    hipStream_t s = (hipStream_t)stream;
    RefineWS w;
    layout_refine(ws, ws_bytes, el->n, count, capacity, &w);
    const uint32_t T = p->horizon_ticks;
    // levels: every split halves a span, and a record holds at most T / delta + 1
    // instants, so after ceil(log2) + 2 levels every item is a leaf or dropped
    uint64_t kmax = (uint64_t)T / delta_ticks + 1;
    int levels = 2;
    while ((1ull << (levels - 2)) < kmax)
        ++levels;
    unsigned int st4[4];
    {
        Stage st("refine", s);
        CD_HIP(launch_object_setup(*el, p->mu, (double)p->start_ticks * p->tick_s, w.oc, w.os,
                                   nullptr, s));
        CD_HIP(launch_fill_u32(w.ctl, 0u, kRefCtlWords, s));
        CD_HIP(launch_fill_u32(w.ctl, (uint32_t)count, 1, s));
        CD_HIP(launch_fill_u64(w.counter, 0ull, 1, s));
        CD_HIP(launch_refine_seed(pairs, (uint32_t)count, p->start_ticks, T, delta_ticks, w.qa,
                                  s));
        for (int lev = 0; lev < levels; ++lev) {
            const uint4 *in = (lev & 1) ? w.qb : w.qa;
            uint4 *outq = (lev & 1) ? w.qa : w.qb;
            // at most count * 2^lev items reach level lev
            uint64_t most = (uint64_t)count << (lev < 32 ? lev : 32);
            if (most > w.qcap)
                most = w.qcap;
            uint32_t blocks = (uint32_t)((most + 255) / 256);
            blocks = blocks < 1 ? 1 : (blocks > 2048 ? 2048 : blocks);
            CD_HIP(launch_refine_level((int)p->box_rule, w.oc, w.os, (uint32_t)el->n, pairs, in,
                                       w.ctl + lev, w.qcap, outq, w.ctl + lev + 1, w.qcap,
                                       w.raw, (unsigned long long)capacity, w.counter,
                                       w.ctl + kRefCtlFlags, delta_ticks, min_steps, p->tick_s,
                                       0.5 * p->threshold_km, blocks, s));
        }
        CD_HIP(launch_refine_status(w.counter, w.ctl + kRefCtlFlags, w.ctl + levels,
                                    w.ctl + kRefCtlStatus, s));
        CD_HIP(hipMemcpyAsync(st4, w.ctl + kRefCtlStatus, sizeof st4, hipMemcpyDeviceToHost, s));
        CD_HIP(hipStreamSynchronize(s));
    }
    unsigned long long cnt = (unsigned long long)st4[0] | ((unsigned long long)st4[1] << 32);
    if (st4[2] & 1u) {
        // a level's work queue overflowed: ask for room for twice that many
        *count_host = 2 * (int64_t)w.qcap;
        return fail(CD_E_CAPACITY, "refinement work queue of %u items overflowed", w.qcap);
    }
    if (st4[3] != 0)
        return fail(CD_E_DEVICE, "refinement did not finish in %d levels", levels);
    *count_host = (int64_t)cnt;
    if (cnt > (unsigned long long)capacity)
        return fail(CD_E_CAPACITY, "%llu leaves exceed capacity %lld", cnt, (long long)capacity);
    if (cnt == 0)
        return CD_OK;
    uint32_t nleaf = (uint32_t)cnt;
    {
        Stage st("refine_canon", s);
        if (nleaf <= (uint32_t)kSmallCanon) {
            CD_HIP(launch_small_canon(w.raw, nleaf, (Rec *)out, w.pos + nleaf, s));
        } else if (nleaf <= (uint32_t)kMediumCanon) {
            CD_HIP(launch_medium_canon(w.raw, w.alt, nleaf, w.flags, w.pos, w.scan, (Rec *)out,
                                       s));
        } else {
            DigitPlan plan = record_plan_bits(T, (uint32_t)el->n);
            void *res = nullptr;
            CD_HIP(radix_sort16(SORT_REC, w.raw, w.alt, nleaf, plan, w.radix, &res, s));
            CD_HIP(launch_unique((const Rec *)res, nleaf, w.flags, w.pos, w.scan, (Rec *)out,
                                 s));
        }
    }
    uint32_t uniq = 0;
    CD_HIP(hipMemcpyAsync(&uniq, w.pos + nleaf, sizeof uniq, hipMemcpyDeviceToHost, s));
    CD_HIP(hipStreamSynchronize(s));
    *count_host = uniq;
    return CD_OK;
}

// ---- potential-collision graph by altitude bands ------------------------------------------

size_t cd_band_filter_ws(int64_t count)
{
    RecWS w;
    return layout_records(nullptr, 0, count, &w);
}

int cd_band_filter(const cd_elements *el, const cd_params *p, const cd_pair *pairs,
                   int64_t count, cd_pair *out, int64_t *count_host, void *ws, size_t ws_bytes,
                   cd_stream_t stream)
{
    int rc = check_elements(el);
    if (!rc)
        rc = check_params(p);
    if (rc)
        return rc;
    if (!count_host)
        return fail(CD_E_INVALID, "count_host is NULL");
    *count_host = 0;
    if (count < 0 || count > 0x7FFFFFFFll)
        return fail(CD_E_INVALID, "count out of range");
    if (count > 0 && (!pairs || !out))
        return fail(CD_E_INVALID, "pairs or out is NULL");
    if (!ws || ws_bytes < cd_band_filter_ws(count))
        return fail(CD_E_WORKSPACE, "band-filter workspace too small");
    if (count == 0)
        return CD_OK;
    hipStream_t s = (hipStream_t)stream;
    RecWS w;
    layout_records(ws, ws_bytes, count, &w);
    uint32_t m = (uint32_t)count;
    CD_HIP(launch_fill_u32(w.flags + m, 0u, 1, s));
    CD_HIP(launch_band_flags(*el, band_pad(p), pairs, m, w.flags, s));
    CD_HIP(scan_exclusive_u32(w.flags, w.pos, (size_t)m + 1, w.scan, s));
    CD_HIP(launch_compact_pairs(pairs, w.flags, w.pos, m, out, s));
    uint32_t kept = 0;
    CD_HIP(hipMemcpyAsync(&kept, w.pos + m, sizeof kept, hipMemcpyDeviceToHost, s));
    CD_HIP(hipStreamSynchronize(s));
    *count_host = kept;
    return CD_OK;
}

size_t cd_band_partition_ws(int64_t n, int32_t nbands)
{
    BandWS w;
    return layout_bands(nullptr, 0, n, nbands, &w);
}

int cd_band_partition(const cd_elements *el, const cd_params *p, int32_t nbands, double *edges,
                      uint32_t *offsets, uint32_t *members, int64_t capacity,
                      int64_t *count_host, void *ws, size_t ws_bytes, cd_stream_t stream)
{
    int rc = check_elements(el);
    if (!rc)
        rc = check_params(p);
    if (rc)
        return rc;
    if (!count_host)
        return fail(CD_E_INVALID, "count_host is NULL");
    *count_host = 0;
    if (nbands < 1 || nbands > kMaxBands)
        return fail(CD_E_INVALID, "nbands must be in [1, %d]", kMaxBands);
    if ((uint64_t)el->n * (uint64_t)nbands > 0xFFFFFFFFull)
        return fail(CD_E_OVERFLOW, "n * nbands must fit 32 bits");
    if (!edges || !offsets || (capacity > 0 && !members) || capacity < 0)
        return fail(CD_E_INVALID, "edges, offsets or members is NULL, or capacity < 0");
    if (!ws || ws_bytes < cd_band_partition_ws(el->n, nbands))
        return fail(CD_E_WORKSPACE, "band-partition workspace too small");
    hipStream_t s = (hipStream_t)stream;
    uint32_t n = (uint32_t)el->n, P = (uint32_t)nbands;
    double pad = band_pad(p);
    if (n == 0) {
        CD_HIP(launch_fill_u32(offsets, 0u, (size_t)P + 1, s));
        CD_HIP(hipStreamSynchronize(s));
        return CD_OK;
    }
    BandWS w;
    layout_bands(ws, ws_bytes, el->n, nbands, &w);
    Stage st("bands", s);
    // edges: every (n / p)-th semi-major axis in sorted order
    CD_HIP(launch_band_axis_keys(*el, w.ka, s));
    DigitPlan plan;
    memset(&plan, 0, sizeof plan);
    for (int sh = 0; sh < 64; sh += 8)
        plan.shift[plan.npass++] = (uint8_t)sh;
    void *res = nullptr;
    CD_HIP(radix_sort16(SORT_KV, w.ka, w.kb, n, plan, w.radix, &res, s));
    CD_HIP(launch_band_edges((const KV *)res, n, P, edges, s));
    // memberships: count, offsets, then the (band, object) keys sorted by band
    CD_HIP(launch_fill_u32(w.cnt + n, 0u, 1, s));
    CD_HIP(launch_band_members(*el, pad, edges, P, w.cnt, nullptr, nullptr, s));
    CD_HIP(scan_exclusive_u32(w.cnt, w.off, (size_t)n + 1, w.scan, s));
    uint32_t total = 0;
    CD_HIP(hipMemcpyAsync(&total, w.off + n, sizeof total, hipMemcpyDeviceToHost, s));
    CD_HIP(hipStreamSynchronize(s));
    *count_host = total;
    if ((int64_t)total > capacity)
        return fail(CD_E_CAPACITY, "%u memberships exceed capacity %lld", total,
                    (long long)capacity);
    CD_HIP(launch_band_members(*el, pad, edges, P, w.cnt, w.off, w.ka, s));
    memset(&plan, 0, sizeof plan);
    for (int sh = 0; sh < bits_for(n - 1 > 0 ? n - 1 : 1); sh += 8)
        plan.shift[plan.npass++] = (uint8_t)sh;
    for (int sh = 0; sh < bits_for(P - 1 > 0 ? P - 1 : 1); sh += 8)
        plan.shift[plan.npass++] = (uint8_t)(32 + sh);
    CD_HIP(radix_sort16(SORT_KV, w.ka, w.kb, total, plan, w.radix, &res, s));
    CD_HIP(launch_band_csr((const KV *)res, total, P, members, offsets, s));
    CD_HIP(hipStreamSynchronize(s));
    return CD_OK;
}

int cd_gather_elements(const cd_elements *el, const uint32_t *ids, int64_t count, double *out,
                       cd_stream_t stream)
{
    int rc = check_elements(el);
    if (rc)
        return rc;
    if (count < 0 || count > 0x7FFFFFFFll)
        return fail(CD_E_INVALID, "count out of range");
    if (count > 0 && (!ids || !out))
        return fail(CD_E_INVALID, "ids or out is NULL");
    CD_HIP(launch_gather_elements(*el, ids, (uint32_t)count, out, (hipStream_t)stream));
    return debug_sync((hipStream_t)stream, "cd_gather_elements");
}

int cd_remap_records(const cd_pair *in, int64_t count, const uint32_t *ids, int64_t nids,
                     cd_pair *out, cd_stream_t stream)
{
    if (count < 0 || count > 0x7FFFFFFFll || nids < 0 || nids > 0xFFFFFFFFll)
        return fail(CD_E_INVALID, "count or nids out of range");
    if (count > 0 && (!in || !ids || !out))
        return fail(CD_E_INVALID, "in, ids or out is NULL");
    CD_HIP(launch_remap_records(in, (uint32_t)count, ids, (uint32_t)nids, out,
                                (hipStream_t)stream));
    return debug_sync((hipStream_t)stream, "cd_remap_records");
}

size_t cd_canonical_records_ws(int64_t count)
{
    RecWS w;
    return layout_records(nullptr, 0, count, &w);
}

int cd_canonical_records(const cd_pair *in, int64_t count, uint32_t horizon_ticks,
                         uint32_t obj_count, cd_pair *out, int64_t *count_host, void *ws,
                         size_t ws_bytes, cd_stream_t stream)
{
    if (!count_host)
        return fail(CD_E_INVALID, "count_host is NULL");
    *count_host = 0;
    if (count < 0 || count > 0x7FFFFFFFll)
        return fail(CD_E_INVALID, "count out of range");
    if (count > 0 && (!in || !out))
        return fail(CD_E_INVALID, "in or out is NULL");
    if (!ws || ws_bytes < cd_canonical_records_ws(count))
        return fail(CD_E_WORKSPACE, "canonical-records workspace too small");
    if (count == 0)
        return CD_OK;
    hipStream_t s = (hipStream_t)stream;
    RecWS w;
    layout_records(ws, ws_bytes, count, &w);
    uint32_t m = (uint32_t)count;
    if (m <= (uint32_t)kSmallCanon) {
        CD_HIP(launch_small_canon((const Rec *)in, m, (Rec *)out, w.pos + m, s));
    } else if (m <= (uint32_t)kMediumCanon) {
        CD_HIP(hipMemcpyAsync(w.raw, in, (size_t)m * sizeof(Rec), hipMemcpyDeviceToDevice, s));
        CD_HIP(launch_medium_canon(w.raw, w.alt, m, w.flags, w.pos, w.scan, (Rec *)out, s));
    } else {
        CD_HIP(hipMemcpyAsync(w.raw, in, (size_t)m * sizeof(Rec), hipMemcpyDeviceToDevice, s));
        DigitPlan plan = record_plan_bits(horizon_ticks, obj_count);
        void *res = nullptr;
        CD_HIP(radix_sort16(SORT_REC, w.raw, w.alt, m, plan, w.radix, &res, s));
        CD_HIP(launch_unique((const Rec *)res, m, w.flags, w.pos, w.scan, (Rec *)out, s));
    }
    uint32_t uniq = 0;
    CD_HIP(hipMemcpyAsync(&uniq, w.pos + m, sizeof uniq, hipMemcpyDeviceToHost, s));
    CD_HIP(hipStreamSynchronize(s));
    *count_host = uniq;
    return CD_OK;
}

// ---- learned per-object step ---------------------------------------------------------

struct MlpWS {
    float *act, *part;
};
size_t layout_mlp(void *base, size_t bytes, int64_t B, MlpWS *w)
{
    Carve c(base, bytes);
    uint64_t nblk = ((uint64_t)B + kMlpOuterSamples - 1) / kMlpOuterSamples;
    w->act = c.take<float>((size_t)258 * (size_t)B);
    w->part = c.take<float>((size_t)nblk * (kMlpParams + 1));
    return c.off;
}

int cd_mlp_features(const cd_elements *el, const cd_params *p, float *x_out, cd_stream_t stream)
{
    int rc = check_elements(el);
    if (!rc)
        rc = check_params(p);
    if (rc)
        return rc;
    if (el->n > 0 && !x_out)
        return fail(CD_E_INVALID, "x_out is NULL");
    CD_HIP(launch_mlp_features(*el, p->mu, x_out, (hipStream_t)stream));
    return debug_sync((hipStream_t)stream, "cd_mlp_features");
}

int cd_dt_mlp(const cd_elements *el, const uint16_t *w_bf16, double fallback_disp_km,
              const cd_params *p, uint32_t *dt_out, float *y_out, cd_stream_t stream)
{
    int rc = check_elements(el);
    if (!rc)
        rc = check_params(p);
    if (rc)
        return rc;
    if (!(fallback_disp_km > 0.0) || !isfinite(fallback_disp_km))
        return fail(CD_E_INVALID, "fallback_disp_km must be finite and > 0");
    if (el->n > 0 && !dt_out)
        return fail(CD_E_INVALID, "dt_out is NULL");
    hipStream_t s = (hipStream_t)stream;
    if (!w_bf16) {
        CD_HIP(launch_dt_heuristic(*el, p->mu, p->tick_s, fallback_disp_km, p->horizon_ticks,
                                   dt_out, s));
        if (y_out && el->n > 0)
            CD_HIP(launch_fill_u32((uint32_t *)y_out, 0x7FC00000u, (size_t)el->n, s));
        return CD_OK;
    }
    CD_HIP(launch_dt_mlp(*el, w_bf16, p->mu, p->tick_s, fallback_disp_km, p->horizon_ticks,
                         dt_out, y_out, s));
    return debug_sync((hipStream_t)stream, "cd_dt_mlp");
}

int cd_mlp_forward(const float *w, const float *x, int64_t batch, float *y_out,
                   cd_stream_t stream)
{
    if (batch < 0 || batch >= (1ll << 31))
        return fail(CD_E_INVALID, "batch out of range");
    if (batch > 0 && (!w || !x || !y_out))
        return fail(CD_E_INVALID, "NULL pointer");
    CD_HIP(launch_mlp_forward(w, x, (uint32_t)batch, y_out, (hipStream_t)stream));
    return debug_sync((hipStream_t)stream, "cd_mlp_forward");
}

size_t cd_mlp_grad_ws(int64_t batch)
{
    MlpWS w;
    return layout_mlp(nullptr, 0, batch > 0 ? batch : 0, &w);
}

int cd_mlp_grad(const float *w, const float *x, const float *target, int64_t batch,
                float *grad_out, float *loss_out, void *ws, size_t ws_bytes, cd_stream_t stream)
{
    if (batch < 1 || batch >= (1ll << 31))
        return fail(CD_E_INVALID, "batch must be in [1, 2^31)");
    if (!w || !x || !target || !grad_out)
        return fail(CD_E_INVALID, "NULL pointer");
    if (!ws || ws_bytes < cd_mlp_grad_ws(batch))
        return fail(CD_E_WORKSPACE, "mlp workspace too small");
    MlpWS m;
    layout_mlp(ws, ws_bytes, batch, &m);
    CD_HIP(launch_mlp_grad(w, x, target, (uint32_t)batch, m.act, m.part, grad_out, loss_out,
                           (hipStream_t)stream));
    return debug_sync((hipStream_t)stream, "cd_mlp_grad");
}

int cd_mlp_adam(float *w, float *m, float *v, const float *g, int64_t step, float lr,
                float beta1, float beta2, float eps, uint16_t *w_bf16_out, cd_stream_t stream)
{
    if (!w || !m || !v || !g)
        return fail(CD_E_INVALID, "NULL pointer");
    if (step < 1)
        return fail(CD_E_INVALID, "step must be >= 1");
    if (!(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
        !(eps >= 0.0f) || !isfinite(lr) || !isfinite(eps))
        return fail(CD_E_INVALID, "Adam hyper-parameters out of range");
    CD_HIP(launch_mlp_adam(w, m, v, g, step, lr, beta1, beta2, eps, w_bf16_out,
                           (hipStream_t)stream));
    return debug_sync((hipStream_t)stream, "cd_mlp_adam");
}

int cd_pair_object_counts(const cd_pair *pairs, int64_t count, int64_t n, uint32_t *counts_out,
                          cd_stream_t stream)
{
    if (count < 0 || n < 0 || n >= (1ll << 31))
        return fail(CD_E_INVALID, "count or n out of range");
    if ((count > 0 && !pairs) || (n > 0 && !counts_out))
        return fail(CD_E_INVALID, "NULL pointer");
    if (n == 0)
        return CD_OK;
    CD_HIP(launch_pair_object_counts(pairs, (uint64_t)count, (uint32_t)n, counts_out,
                                     (hipStream_t)stream));
    return debug_sync((hipStream_t)stream, "cd_pair_object_counts");
}

} // extern "C"
