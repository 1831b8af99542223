// C ABI of the exact string matching library: argument validation, planning,
// workspace management, corpora and kernel timing. Device work is delegated to
// the launchers in sm_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sm.h"
#include "sm_internal.h"
#include "sm_trace.h"

using namespace sm;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static int fail(int status, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return status;
}

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(e_ == hipErrorOutOfMemory ? SM_ENOMEM : SM_EDEVICE, "%s: %s (%s:%d)", \
                        #expr, hipGetErrorString(e_), __FILE__, __LINE__);                 \
    } while (0)

const char *sm::sm_set_error(int status, const char *msg)
{
    fail(status, "%s", msg);
    return g_err.c_str();
}

extern "C" const char *sm_version(void) { return "sm 0.1 (gfx950)"; }
extern "C" const char *sm_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// device check: the code objects are built for gfx950 only
// ---------------------------------------------------------------------------
static int check_device()
{
    static std::mutex mu;
    static std::vector<int> ok;  // per device: 0 unknown, 1 ok, -1 bad
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> g(mu);
    if ((int)ok.size() <= dev) ok.resize(dev + 1, 0);
    if (ok[dev] == 0) {
        hipDeviceProp_t prop;
        HIP_TRY(hipGetDeviceProperties(&prop, dev));
        ok[dev] = (strncmp(prop.gcnArchName, "gfx950", 6) == 0) ? 1 : -1;
        if (ok[dev] < 0)
            return fail(SM_EDEVICE, "device %d is %s; this library is built for gfx950 only", dev,
                        prop.gcnArchName);
    }
    if (ok[dev] < 0) return fail(SM_EDEVICE, "device %d is not gfx950", dev);
    return SM_OK;
}

// ---------------------------------------------------------------------------
// planner
// ---------------------------------------------------------------------------
// Effective alphabet size from the pattern alone: the sigma for which a random
// text of that alphabet shows d distinct bytes in m draws, d the pattern's
// distinct-byte count (sigma (1 - (1 - 1/sigma)^m) = d, solved by bisection).
// m == d gives no upper bound: 256.
static int sigma_from_pattern(const uint8_t *p, uint64_t m)
{
    bool seen[256] = {false};
    int d = 0;
    for (uint64_t k = 0; k < m; k++)
        if (!seen[p[k]]) { seen[p[k]] = true; d++; }
    if ((uint64_t)d >= m) return 256;
    double lo = 1.0, hi = 256.0;
    for (int it = 0; it < 40; it++) {
        const double s = 0.5 * (lo + hi);
        const double e = s * (1.0 - std::pow(1.0 - 1.0 / s, (double)m));
        if (e < d) lo = s; else hi = s;
    }
    int s = (int)std::lround(0.5 * (lo + hi));
    return s < 1 ? 1 : s;
}

// smallest q with sigma^q >= 64 * (m - q + 1): few pattern q-grams per q-gram space
static int choose_q(uint64_t m, int sigma)
{
    if (sigma < 2) sigma = 2;
    const double ls = std::log((double)sigma);
    int q = 1;
    for (; q < Q_MAX; q++) {
        double windows = (double)(m >= (uint64_t)q ? m - q + 1 : 1);
        if (q * ls >= std::log(64.0 * windows)) break;
    }
    if (q < 2) q = 2;
    if ((uint64_t)q > m) q = (int)m;
    return q;
}

static int choose_hbits(uint64_t m, int q)
{
    uint64_t grams = m - q + 1;
    int b = 0;
    while ((1ull << b) < grams) b++;
    b += 2;
    return std::min(H_MAX, std::max(H_MIN, b));
}

namespace {
// Built-in tuning table, measured on MI355X by paper_1012_2547_amd/tune.py.
const sm_tune_entry k_builtin_tune[] = {
#include "tune_table.inc"
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0}};
std::mutex g_tune_mu;
std::vector<sm_tune_entry> g_tune;  // empty: the built-in table
bool g_tune_custom = false;

bool tune_lookup(int sigma, uint64_t m, sm_tune_entry &out)
{
    std::lock_guard<std::mutex> g(g_tune_mu);
    const sm_tune_entry *e = g_tune_custom ? g_tune.data() : k_builtin_tune;
    const size_t n = g_tune_custom ? g_tune.size() : sizeof(k_builtin_tune) / sizeof(k_builtin_tune[0]) - 1;
    for (size_t k = 0; k < n; k++)
        if (sigma >= e[k].sigma_lo && sigma <= e[k].sigma_hi && m >= e[k].m_lo && m <= e[k].m_hi) {
            out = e[k];
            return true;
        }
    return false;
}
}  // namespace

// Smallest lane_bytes the planner may choose for a pattern of length m (any sigma).
static int min_auto_lane(uint64_t m)
{
    std::lock_guard<std::mutex> g(g_tune_mu);
    const sm_tune_entry *e = g_tune_custom ? g_tune.data() : k_builtin_tune;
    const size_t n = g_tune_custom ? g_tune.size() : sizeof(k_builtin_tune) / sizeof(k_builtin_tune[0]) - 1;
    int lane = AUTO_MIN_LANE;
    for (size_t k = 0; k < n; k++)
        if (m >= e[k].m_lo && m <= e[k].m_hi && e[k].lane_bytes && e[k].lane_bytes < lane)
            lane = e[k].lane_bytes;
    return lane;
}

extern "C" int sm_tune_set(const sm_tune_entry *entries, uint32_t count)
{
    if (count && !entries) return fail(SM_EINVAL, "entries is NULL");
    for (uint32_t k = 0; k < count; k++) {
        const sm_tune_entry &e = entries[k];
        if (e.algo < ALGO_SHIFT_AND || e.algo >= ALGO_COUNT_ || e.m_lo > e.m_hi || e.sigma_lo > e.sigma_hi ||
            (e.lane_bytes && e.lane_bytes != 16 && e.lane_bytes != 32 && e.lane_bytes != 64 && e.lane_bytes != 128) ||
            e.q < 0 || e.q > Q_MAX || e.tiles_per_wg < 0 || e.tiles_per_wg > 4096 ||
            (e.hbits && (e.hbits < H_MIN || e.hbits > H_MAX)))
            return fail(SM_EINVAL, "invalid tuning entry %u", k);
    }
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune.assign(entries, entries + count);
    g_tune_custom = count > 0;
    return SM_OK;
}

extern "C" int sm_tune_get(sm_tune_entry *entries, uint32_t cap, uint32_t *count)
{
    if (!count || (cap && !entries)) return fail(SM_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> g(g_tune_mu);
    const sm_tune_entry *e = g_tune_custom ? g_tune.data() : k_builtin_tune;
    const size_t n = g_tune_custom ? g_tune.size() : sizeof(k_builtin_tune) / sizeof(k_builtin_tune[0]) - 1;
    for (size_t k = 0; k < n && k < cap; k++) entries[k] = e[k];
    *count = (uint32_t)n;
    return SM_OK;
}

static int make_plan(const uint8_t *pat, uint64_t m, const sm_opts *o, int sigma_known, Plan &p)
{
    sm_opts z;
    memset(&z, 0, sizeof z);
    if (!o) o = &z;
    if (o->reserved[0] || o->reserved[1]) return fail(SM_EINVAL, "sm_opts.reserved must be zero");
    if (o->algo < 0 || o->algo >= ALGO_COUNT_) return fail(SM_EINVAL, "unknown algorithm %d", o->algo);
    if (o->lane_bytes && o->lane_bytes != 16 && o->lane_bytes != 32 && o->lane_bytes != 64 &&
        o->lane_bytes != 128)
        return fail(SM_EINVAL, "lane_bytes must be 16, 32, 64 or 128 (got %d)", o->lane_bytes);
    if (o->q < 0 || o->q > Q_MAX) return fail(SM_EINVAL, "q must be in [1, %d]", Q_MAX);
    if (o->hbits && (o->hbits < H_MIN || o->hbits > H_MAX))
        return fail(SM_EINVAL, "hbits must be in [%d, %d]", H_MIN, H_MAX);
    if (o->tiles_per_wg < 0 || o->tiles_per_wg > 4096)
        return fail(SM_EINVAL, "tiles_per_wg must be in [1, 4096]");
    if (o->algo == ALGO_BRUTE && m > (uint64_t)BRUTE_MAX_M)
        return fail(SM_EINVAL, "brute force takes m <= %d (m = %llu)", BRUTE_MAX_M, (unsigned long long)m);
    if (o->algo == ALGO_BLOCK && (m < (uint64_t)BF_MIN_M || m > (uint64_t)BF_MAX_M))
        return fail(SM_EINVAL, "the block filter needs %d <= m <= %d (m = %llu)", BF_MIN_M, BF_MAX_M,
                    (unsigned long long)m);
    if (o->algo == ALGO_BNDM && m > BP_MAX_M)
        return fail(SM_EINVAL, "BNDM needs m <= %d (m = %llu)", BP_MAX_M, (unsigned long long)m);
    if (o->algo == ALGO_FSBNDM && m > (uint64_t)FSBNDM_MAX_M)
        return fail(SM_EINVAL, "FSBNDM needs m <= %d (m = %llu)", FSBNDM_MAX_M, (unsigned long long)m);
    if (o->q && (uint64_t)o->q > m)
        return fail(SM_EINVAL, "q = %d exceeds m = %llu", o->q, (unsigned long long)m);

    int sigma = o->sigma_hint > 0 ? o->sigma_hint : sigma_known;
    if (sigma <= 0) sigma = sigma_from_pattern(pat, m);
    if (sigma > 256) sigma = 256;

    // the tuning table's choice for (sigma, m), then explicit options on top
    sm_tune_entry te;
    const bool have = tune_lookup(sigma, m, te);
    int algo = have ? te.algo : 0;
    // entries not applicable to this m
    if (algo != ALGO_HASHQ && algo != ALGO_BLOCK && algo != ALGO_SBNDM && algo != ALGO_SHIFT_AND && m > BP_MAX_M)
        algo = 0;
    if (algo == ALGO_BLOCK && (m < (uint64_t)BF_MIN_M || m > (uint64_t)BF_MAX_M)) algo = 0;
    if (algo == ALGO_BRUTE && m > (uint64_t)BRUTE_MAX_M) algo = 0;
    if (algo == ALGO_FSBNDM && m > (uint64_t)FSBNDM_MAX_M) algo = 0;
    if (have && te.algo == ALGO_HASHQ && te.q && (uint64_t)te.q > m) algo = 0;
    // the block filter expects varied 16-byte blocks: not on a text of (nearly) one symbol
    if (algo == ALGO_BLOCK && sigma < 2) algo = 0;
    // on such a text every window of a skip algorithm can match up to m - 1 bytes before
    // it shifts by one (O(nm), the adversarial case of the paper's window-based families);
    // Shift-And takes one step per byte whatever the text (for m > 64 on the pattern's
    // last 49 bytes, the rest verified, once per period on a periodic run)
    bool use_entry = algo != 0 && (o->algo == ALGO_AUTO || o->algo == algo);
    bool one_symbol = false;
    if (sigma < 2 && o->algo == ALGO_AUTO && algo != ALGO_SHIFT_AND) {
        algo = ALGO_SHIFT_AND;
        use_entry = false;
        one_symbol = true;
    }
    if (o->algo != ALGO_AUTO) algo = o->algo;
    if (algo == 0) {  // heuristic when no table entry applies
        if (m <= 12) algo = ALGO_SHIFT_AND;
        else if (m <= BP_MAX_M) algo = ALGO_SBNDM;
        else algo = ALGO_HASHQ;
    }
    p.m = m;
    p.algo = algo;
    p.q = 0;
    p.hbits = 0;
    if (algo == ALGO_SBNDM) {  // q-gram width of the window's first read
        const int q = o->q ? o->q : (use_entry ? te.q : 0);
        if (q > 1 && q != 2 && q != 4 && q != 8) return fail(SM_EINVAL, "SBNDM takes q in {1, 2, 4, 8} (got %d)", q);
        p.q = (q > 1 && (uint64_t)q <= m) ? q : 0;
    }
    if (algo == ALGO_BNDM) {  // BNDMq: the window's last q bytes at once
        const int q = o->q ? o->q : (use_entry ? te.q : 0);
        if (q > 1 && q != 2 && q != 4) return fail(SM_EINVAL, "BNDM takes q in {1, 2, 4} (got %d)", q);
        p.q = (q > 1 && (uint64_t)q <= m) ? q : 0;
    }
    if (algo == ALGO_HASHQ) {
        p.q = o->q ? o->q : (use_entry && te.q ? te.q : choose_q(m, sigma));
        if ((uint64_t)p.q > m) p.q = (int)m;
        p.hbits = o->hbits ? o->hbits : (use_entry && te.hbits ? te.hbits : choose_hbits(m, p.q));
    }
    // texts of one symbol: 128-start lanes, two tiles per workgroup (measured on MI355X
    // at n = 2^30 for m = 4 .. 1000: the best or within 2 % of it at every m)
    p.lane_bytes = o->lane_bytes ? o->lane_bytes
                                 : (use_entry && te.lane_bytes ? te.lane_bytes : (one_symbol ? 128 : 64));
    if (algo == ALGO_BLOCK) p.lane_bytes = (int32_t)bf_stride(m);  // starts per sampled block
    p.tiles_per_wg = o->tiles_per_wg ? o->tiles_per_wg
                                     : (use_entry && te.tiles_per_wg ? te.tiles_per_wg : (one_symbol ? 2 : 1));
    // a tile of 256 * L starts expects 256 * L * sigma^-m hits on an i.i.d. text: at
    // most the stash (256) when sigma^m >= L; denser tiles go to the emit pass anyway
    p.slots = (double)m * std::log((double)sigma) >= std::log((double)p.lane_bytes) ? 1 : 0;
    // the suffix form of Shift-And (m > 49) verifies each hit from global memory: lanes
    // keep their first hits so that tiles with few hits are not scanned twice
    if (algo == ALGO_SHIFT_AND && m > (uint64_t)SA_SUFFIX) {
        p.slots = 1;
        // The last 17 bytes on a 32-bit state scan in about half the operations of the
        // last 49 on a 64-bit one, and a start one period after an occurrence is still
        // taken without reading when the period is at most 17. A pattern whose smallest
        // period lies in (17, 49] keeps the 49-byte suffix, so that such starts (every
        // period of a periodic text) are not read in full. Beyond 16 MiB the pattern is not
        // compared with itself on the host (49 passes over it): the 49-byte suffix is kept.
        uint32_t per = 0;
        const bool look = m <= (1ull << 24);
        for (uint32_t d = 1; look && d <= (uint32_t)SA_SUFFIX && !per; d++)
            if (memcmp(pat, pat + d, m - d) == 0) per = d;
        p.sfx = (!look || per > (uint32_t)SA_SHORT) ? SA_SUFFIX : SA_SHORT;
    }
    return SM_OK;
}

int sm::plan_pattern_opts(const uint8_t *pat, uint64_t m, const sm_opts *o, Plan &p)
{
    return make_plan(pat, m, o, 0, p);
}

int sm::plan_pattern(const uint8_t *pat, uint64_t m, int sigma, Plan &p)
{
    return make_plan(pat, m, nullptr, sigma, p);
}

// ---------------------------------------------------------------------------
// kernel timing
// ---------------------------------------------------------------------------
namespace {
struct ProfRec {
    hipEvent_t e0, e1, e2, e3;  // start, after prep, after the count kernel, end
    uint64_t n;
    bool sampled;  // block filter: the count pass reads sampled blocks only
};
std::mutex g_prof_mu;
uint32_t g_prof_every = 0;  // 0: off; k: every k-th call is recorded
uint64_t g_prof_seen = 0;   // calls since enabling
std::vector<ProfRec> g_prof;
std::vector<BatchProfRec> g_prof_batch;
}  // namespace

bool sm::prof_batch_begin(hipStream_t st, BatchProfRec &r)
{
    {
        std::lock_guard<std::mutex> g(g_prof_mu);
        if (!g_prof_every) return false;
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return false;
    memset(&r, 0, sizeof r);
    hipEvent_t *ev[4] = {&r.e0, &r.e1, &r.e2, &r.e3};
    for (int k = 0; k < 4; k++) {
        if (hipEventCreate(ev[k]) != hipSuccess) {
            for (int j = 0; j < k; j++) (void)hipEventDestroy(*ev[j]);
            return false;
        }
    }
    if (hipEventRecord(r.e0, st) != hipSuccess) {
        prof_batch_discard(r);
        return false;
    }
    return true;
}

void sm::prof_batch_push(const BatchProfRec &r)
{
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof_batch.push_back(r);
}

void sm::prof_batch_discard(BatchProfRec &r)
{
    (void)hipEventDestroy(r.e0);
    (void)hipEventDestroy(r.e1);
    (void)hipEventDestroy(r.e2);
    (void)hipEventDestroy(r.e3);
    memset(&r, 0, sizeof r);
}

extern "C" int sm_prof_enable(int every)
{
    if (every < 0) return fail(SM_EINVAL, "profiling stride must be >= 0");
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof_every = (uint32_t)every;
    g_prof_seen = 0;
    return SM_OK;
}

extern "C" int sm_prof_collect(sm_prof *out)
{
    if (!out) return fail(SM_EINVAL, "out is NULL");
    std::vector<ProfRec> recs;
    std::vector<BatchProfRec> brecs;
    {
        std::lock_guard<std::mutex> g(g_prof_mu);
        recs.swap(g_prof);
        brecs.swap(g_prof_batch);
    }
    memset(out, 0, sizeof *out);
    int st = SM_OK;
    for (auto &r : recs) {
        float a = 0, b = 0, c = 0;
        if (hipEventSynchronize(r.e3) == hipSuccess && hipEventElapsedTime(&a, r.e1, r.e2) == hipSuccess &&
            hipEventElapsedTime(&b, r.e2, r.e3) == hipSuccess && hipEventElapsedTime(&c, r.e0, r.e3) == hipSuccess) {
            out->calls++;
            out->count_ms += a;
            out->emit_ms += b;
            out->total_ms += c;
            out->text_bytes += r.n;
            if (r.sampled) {
                out->sampled_calls++;
                out->sampled_count_ms += a;
            }
        } else {
            st = fail(SM_EDEVICE, "event timing failed");
        }
        (void)hipEventDestroy(r.e0);
        (void)hipEventDestroy(r.e1);
        (void)hipEventDestroy(r.e2);
        (void)hipEventDestroy(r.e3);
    }
    for (auto &r : brecs) {
        float a = 0, b = 0;
        if (hipEventSynchronize(r.e3) == hipSuccess && hipEventElapsedTime(&a, r.e1, r.e2) == hipSuccess &&
            hipEventElapsedTime(&b, r.e0, r.e3) == hipSuccess) {
            out->batch_calls++;
            out->batch_ms += b;
            out->filter_launches += r.filter_launches;
            out->filter_ms += a;
            out->filter_pattern_bytes += r.filter_pattern_bytes;
        } else {
            st = fail(SM_EDEVICE, "event timing failed");
        }
        prof_batch_discard(r);
    }
    return st;
}

// ---------------------------------------------------------------------------
// core: validated, planned, asynchronous
// ---------------------------------------------------------------------------
static int validate_common(const uint8_t *text, uint64_t n, const uint8_t *pat, uint64_t m)
{
    if (m == 0) return fail(SM_EINVAL, "empty pattern (m = 0)");
    if (!pat) return fail(SM_EINVAL, "pattern is NULL");
    if (!text && n > 0) return fail(SM_EINVAL, "text is NULL with n > 0");
    if (m > 0xFFFFFFFFull) return fail(SM_EINVAL, "m must be < 2^32");
    return SM_OK;
}

// Whether a plan for a pattern of length m under opts may keep hit bitmaps beyond
// m <= 64: Shift-And's suffix form does, which the planner takes on texts of one
// dominant symbol (sigma < 2), where the tuning table picks it, or when it is forced.
static bool may_keep_bitmap(uint64_t m, const sm_opts *o)
{
    if (m <= (uint64_t)BP_MAX_M) return true;
    if (o && o->algo) return o->algo == ALGO_SHIFT_AND;
    if (o && o->sigma_hint > 0) {  // Shift-And on a text of one symbol, or where the table says
        if (o->sigma_hint < 2) return true;
        sm_tune_entry te;
        return tune_lookup(std::min(o->sigma_hint, 256), m, te) && te.algo == ALGO_SHIFT_AND;
    }
    return true;
}

static bool plan_keeps_bitmap(const Plan &p)
{
    return p.m <= (uint64_t)BP_MAX_M || p.algo == ALGO_SHIFT_AND;
}

static uint64_t plan_lead(const Plan &p) { return p.algo == ALGO_BLOCK ? BF_LEAD : 0; }

extern "C" uint64_t sm_workspace_size(uint64_t n, uint64_t m, const sm_opts *opts)
{
    // explicit lanes, else the smallest the planner could pick for this m (the
    const bool block_range = m >= (uint64_t)BF_MIN_M && m <= (uint64_t)BF_MAX_M;
    Plan p;
    p.lane_bytes = (opts && opts->lane_bytes) ? opts->lane_bytes : min_auto_lane(m);
    uint64_t need = 0;
    if (!(opts && opts->algo == ALGO_BLOCK && block_range))
        need = ws_layout(n, m, tile_starts(p), may_keep_bitmap(m, opts)).need;
    // the block filter, when forced or when the planner may take it (its tiles of
    // 256 blocks may start BF_LEAD starts early)
    if (block_range && (!opts || opts->algo == ALGO_AUTO || opts->algo == ALGO_BLOCK)) {
        p.lane_bytes = (int32_t)bf_stride(m);
        need = std::max(need, ws_layout(n, m, tile_starts(p), false, BF_LEAD).need);
    }
    return need;
}

extern "C" uint64_t sm_workspace_size_upto(uint64_t n, uint64_t m_max, const sm_opts *opts)
{
    // every length up to the block filter's range, one by one
    const uint64_t lim = std::min<uint64_t>(m_max, (uint64_t)BF_MAX_M + 1);
    uint64_t best = 0;
    for (uint64_t m = 1; m <= lim; m++) best = std::max(best, sm_workspace_size(n, m, opts));
    if (m_max <= lim) return best;
    // above it: the tile part only shrinks as m grows and the pattern copy grows,
    // so the narrowest lane any entry covering (lim, m_max] may pick, at m = lim + 1,
    // with the pattern copy of m_max bounds every size
    int lb = (opts && opts->lane_bytes) ? opts->lane_bytes : AUTO_MIN_LANE;
    if (!(opts && opts->lane_bytes)) {
        std::lock_guard<std::mutex> g(g_tune_mu);
        const sm_tune_entry *e = g_tune_custom ? g_tune.data() : k_builtin_tune;
        const size_t ne = g_tune_custom ? g_tune.size() : sizeof(k_builtin_tune) / sizeof(k_builtin_tune[0]) - 1;
        for (size_t k = 0; k < ne; k++)
            if (e[k].m_hi > lim && e[k].m_lo <= m_max && e[k].lane_bytes && e[k].lane_bytes < lb)
                lb = e[k].lane_bytes;
    }
    Plan p;
    p.lane_bytes = lb;
    const WsLayout w = ws_layout(n, lim + 1, tile_starts(p), may_keep_bitmap(lim + 1, opts));
    return std::max(best, w.need + align_up(m_max + 64, 256) - align_up(lim + 1 + 64, 256));
}

static int run_async(const uint8_t *d_text, uint64_t n, const uint8_t *pat, uint64_t m,
                     int64_t *d_out, uint64_t cap, uint64_t *d_count, void *d_work,
                     uint64_t work_bytes, const sm_opts *opts, hipStream_t st, bool write,
                     int sigma_known, uint64_t first = 0, bool may_profile = true)
{
    TraceRange tr(write ? "sm.find_all.enqueue" : "sm.count.enqueue");
    int r = validate_common(d_text, n, pat, m);
    if (r) return r;
    if (!d_count) return fail(SM_EINVAL, "d_count is NULL");
    if (write && !d_out && cap > 0) return fail(SM_EINVAL, "output is NULL with cap > 0");
    Plan plan;
    r = make_plan(pat, m, opts, sigma_known, plan);
    if (r) return r;
    if ((r = check_device())) return r;
    if (n == 0 || m > n) {
        HIP_TRY(launch_set_u64(d_count, 0, st));
        return SM_OK;
    }
    const WsLayout w = ws_layout(n, m, tile_starts(plan), plan_keeps_bitmap(plan), plan_lead(plan));
    const uint64_t need = write ? w.need : w.need_count;
    if (!d_work || work_bytes < need)
        return fail(SM_EINVAL, "workspace too small: need %llu bytes", (unsigned long long)need);
    if (((uintptr_t)d_work & 255) != 0) return fail(SM_EINVAL, "workspace must be 256-byte aligned");
    uint8_t *ws = static_cast<uint8_t *>(d_work);
    Params *prm = reinterpret_cast<Params *>(ws + w.params);
    uint8_t *dpat = ws + w.pat;
    FindWs fw;
    fw.tile_cnt = reinterpret_cast<uint32_t *>(ws + w.tile_cnt);
    fw.super = reinterpret_cast<uint64_t *>(ws + w.super);
    fw.list = reinterpret_cast<TileEntry *>(ws + w.list);
    fw.nlist = reinterpret_cast<uint64_t *>(ws + w.nlist);
    fw.stash = reinterpret_cast<uint16_t *>(ws + w.stash);
    fw.bits = w.bits ? reinterpret_cast<uint32_t *>(ws + w.bits) : nullptr;
    fw.ntiles = w.ntiles;

    bool prof;
    ProfRec rec{};
    {
        std::lock_guard<std::mutex> g(g_prof_mu);
        prof = may_profile && g_prof_every && g_prof_seen++ % g_prof_every == 0;
    }
    if (prof) {
        HIP_TRY(hipEventCreate(&rec.e0));
        HIP_TRY(hipEventCreate(&rec.e1));
        HIP_TRY(hipEventCreate(&rec.e2));
        HIP_TRY(hipEventCreate(&rec.e3));
        rec.n = n;
        rec.sampled = plan.algo == ALGO_BLOCK;
        HIP_TRY(hipEventRecord(rec.e0, st));
    }
    HIP_TRY(launch_prep(plan, pat, prm, dpat, d_count, fw.super, num_super(w.ntiles), st));
    if (prof) HIP_TRY(hipEventRecord(rec.e1, st));
    if (write) {
        HIP_TRY(launch_find(plan, d_text, n, prm, dpat, fw, d_out, first, cap, d_count, st,
                            prof ? rec.e2 : nullptr));
    } else {
        HIP_TRY(launch_count(plan, d_text, n, prm, dpat, fw, d_count, st, prof ? rec.e2 : nullptr));
    }
    if (prof) {
        HIP_TRY(hipEventRecord(rec.e3, st));
        std::lock_guard<std::mutex> g(g_prof_mu);
        g_prof.push_back(rec);
    }
    return SM_OK;
}

extern "C" int sm_find_all_async(const uint8_t *d_text, uint64_t n, const uint8_t *pat, uint64_t m,
                                 int64_t *d_out, uint64_t cap, uint64_t *d_count, void *d_work,
                                 uint64_t work_bytes, const sm_opts *opts, void *stream)
{
    return run_async(d_text, n, pat, m, d_out, cap, d_count, d_work, work_bytes, opts,
                     (hipStream_t)stream, true, 0);
}

extern "C" int sm_count_async(const uint8_t *d_text, uint64_t n, const uint8_t *pat, uint64_t m,
                              uint64_t *d_count, void *d_work, uint64_t work_bytes,
                              const sm_opts *opts, void *stream)
{
    return run_async(d_text, n, pat, m, nullptr, 0, d_count, d_work, work_bytes, opts,
                     (hipStream_t)stream, false, 0);
}

// ---------------------------------------------------------------------------
// find_all without allocation: the workspace is a static device array
// ---------------------------------------------------------------------------
// Every device the library runs on holds its own copy of this array (code-object
// memory) until the process ends. In host code its name is only a host-side stand-in:
// kernels take the per-device address from hipGetSymbolAddress instead.
static __device__ __align__(256) uint8_t scratch[SM_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kScratchDevices];  // per device: device address of `scratch`, once looked up

// Device address of the current device's scratch array (looked up once per device,
// with that device current).
int static_scratch(void **out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kScratchDevices)
        return fail(SM_EDEVICE, "device %d: the static scratch is tracked for devices 0..%d only", dev,
                    kScratchDevices - 1);
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(SM_EDEVICE, "hipGetSymbolAddress returned NULL for the static scratch");
        if (((uintptr_t)p & 255) != 0) return fail(SM_EDEVICE, "static scratch is not 256-byte aligned");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SM_OK;
}
}  // namespace

extern "C" int sm_find_all_noalloc(const uint8_t *d_text, uint64_t n, const uint8_t *pat, uint64_t m,
                                   int64_t *d_out, uint64_t cap, uint64_t *d_count,
                                   const sm_opts *opts, void *stream)
{
    int r = validate_common(d_text, n, pat, m);
    if (r) return r;
    if (!d_count) return fail(SM_EINVAL, "d_count is NULL");
    if (!d_out && cap > 0) return fail(SM_EINVAL, "output is NULL with cap > 0");
    if (m > (uint64_t)PREP_INLINE)
        return fail(SM_EINVAL, "sm_find_all_noalloc takes patterns of at most %d bytes (m = %llu)",
                    PREP_INLINE, (unsigned long long)m);
    Plan plan;
    if ((r = make_plan(pat, m, opts, 0, plan))) return r;
    if (n > 0 && m <= n) {
        const uint64_t need = ws_layout(n, m, tile_starts(plan), plan_keeps_bitmap(plan), plan_lead(plan)).need;
        if (need > (uint64_t)SM_NOALLOC_SCRATCH_BYTES)
            return fail(SM_EINVAL,
                        "sm_find_all_noalloc: n = %llu, m = %llu needs %llu bytes of workspace, more than "
                        "the %llu bytes of static scratch; use sm_find_all_async with a caller workspace",
                        (unsigned long long)n, (unsigned long long)m, (unsigned long long)need,
                        (unsigned long long)SM_NOALLOC_SCRATCH_BYTES);
    }
    if ((r = check_device())) return r;
    void *ws = nullptr;
    if ((r = static_scratch(&ws))) return r;
    return run_async(d_text, n, pat, m, d_out, cap, d_count, ws, (uint64_t)SM_NOALLOC_SCRATCH_BYTES, opts,
                     (hipStream_t)stream, true, 0, 0, false);
}

extern "C" int sm_plan_query(const uint8_t *pat, uint64_t m, const sm_opts *opts, sm_plan_info *info)
{
    if (m == 0) return fail(SM_EINVAL, "empty pattern (m = 0)");
    if (!pat || !info) return fail(SM_EINVAL, "NULL argument");
    Plan p;
    int r = make_plan(pat, m, opts, 0, p);
    if (r) return r;
    info->algo = p.algo;
    info->lane_bytes = p.lane_bytes;
    info->q = p.q;
    info->hbits = p.hbits;
    info->tiles_per_wg = p.tiles_per_wg;
    info->suffix = p.sfx;
    return SM_OK;
}

// ---------------------------------------------------------------------------
// synchronous device forms: per-thread cached workspace
// ---------------------------------------------------------------------------
namespace {
struct Scratch {
    int dev = -1;
    void *ws = nullptr;
    uint64_t ws_bytes = 0;
    uint64_t *d_count = nullptr;
    ~Scratch()
    {
        // process teardown: the HIP runtime may already be gone; leak silently
    }
};
thread_local Scratch g_scratch;

int scratch_get(uint64_t need, void **ws, uint64_t **d_count)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    Scratch &s = g_scratch;
    if (s.dev != dev) {
        s = Scratch();
        s.dev = dev;
    }
    if (!s.d_count) HIP_TRY(hipMalloc((void **)&s.d_count, 256));
    if (s.ws_bytes < need) {
        if (s.ws) HIP_TRY(hipFree(s.ws));
        s.ws = nullptr;
        s.ws_bytes = 0;
        uint64_t sz = std::max<uint64_t>(need, 1 << 20);
        HIP_TRY(hipMalloc(&s.ws, sz));
        s.ws_bytes = sz;
    }
    *ws = s.ws;
    *d_count = s.d_count;
    return SM_OK;
}
}  // namespace

static int run_sync_dev(const uint8_t *d_text, uint64_t n, const uint8_t *pat, uint64_t m,
                        int64_t *d_out, uint64_t cap, uint64_t *count, hipStream_t st, bool write,
                        int sigma_known)
{
    TraceRange tr(write ? "sm.find_all" : "sm.count");
    int r = validate_common(d_text, n, pat, m);
    if (r) return r;
    if (!count) return fail(SM_EINVAL, "count is NULL");
    if (write && !d_out && cap > 0) return fail(SM_EINVAL, "output is NULL with cap > 0");
    Plan plan;
    if ((r = make_plan(pat, m, nullptr, sigma_known, plan))) return r;
    if (n == 0 || m > n) {
        *count = 0;
        return SM_OK;
    }
    if ((r = check_device())) return r;
    sm_opts o;
    memset(&o, 0, sizeof o);
    o.sigma_hint = sigma_known;
    const uint64_t need = sm_workspace_size(n, m, &o);
    void *ws;
    uint64_t *dc;
    if ((r = scratch_get(need, &ws, &dc))) return r;
    r = run_async(d_text, n, pat, m, d_out, cap, dc, ws, need, &o, st, write, sigma_known);
    if (r) return r;
    uint64_t total = 0;
    HIP_TRY(hipMemcpyAsync(&total, dc, 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    *count = total;
    return (write && total > cap) ? SM_TRUNCATED : SM_OK;
}

extern "C" int sm_find_all_dev(const uint8_t *d_text, uint64_t n, const uint8_t *pat, uint64_t m,
                               int64_t *d_out, uint64_t cap, uint64_t *count, void *stream)
{
    return run_sync_dev(d_text, n, pat, m, d_out, cap, count, (hipStream_t)stream, true, 0);
}

extern "C" int sm_count_dev(const uint8_t *d_text, uint64_t n, const uint8_t *pat, uint64_t m,
                            uint64_t *count, void *stream)
{
    return run_sync_dev(d_text, n, pat, m, nullptr, 0, count, (hipStream_t)stream, false, 0);
}

// ---------------------------------------------------------------------------
// host-buffer forms
// ---------------------------------------------------------------------------
namespace {
struct DevBuf {
    void *p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
};
}  // namespace

static int run_host(const uint8_t *text, uint64_t n, const uint8_t *pat, uint64_t m,
                    int64_t *out_pos, uint64_t cap, uint64_t *count, bool write)
{
    int r = validate_common(text, n, pat, m);
    if (r) return r;
    if (!count) return fail(SM_EINVAL, "count is NULL");
    if (write && !out_pos && cap > 0) return fail(SM_EINVAL, "out_pos is NULL with cap > 0");
    Plan plan;
    if ((r = make_plan(pat, m, nullptr, 0, plan))) return r;
    if (n == 0 || m > n) {
        *count = 0;
        return SM_OK;
    }
    if ((r = check_device())) return r;
    DevBuf dt, dout;
    HIP_TRY(hipMalloc(&dt.p, align_up(n, 256)));
    HIP_TRY(hipMemcpy(dt.p, text, n, hipMemcpyHostToDevice));
    const uint64_t ncap = std::min<uint64_t>(cap, n - m + 1);
    if (write && ncap) HIP_TRY(hipMalloc(&dout.p, ncap * 8));
    uint64_t total = 0;
    r = run_sync_dev((const uint8_t *)dt.p, n, pat, m, (int64_t *)dout.p, write ? ncap : 0, &total,
                     nullptr, write, 0);
    if (r < 0) return r;
    if (write && ncap) {
        const uint64_t k = std::min<uint64_t>(total, ncap);
        if (k) HIP_TRY(hipMemcpy(out_pos, dout.p, k * 8, hipMemcpyDeviceToHost));
    }
    *count = total;
    return (write && total > cap) ? SM_TRUNCATED : SM_OK;
}

extern "C" int sm_find_all(const uint8_t *text, uint64_t n, const uint8_t *pat, uint64_t m,
                           int64_t *out_pos, uint64_t cap, uint64_t *count)
{
    return run_host(text, n, pat, m, out_pos, cap, count, true);
}

extern "C" int sm_count(const uint8_t *text, uint64_t n, const uint8_t *pat, uint64_t m, uint64_t *count)
{
    return run_host(text, n, pat, m, nullptr, 0, count, false);
}

// ---------------------------------------------------------------------------
// corpora
// ---------------------------------------------------------------------------

extern "C" int sm_corpus_open(const uint8_t *text, uint64_t n, int text_on_device, sm_corpus **corpus)
{
    if (!corpus) return fail(SM_EINVAL, "corpus is NULL");
    if (!text && n > 0) return fail(SM_EINVAL, "text is NULL with n > 0");
    int r = check_device();
    if (r) return r;
    sm_corpus *c = new sm_corpus();
    memset(c->hist, 0, sizeof c->hist);
    HIP_TRY(hipGetDevice(&c->dev));
    if (text_on_device) {
        c->d_text = text;
        c->owned = false;
    } else if (n > 0) {
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, align_up(n, 256));
        if (e != hipSuccess) {
            delete c;
            return fail(SM_ENOMEM, "corpus allocation of %llu bytes failed: %s", (unsigned long long)n,
                        hipGetErrorString(e));
        }
        e = hipMemcpy(p, text, n, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(p);
            delete c;
            return fail(SM_EDEVICE, "corpus upload failed: %s", hipGetErrorString(e));
        }
        c->d_text = (const uint8_t *)p;
        c->owned = true;
    }
    c->n = n;
    if (n > 0) {
        uint64_t *dh = nullptr;
        hipError_t e = hipMalloc((void **)&dh, 256 * 8);
        if (e == hipSuccess) e = hipMemset(dh, 0, 256 * 8);
        if (e == hipSuccess) e = launch_histogram(c->d_text, n, dh, nullptr);
        if (e == hipSuccess) e = hipMemcpy(c->hist, dh, 256 * 8, hipMemcpyDeviceToHost);
        if (dh) (void)hipFree(dh);
        if (e != hipSuccess) {
            if (c->owned) (void)hipFree((void *)c->d_text);
            delete c;
            return fail(SM_EDEVICE, "corpus histogram failed: %s", hipGetErrorString(e));
        }
        double s2 = 0;
        for (int k = 0; k < 256; k++) {
            c->sigma += c->hist[k] ? 1 : 0;
            const double pk = (double)c->hist[k] / (double)n;
            s2 += pk * pk;
        }
        c->sigma_eff = s2 > 0 ? 1.0 / s2 : 0;
    }
    *corpus = c;
    return SM_OK;
}

extern "C" int sm_corpus_close(sm_corpus *c)
{
    if (!c) return fail(SM_EINVAL, "corpus is NULL");
    if (c->owned && c->d_text) (void)hipFree((void *)c->d_text);
    delete c;
    return SM_OK;
}

extern "C" int sm_corpus_stats(const sm_corpus *c, uint64_t *histogram, int32_t *sigma,
                               double *sigma_eff)
{
    if (!c) return fail(SM_EINVAL, "corpus is NULL");
    if (histogram) memcpy(histogram, c->hist, sizeof c->hist);
    if (sigma) *sigma = c->sigma;
    if (sigma_eff) *sigma_eff = c->sigma_eff;
    return SM_OK;
}

int sm::corpus_sigma(const sm_corpus *c)
{
    int s = (int)std::lround(c->sigma_eff);
    return s < 1 ? 1 : (s > 256 ? 256 : s);
}

extern "C" int sm_corpus_find_all_async(sm_corpus *c, const uint8_t *pat, uint64_t m, int64_t *d_out,
                                        uint64_t cap, uint64_t *d_count, void *d_work,
                                        uint64_t work_bytes, const sm_opts *opts, void *stream)
{
    if (!c) return fail(SM_EINVAL, "corpus is NULL");
    return run_async(c->d_text, c->n, pat, m, d_out, cap, d_count, d_work, work_bytes, opts,
                     (hipStream_t)stream, true, corpus_sigma(c));
}

int sm::corpus_find_window_async(sm_corpus *c, const uint8_t *pat, uint64_t m, int64_t *d_out,
                                 uint64_t first, uint64_t cap, uint64_t *d_count, void *d_work,
                                 uint64_t work_bytes, hipStream_t stream)
{
    if (!c) return fail(SM_EINVAL, "corpus is NULL");
    return run_async(c->d_text, c->n, pat, m, d_out, cap, d_count, d_work, work_bytes, nullptr,
                     stream, true, corpus_sigma(c), first);
}

extern "C" int sm_corpus_count_async(sm_corpus *c, const uint8_t *pat, uint64_t m, uint64_t *d_count,
                                     void *d_work, uint64_t work_bytes, const sm_opts *opts,
                                     void *stream)
{
    if (!c) return fail(SM_EINVAL, "corpus is NULL");
    return run_async(c->d_text, c->n, pat, m, nullptr, 0, d_count, d_work, work_bytes, opts,
                     (hipStream_t)stream, false, corpus_sigma(c));
}

extern "C" int sm_corpus_text(const sm_corpus *c, const uint8_t **d_text, uint64_t *n)
{
    if (!c) return fail(SM_EINVAL, "corpus is NULL");
    if (d_text) *d_text = c->d_text;
    if (n) *n = c->n;
    return SM_OK;
}

extern "C" int sm_corpus_find_all(sm_corpus *c, const uint8_t *pat, uint64_t m, int64_t *out_pos,
                                  uint64_t cap, uint64_t *count)
{
    if (!c) return fail(SM_EINVAL, "corpus is NULL");
    int r = validate_common(c->d_text, c->n, pat, m);
    if (r) return r;
    if (!count) return fail(SM_EINVAL, "count is NULL");
    if (!out_pos && cap > 0) return fail(SM_EINVAL, "out_pos is NULL with cap > 0");
    if (c->n == 0 || m > c->n) {
        *count = 0;
        return SM_OK;
    }
    HIP_TRY(hipSetDevice(c->dev));
    DevBuf dout;
    const uint64_t ncap = std::min<uint64_t>(cap, c->n - m + 1);
    if (ncap) HIP_TRY(hipMalloc(&dout.p, ncap * 8));
    uint64_t total = 0;
    r = run_sync_dev(c->d_text, c->n, pat, m, (int64_t *)dout.p, ncap, &total, nullptr, true, corpus_sigma(c));
    if (r < 0) return r;
    const uint64_t k = std::min<uint64_t>(total, ncap);
    if (k) HIP_TRY(hipMemcpy(out_pos, dout.p, k * 8, hipMemcpyDeviceToHost));
    *count = total;
    return total > cap ? SM_TRUNCATED : SM_OK;
}

extern "C" int sm_corpus_count(sm_corpus *c, const uint8_t *pat, uint64_t m, uint64_t *count)
{
    if (!c) return fail(SM_EINVAL, "corpus is NULL");
    int r = validate_common(c->d_text, c->n, pat, m);
    if (r) return r;
    if (!count) return fail(SM_EINVAL, "count is NULL");
    if (c->n == 0 || m > c->n) {
        *count = 0;
        return SM_OK;
    }
    HIP_TRY(hipSetDevice(c->dev));
    return run_sync_dev(c->d_text, c->n, pat, m, nullptr, 0, count, nullptr, false, corpus_sigma(c));
}
