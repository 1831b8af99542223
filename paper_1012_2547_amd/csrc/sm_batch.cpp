// C ABI of the batched multi-pattern search: planning and grouping of the
// patterns, workspace layout, the count and windowed write steps (kernels in
// sm_batch.hip), the batch handle and the synchronous forms.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <string_view>
#include <unordered_map>
#include <vector>

#include "../../include/sm.h"
#include "sm_batch_host.h"
#include "sm_trace.h"

using namespace sm;

int sm::batch_err(int status, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    sm_set_error(status, buf);
    return status;
}

#define err sm::batch_err

#define HIP_OK(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return err(e_ == hipErrorOutOfMemory ? SM_ENOMEM : SM_EDEVICE, "%s: %s", #expr, \
                       hipGetErrorString(e_));                                              \
    } while (0)

namespace {

constexpr uint64_t BT = (uint64_t)BLOCK * BATCH_LANE;

int var_of(const Plan &p)
{
    if (p.algo == ALGO_SHIFT_AND) return p.m <= 17 ? 0 : (p.m <= 49 ? 1 : (p.m <= 61 ? 2 : 3));
    if (p.algo == ALGO_HASHQ) return (p.q + 3) / 4;
    return 0;
}

int table_bytes(uint32_t algo, uint32_t var)
{
    if (algo == ALGO_HASHQ) return 1 << BATCH_HBITS_MAX;
    return (algo == ALGO_SHIFT_AND && var == 0) ? 1024 : 2048;
}

uint64_t pat_region(uint64_t m) { return align_up(m, 16) + 16; }  // verify reads 16 bytes past m

// Table of one prefix-filter group (layout in sm_internal.h): the patterns
// mem[0 .. count) (sorted indices) of q-class q.
// Returns whether the group is flat (every pattern has m == q and every bucket
// holds one slot).
bool build_mq_table(const BatchJob &j, const uint32_t *mem, uint32_t count, uint32_t q, uint8_t *T,
                    bool slot_counts)
{
    uint32_t *bits = reinterpret_cast<uint32_t *>(T + MQ_OFF_BITS);
    uint16_t *rank = reinterpret_cast<uint16_t *>(T + MQ_OFF_RANK);
    uint16_t *bstart = reinterpret_cast<uint16_t *>(T + MQ_OFF_BSTART);
    uint32_t *spre = reinterpret_cast<uint32_t *>(T + MQ_OFF_SPRE);
    uint16_t *sstart = reinterpret_cast<uint16_t *>(T + MQ_OFF_SSTART);
    uint16_t *srep = reinterpret_cast<uint16_t *>(T + MQ_OFF_SREP);
    uint16_t *pid = reinterpret_cast<uint16_t *>(T + MQ_OFF_PID);
    uint16_t *m16 = reinterpret_cast<uint16_t *>(T + MQ_OFF_M);
    uint32_t *pre2 = reinterpret_cast<uint32_t *>(T + MQ_OFF_PRE2);
    uint32_t *spi = reinterpret_cast<uint32_t *>(T + MQ_OFF_SPI);
    uint32_t *poff = reinterpret_cast<uint32_t *>(T + MQ_OFF_POFF);
    uint16_t *cid = reinterpret_cast<uint16_t *>(T + MQ_OFF_CID);
    struct Ent {
        uint32_t h, lo, hi, l;
    };
    std::vector<Ent> ents(count);
    for (uint32_t l = 0; l < count; l++) {
        const BatchPat &bp = j.bpats[mem[l]];
        const uint8_t *pp = j.pats + j.pat_off[bp.index];
        uint32_t w[4] = {0, 0, 0, 0};
        for (uint32_t k = 0; k < q; k++) w[k >> 2] |= (uint32_t)pp[k] << (8 * (k & 3));
        const uint32_t nb = std::min<uint32_t>(bp.m - q, 8);
        for (uint32_t k = 0; k < nb; k++) w[2 + (k >> 2)] |= (uint32_t)pp[q + k] << (8 * (k & 3));
        pre2[2 * l] = w[2];
        pre2[2 * l + 1] = w[3];
        m16[l] = (uint16_t)bp.m;
        spi[l] = mem[l];
        poff[l] = (uint32_t)bp.pat_off;
        ents[l] = {mq_key(w[0], w[1], q), w[0], w[1], l};
        bits[ents[l].h >> 5] |= 1u << (ents[l].h & 31);
    }
    // buckets by hash, slots by prefix inside a bucket, m == q patterns first in a slot
    std::sort(ents.begin(), ents.end(), [&](const Ent &x, const Ent &y) {
        if (x.h != y.h) return x.h < y.h;
        if (x.lo != y.lo) return x.lo < y.lo;
        if (x.hi != y.hi) return x.hi < y.hi;
        return x.l < y.l;
    });
    uint32_t nb = 0, ns = 0, np = 0;
    for (uint32_t e = 0; e < count; e++) {
        const Ent &x = ents[e];
        const bool new_bucket = e == 0 || x.h != ents[e - 1].h;
        const bool new_slot = new_bucket || x.lo != ents[e - 1].lo || x.hi != ents[e - 1].hi;
        if (new_bucket) bstart[nb++] = (uint16_t)ns;
        if (new_slot) {
            spre[2 * ns] = x.lo;
            spre[2 * ns + 1] = x.hi;
            srep[ns] = (uint16_t)MQ_NONE;
            sstart[ns] = (uint16_t)np;
            ns++;
        }
        if (slot_counts && m16[x.l] == q) {  // counted by the slot: its first such pattern holds the count
            if (srep[ns - 1] == MQ_NONE) srep[ns - 1] = (uint16_t)x.l;
            cid[x.l] = srep[ns - 1];
        } else {
            pid[np++] = (uint16_t)x.l;
            cid[x.l] = (uint16_t)x.l;
        }
    }
    bstart[nb] = (uint16_t)ns;
    sstart[ns] = (uint16_t)np;
    uint32_t acc = 0;
    for (int w = 0; w < MQ_WORDS; w++) {
        rank[w] = (uint16_t)acc;
        acc += (uint32_t)__builtin_popcount(bits[w]);
    }
    return np == 0 && ns == nb;
}

BatchLayout layout_of(const BatchJob &j, uint64_t single)
{
    BatchLayout L;
    const uint64_t np = j.bpats.size();
    uint64_t o = 0;
    L.pats = o;
    o = align_up(o + np * sizeof(BatchPat), 256);
    L.groups = o;
    o = align_up(o + j.groups.size() * sizeof(BatchGroup), 256);
    L.cgroups = o;
    o = align_up(o + j.cgroups.size() * sizeof(BatchGroup), 256);
    L.mqgroups = o;
    o = align_up(o + j.mq.size() * sizeof(MqGroup), 256);
    L.mqtabs = o;
    o = align_up(o + j.mqtab.size(), 256);
    L.mqwtabs = o;
    o = align_up(o + j.mqwtab.size(), 256);
    L.params = o;
    o = align_up(o + np * sizeof(Params), 256);
    L.patbytes = o;
    o = align_up(o + j.patbytes, 256);
    L.cnt = o;
    o = align_up(o + np * j.nchunks * 4, 256);
    L.chunk_off = o;
    o = align_up(o + np * j.nchunks * 8, 256);
    L.totals = o;
    o = align_up(o + (uint64_t)j.P * 8, 256);
    L.csr = o;
    o = align_up(o + ((uint64_t)j.P + 1) * 8, 256);
    L.wgroups = o;
    o = align_up(o + np * sizeof(BatchGroup), 16);
    L.wroute = o;
    o = align_up(o + np, 16);
    L.mqwlist = o;
    o = align_up(o + j.mq.size() * 4, 256);
    L.hqgroups = o;
    o = align_up(o + (uint64_t)j.max_hq * sizeof(MqGroup), 256);
    L.hqtabs = o;
    o = align_up(o + (uint64_t)j.max_hq * MQ_TAB_BYTES, 256);
    const uint64_t items = j.stash ? j.nchunks * j.mq.size() : 0;
    L.mqstash = o;
    o = align_up(o + items * MQ_STASH * 4, 256);
    L.mqstash_n = o;
    o = align_up(o + items * 4, 256);
    L.single = o;
    o = align_up(o + single, 256);
    L.need = o;
    return L;
}

__global__ void fill_u64_kernel(uint64_t *p, uint64_t n, uint64_t v)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t st)
{
    if (!n) return hipSuccess;
    uint64_t g = (n + 255) / 256;
    if (g > 1024) g = 1024;
    hipLaunchKernelGGL(fill_u64_kernel, dim3((uint32_t)g), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

BatchLaunch launch_of(const BatchJob &j, uint8_t *ws)
{
    BatchLaunch B;
    memset(&B, 0, sizeof B);
    B.text = j.c->d_text;
    B.n = j.c->n;
    B.pats = reinterpret_cast<const BatchPat *>(ws + j.L.pats);
    B.groups = reinterpret_cast<const BatchGroup *>(ws + j.L.groups);
    B.host_groups = j.groups.data();
    B.cgroups = reinterpret_cast<const BatchGroup *>(ws + j.L.cgroups);
    B.host_cgroups = j.cgroups.data();
    B.ncgroups = (uint32_t)j.cgroups.size();
    B.mqgroups = reinterpret_cast<const MqGroup *>(ws + j.L.mqgroups);
    B.host_mq = j.mq.data();
    B.mqtabs = ws + j.L.mqtabs;
    B.mqwtabs = ws + j.L.mqwtabs;
    B.nmq = (uint32_t)j.mq.size();
    if (j.stash && j.nchunks && !j.mq.empty()) {
        B.mqstash = reinterpret_cast<uint32_t *>(ws + j.L.mqstash);
        B.mqstash_n = reinterpret_cast<uint32_t *>(ws + j.L.mqstash_n);
    }
    B.mq_max_m = j.mq_max_m;
    B.params = reinterpret_cast<const Params *>(ws + j.L.params);
    B.patbytes = ws + j.L.patbytes;
    B.npats = (uint32_t)j.bpats.size();
    B.npats_total = j.P;
    B.ngroups = (uint32_t)j.groups.size();
    B.chunk_tiles = j.chunk_tiles;
    B.nchunks = j.nchunks;
    B.ntiles = j.ntiles;
    B.cnt = reinterpret_cast<uint32_t *>(ws + j.L.cnt);
    return B;
}

int check_corpus(const sm_corpus *c)
{
    if (!c) return err(SM_EINVAL, "corpus is NULL");
    if (hipSetDevice(c->dev) != hipSuccess) return err(SM_EDEVICE, "cannot select the corpus's device");
    return SM_OK;
}

int check_ws(const BatchJob &j, const void *d_work, uint64_t work_bytes)
{
    if (!d_work || work_bytes < j.L.need)
        return err(SM_EINVAL, "workspace too small: need %llu bytes", (unsigned long long)j.L.need);
    if ((uintptr_t)d_work & 255) return err(SM_EINVAL, "workspace must be 256-byte aligned");
    return SM_OK;
}

struct DevFree {
    void *p = nullptr;
    ~DevFree()
    {
        if (p) (void)hipFree(p);
    }
};

}  // namespace

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
int sm::batch_plan(sm_corpus *c, const uint8_t *pats, const uint64_t *pat_off, uint32_t P, int ws,
                   BatchJob &j)
{
    if (!pats || !pat_off) return err(SM_EINVAL, "patterns or offsets are NULL");
    j.c = c;
    j.P = P;
    j.pats = pats;
    j.pat_off = pat_off;
    const int sigma = corpus_sigma(c);
    uint64_t min_m = UINT64_MAX, single = 0;
    for (uint32_t i = 0; i < P; i++) {
        if (pat_off[i + 1] < pat_off[i]) return err(SM_EINVAL, "pattern offsets decrease at %u", i);
        const uint64_t m = pat_off[i + 1] - pat_off[i];
        if (m == 0) return err(SM_EINVAL, "pattern %u is empty", i);
        if (m > 0xFFFFFFFFull) return err(SM_EINVAL, "pattern %u is longer than 2^32-1", i);
        if (m > c->n) continue;  // no occurrence
        if (m > (uint64_t)BATCH_MAX_M) {
            j.longp.push_back(i);
            sm_opts o;
            memset(&o, 0, sizeof o);
            o.sigma_hint = sigma;  // planned with the corpus's alphabet, as the search will be
            single = std::max(single, sm_workspace_size(c->n, m, &o));
            continue;
        }
        Plan p;
        int r = plan_pattern(pats + pat_off[i], m, sigma, p);
        if (r) return r;
        if (p.algo == ALGO_BLOCK || p.algo == ALGO_BRUTE || p.algo == ALGO_FSBNDM ||  // single-pattern
            ((p.algo == ALGO_SHIFT_AND || p.algo == ALGO_SBNDM) &&  // only: the batch takes Hash-q,
             m > (uint64_t)BP_MAX_M)) {                              // Shift-And or SBNDM (m <= 64)
            sm_opts o;
            memset(&o, 0, sizeof o);
            o.algo = p.algo == ALGO_BRUTE ? ALGO_SHIFT_AND : (p.algo == ALGO_FSBNDM ? ALGO_SBNDM : ALGO_HASHQ);
            o.sigma_hint = sigma;
            if ((r = plan_pattern_opts(pats + pat_off[i], m, &o, p))) return r;
        }
        BatchPat bp;
        memset(&bp, 0, sizeof bp);
        bp.m = (uint32_t)m;
        bp.algo = (uint32_t)p.algo;
        bp.q = (uint32_t)p.q;
        bp.hbits = (uint32_t)std::min(p.hbits, BATCH_HBITS_MAX);
        bp.var = (uint32_t)var_of(p);
        bp.index = i;
        j.bpats.push_back(bp);
        min_m = std::min<uint64_t>(min_m, m);
    }
    std::stable_sort(j.bpats.begin(), j.bpats.end(), [](const BatchPat &x, const BatchPat &y) {
        if (x.algo != y.algo) return x.algo < y.algo;
        if (x.var != y.var) return x.var < y.var;
        return x.m < y.m;
    });
    uint64_t off = 0;
    for (auto &bp : j.bpats) {
        bp.pat_off = off;
        off += pat_region(bp.m);
    }
    j.patbytes = off;
    j.mq_of.assign(j.bpats.size(), -1);
    // q-classes (q = min(m, MQ_QMAX)) with at least MQ_MIN patterns are counted by
    // the prefix filter; the others by their own scanners
    std::vector<uint32_t> qcount(MQ_QMAX + 1, 0);
    for (const auto &bp : j.bpats) qcount[std::min<uint32_t>(bp.m, MQ_QMAX)]++;
    auto in_mq = [&](const BatchPat &bp) { return qcount[std::min<uint32_t>(bp.m, MQ_QMAX)] >= (uint32_t)MQ_MIN; };
    // groups: consecutive sorted patterns of one kernel variant, within the LDS
    // table budget; the count groups also stop at filtered patterns
    auto make_groups = [&](std::vector<BatchGroup> &out, bool skip_mq) {
        for (uint32_t k = 0; k < j.bpats.size();) {
            if (skip_mq && in_mq(j.bpats[k])) {
                k++;
                continue;
            }
            const BatchPat &b = j.bpats[k];
            const uint32_t cap =
                (uint32_t)std::min<int>(BATCH_GROUP_MAX, BATCH_TABLE_BYTES / table_bytes(b.algo, b.var));
            BatchGroup g;
            memset(&g, 0, sizeof g);
            g.first = k;
            g.algo = b.algo;
            g.var = b.var;
            while (k < j.bpats.size() && g.count < cap && j.bpats[k].algo == b.algo &&
                   j.bpats[k].var == b.var && !(skip_mq && in_mq(j.bpats[k]))) {
                g.max_m = std::max(g.max_m, j.bpats[k].m);
                g.count++;
                k++;
            }
            out.push_back(g);
        }
    };
    make_groups(j.groups, false);
    make_groups(j.cgroups, true);
    // filter groups: each q-class by length, cut into groups of MQ_G
    for (uint32_t q = 1; q <= (uint32_t)MQ_QMAX; q++) {
        if (qcount[q] < (uint32_t)MQ_MIN) continue;
        std::vector<uint32_t> mem;
        for (uint32_t k = 0; k < j.bpats.size(); k++)
            if (std::min<uint32_t>(j.bpats[k].m, MQ_QMAX) == q) mem.push_back(k);
        std::stable_sort(mem.begin(), mem.end(), [&](uint32_t x, uint32_t y) { return j.bpats[x].m < j.bpats[y].m; });
        for (size_t b = 0; b < mem.size(); b += MQ_G) {
            const size_t e = std::min(mem.size(), b + (size_t)MQ_G);
            MqGroup g;
            memset(&g, 0, sizeof g);
            g.count = (uint32_t)(e - b);
            g.q = q;
            g.min_m = j.bpats[mem[b]].m;
            g.max_m = j.bpats[mem[e - 1]].m;
            g.tab_off = (uint64_t)j.mq.size() * MQ_TAB_BYTES;
            j.mq_max_m = std::max(j.mq_max_m, g.max_m);
            j.mq.push_back(g);
            j.mqtab.resize(j.mqtab.size() + MQ_TAB_BYTES, 0);
            j.mq.back().flat = build_mq_table(j, mem.data() + b, g.count, q, j.mqtab.data() + g.tab_off, true) ? 1u : 0u;
            j.mqwtab.resize(j.mqtab.size(), 0);
            build_mq_table(j, mem.data() + b, g.count, q, j.mqwtab.data() + g.tab_off, false);
            for (size_t e2 = b; e2 < e; e2++) j.mq_of[mem[e2]] = (int32_t)(j.mq.size() - 1);
        }
    }
    if (j.patbytes >= (1ull << 32)) return err(SM_EINVAL, "batch patterns exceed 4 GiB");
    j.stash = ws == WS_WRITE;
    j.max_hq = (uint32_t)(j.bpats.size() / MQ_G + MQ_QMAX);
    if (!j.bpats.empty()) {
        j.ntiles = (c->n - min_m + 1 + BT - 1) / BT;
        // aim for several thousand (chunk, group) items in the count pass
        const uint64_t ng = std::max<uint64_t>(1, j.cgroups.size() + j.mq.size());
        uint64_t want = j.ntiles * ng / 8192;
        uint32_t ct = 1;
        while ((uint64_t)ct * 2 <= want && ct < 256) ct *= 2;
        j.chunk_tiles = ct;
        j.nchunks = (j.ntiles + ct - 1) / ct;
    }
    if (ws == WS_WRITE && !j.bpats.empty()) {
        // single-pattern scratch for every m up to single_max_m
        uint32_t top = 0;
        for (const auto &bp : j.bpats) top = std::max(top, bp.m);
        j.single_max_m = std::min<uint32_t>(top, SINGLE_ROUTE_MAX_M);
        single = std::max(single, sm_workspace_size_upto(c->n, j.single_max_m, nullptr));
    }
    j.L = layout_of(j, ws == WS_NONE ? 0 : single);
    return SM_OK;
}

uint64_t sm::batch_image_bytes(const BatchJob &j) { return j.L.cnt; }

uint64_t sm::batch_stash_items(const BatchJob &j) { return j.stash ? j.nchunks * j.mq.size() : 0; }

void sm::batch_fill_image(const BatchJob &j, uint8_t *h)
{
    memset(h, 0, j.L.cnt);
    memcpy(h + j.L.pats, j.bpats.data(), j.bpats.size() * sizeof(BatchPat));
    memcpy(h + j.L.groups, j.groups.data(), j.groups.size() * sizeof(BatchGroup));
    memcpy(h + j.L.cgroups, j.cgroups.data(), j.cgroups.size() * sizeof(BatchGroup));
    memcpy(h + j.L.mqgroups, j.mq.data(), j.mq.size() * sizeof(MqGroup));
    memcpy(h + j.L.mqtabs, j.mqtab.data(), j.mqtab.size());
    memcpy(h + j.L.mqwtabs, j.mqwtab.data(), j.mqwtab.size());
    for (const auto &bp : j.bpats) memcpy(h + j.L.patbytes + bp.pat_off, j.pats + j.pat_off[bp.index], bp.m);
}

// ---------------------------------------------------------------------------
// count and write steps
// ---------------------------------------------------------------------------
int sm::batch_count_enqueue(BatchJob &j, uint8_t *ws, const uint8_t *h_image, uint64_t *d_totals,
                            uint64_t *d_csr, bool keep_chunk_off, hipStream_t st)
{
    HIP_OK(fill_u64(d_totals, j.P, 0, st));
    if (!j.bpats.empty()) {
        std::vector<uint8_t> own;
        if (!h_image) {
            own.resize(batch_image_bytes(j));
            batch_fill_image(j, own.data());
            h_image = own.data();
        }
        // the params region is written by the prep kernel; copy around it
        HIP_OK(hipMemcpyAsync(ws, h_image, j.L.params, hipMemcpyHostToDevice, st));
        HIP_OK(hipMemcpyAsync(ws + j.L.patbytes, h_image + j.L.patbytes, j.L.cnt - j.L.patbytes,
                              hipMemcpyHostToDevice, st));
        BatchLaunch B = launch_of(j, ws);
        B.chunk_off_out = keep_chunk_off ? reinterpret_cast<uint64_t *>(ws + j.L.chunk_off) : nullptr;
        B.totals = d_totals;
        B.csr_out = nullptr;  // long patterns first, the CSR below
        B.write = false;
        B.prep = true;
        HIP_OK(launch_batch(B, st));
    }
    for (uint32_t i : j.longp) {
        const uint64_t m = j.pat_off[i + 1] - j.pat_off[i];
        int r = sm_corpus_count_async(j.c, j.pats + j.pat_off[i], m, d_totals + i, ws + j.L.single,
                                      j.L.need - j.L.single, nullptr, st);
        if (r) return r;
    }
    if (d_csr) HIP_OK(launch_csr_scan(d_totals, j.P, d_csr, st));
    return SM_OK;
}

namespace {
// 0 automatic, 1 own scanners only, 2 shared filter when sparse, 3 single-pattern
// pipeline wherever the workspace allows
std::atomic<int> g_write_policy{0};
}

extern "C" int sm_batch_set_write_policy(int policy)
{
    if (policy < 0 || policy > 3) return err(SM_EINVAL, "write policy must be 0, 1, 2 or 3");
    g_write_policy = policy;
    return SM_OK;
}

sm::PlanStaging::~PlanStaging()
{
    if (ev) {
        (void)hipEventSynchronize(ev);
        (void)hipEventDestroy(ev);
    }
    if (host) (void)hipHostFree(host);
}

int sm::batch_write_plan(BatchJob &j, uint8_t *ws, const uint64_t *h_csr, uint64_t lo, uint64_t hi,
                         hipStream_t st, PlanStaging &stg)
{
    const int policy = g_write_policy;
    j.wplan = true;
    j.wgroups.clear();
    j.mqwlist.clear();
    j.hq.clear();
    j.hqtab.clear();
    j.singlep.clear();
    j.wroute.assign(j.bpats.size(), 0);
    if (j.bpats.empty()) return SM_OK;
    // A pattern may share its count group's filter write pass when its hits are
    // sparse enough to be sorted in LDS (at most 16 per 4096 starts on average). That
    // pass copies out the hits the count step kept -- those of a pattern with at most
    // MQ_CAP hits in a chunk, in the chunks whose item did not overflow -- and scans
    // the other chunks again at about 2/5 of a per-pattern rescan's rate. So a
    // pattern whose hits are mostly kept (on average at most MQ_CAP / 2 per chunk, in
    // a group that kept most items) shares the pass; a heavier one does when the
    // rescans of all such patterns of its group exceed 2.5 texts. A pattern with at
    // least one occurrence per SINGLE_ROUTE_DENSITY text bytes in the window goes to
    // the single-pattern pipeline instead: one text read plus a coalesced emit,
    // against 40 to 60 ps per position written from a batch pass.
    const double n = (double)j.c->n, nch = (double)j.nchunks;
    const double chunk_bytes = (double)j.chunk_tiles * BT;
    const size_t nmq = j.mq.size();
    // per filter group: the fraction of chunks whose item overflowed (1: unknown)
    std::vector<double> ovf(nmq, 1.0);
    if (j.stash && j.h_stash_n && j.nchunks) {
        for (size_t g = 0; g < nmq; g++) {
            uint64_t k = 0;
            for (uint64_t c = 0; c < j.nchunks; c++) k += j.h_stash_n[c * nmq + g] > MQ_STASH;
            ovf[g] = (double)k / nch;
        }
    }
    // 0: none, 1: own scanner, 2: filter, 3: single-pattern pipeline
    std::vector<uint8_t> &route = j.wroute;
    std::vector<double> wcount(j.bpats.size(), 0.0);  // occurrences inside the window
    std::vector<uint8_t> heavy(j.bpats.size(), 0);    // routed to the filter, hits mostly not kept
    std::vector<double> gcover(nmq, 0.0);
    for (size_t k = 0; k < j.bpats.size(); k++) {
        const uint32_t i = j.bpats[k].index;
        // occurrences of this pattern inside the window [lo, hi)
        const uint64_t a0 = std::max(h_csr[i], lo), a1 = std::min(h_csr[i + 1], hi);
        const double c = a0 < a1 ? (double)(a1 - a0) : 0.0;
        if (c == 0) continue;
        wcount[k] = c;
        if (j.bpats[k].m <= j.single_max_m &&
            (policy == 3 || (policy == 0 && c * SINGLE_ROUTE_DENSITY >= n))) {
            route[k] = 3;
            j.singlep.push_back(i);
            continue;
        }
        const int32_t g = j.mq_of[k];
        const bool sparse = c * 4096.0 / n <= 16.0;
        route[k] = 1;
        if (g < 0 || !sparse || policy == 1) continue;
        const double total = (double)(h_csr[i + 1] - h_csr[i]);
        const bool kept = ovf[g] <= 0.25 && total <= nch * (MQ_CAP / 2);
        const double cover = nch * (1.0 - std::exp(-c / nch)) * chunk_bytes;
        if (kept) {
            route[k] = 2;
        } else if (policy == 2 || cover * 16 >= n) {
            route[k] = 4;
            heavy[k] = 1;
            gcover[g] += cover;
        }
    }
    if (policy == 0) {
        for (size_t k = 0; k < j.bpats.size(); k++)
            if (heavy[k] && gcover[j.mq_of[k]] < 2.5 * n) route[k] = 1;
    }
    if (policy == 0 && j.single_max_m) {
        // The heavy patterns of a group cost a text pass of the group's filter; when
        // that exceeds searching them one by one (about one text read each, plus the
        // coalesced emit), the single-pattern pipeline takes them.
        std::vector<double> alone(nmq, 0.0);
        std::vector<uint8_t> can(nmq, 1);
        for (size_t k = 0; k < j.bpats.size(); k++) {
            if (route[k] != 4) continue;
            const int32_t g = j.mq_of[k];
            if (j.bpats[k].m > j.single_max_m) can[g] = 0;
            alone[g] += n * SINGLE_COST_PER_BYTE + wcount[k] * SINGLE_COST_PER_POS;
        }
        for (size_t k = 0; k < j.bpats.size(); k++) {
            if (route[k] != 4) continue;
            const int32_t g = j.mq_of[k];
            if (can[g] && alone[g] < n * FILTER_COST_PER_BYTE) {
                route[k] = 3;
                j.singlep.push_back(j.bpats[k].index);
            }
        }
    }
    // per-pattern write groups: consecutive sorted patterns routed to their own scanner
    for (uint32_t k = 0; k < j.bpats.size();) {
        if (route[k] != 1) {
            k++;
            continue;
        }
        const BatchPat &b = j.bpats[k];
        const uint32_t cap =
            (uint32_t)std::min<int>(BATCH_GROUP_MAX, BATCH_TABLE_BYTES / table_bytes(b.algo, b.var));
        BatchGroup g;
        memset(&g, 0, sizeof g);
        g.first = k;
        g.algo = b.algo;
        g.var = b.var;
        while (k < j.bpats.size() && g.count < cap && route[k] == 1 && j.bpats[k].algo == b.algo &&
               j.bpats[k].var == b.var) {
            g.max_m = std::max(g.max_m, j.bpats[k].m);
            g.count++;
            k++;
        }
        if (g.count == 0) {
            k++;
            continue;
        }
        j.wgroups.push_back(g);
    }
    // count groups with patterns written from the kept hits (ascending: q order)
    {
        std::vector<uint8_t> used(nmq, 0);
        for (size_t k = 0; k < j.bpats.size(); k++)
            if (route[k] == 2) used[j.mq_of[k]] = 1;
        for (size_t g = 0; g < nmq; g++)
            if (used[g]) j.mqwlist.push_back((uint32_t)g);
    }
    // filter pass groups of the heavy patterns: every q-class together, by length, in
    // groups of MQ_G, each hashing the prefix its shortest pattern has (q = min(m,
    // MQ_QMAX)): a pass over the text costs per start whatever the group holds, so a
    // window's few heavy patterns of several lengths share one pass
    {
        std::vector<uint32_t> mem;
        for (uint32_t k = 0; k < j.bpats.size(); k++)
            if (route[k] == 4) mem.push_back(k);
        std::stable_sort(mem.begin(), mem.end(), [&](uint32_t x, uint32_t y) { return j.bpats[x].m < j.bpats[y].m; });
        for (size_t b = 0; b < mem.size(); b += MQ_G) {
            const size_t e = std::min(mem.size(), b + (size_t)MQ_G);
            const uint32_t q = std::min<uint32_t>(j.bpats[mem[b]].m, MQ_QMAX);
            MqGroup g;
            memset(&g, 0, sizeof g);
            g.count = (uint32_t)(e - b);
            g.q = q;
            g.min_m = j.bpats[mem[b]].m;
            g.max_m = j.bpats[mem[e - 1]].m;
            g.tab_off = (uint64_t)j.hq.size() * MQ_TAB_BYTES;
            j.hq.push_back(g);
            j.hqtab.resize(j.hqtab.size() + MQ_TAB_BYTES, 0);
            build_mq_table(j, mem.data() + b, g.count, q, j.hqtab.data() + g.tab_off, false);
        }
    }
    if (j.hq.size() > j.max_hq) return err(SM_EDEVICE, "internal: write plan larger than its workspace");
    // the plan into the workspace region [L.wgroups, L.mqwlist + list), one copy from
    // pinned staging that no earlier upload still reads
    const uint64_t bytes = j.L.hqtabs + j.hqtab.size() - j.L.wgroups;
    if (stg.pending) {
        HIP_OK(hipEventSynchronize(stg.ev));
        stg.pending = false;
    }
    if (!stg.ev) HIP_OK(hipEventCreateWithFlags(&stg.ev, hipEventDisableTiming));
    if (stg.cap < bytes) {
        if (stg.host) HIP_OK(hipHostFree(stg.host));
        stg.host = nullptr;
        stg.cap = 0;
        HIP_OK(hipHostMalloc((void **)&stg.host, bytes, hipHostMallocDefault));
        stg.cap = bytes;
    }
    uint8_t *h = stg.host;
    memcpy(h, j.wgroups.data(), j.wgroups.size() * sizeof(BatchGroup));
    memcpy(h + (j.L.wroute - j.L.wgroups), j.wroute.data(), j.wroute.size());
    memcpy(h + (j.L.mqwlist - j.L.wgroups), j.mqwlist.data(), j.mqwlist.size() * 4);
    memcpy(h + (j.L.hqgroups - j.L.wgroups), j.hq.data(), j.hq.size() * sizeof(MqGroup));
    memcpy(h + (j.L.hqtabs - j.L.wgroups), j.hqtab.data(), j.hqtab.size());
    HIP_OK(hipMemcpyAsync(ws + j.L.wgroups, h, bytes, hipMemcpyHostToDevice, st));
    HIP_OK(hipEventRecord(stg.ev, st));
    stg.pending = true;
    return SM_OK;
}

int sm::batch_write_enqueue(BatchJob &j, uint8_t *ws, const uint64_t *d_csr, const uint64_t *h_csr,
                            uint64_t *d_totals, int64_t *d_out, uint64_t lo, uint64_t hi,
                            hipStream_t st)
{
    if (hi <= lo) return SM_OK;
    if (!j.bpats.empty()) {
        BatchLaunch B = launch_of(j, ws);
        if (j.wplan) {
            B.groups = reinterpret_cast<const BatchGroup *>(ws + j.L.wgroups);
            B.host_groups = j.wgroups.data();
            B.ngroups = (uint32_t)j.wgroups.size();
            B.mqwlist = reinterpret_cast<const uint32_t *>(ws + j.L.mqwlist);
            B.host_mqwlist = j.mqwlist.data();
            B.nmqw = (uint32_t)j.mqwlist.size();
            B.wroute = ws + j.L.wroute;
            B.hqgroups = reinterpret_cast<const MqGroup *>(ws + j.L.hqgroups);
            B.host_hq = j.hq.data();
            B.hqtabs = ws + j.L.hqtabs;
            B.nhq = (uint32_t)j.hq.size();
        }
        B.chunk_off = reinterpret_cast<const uint64_t *>(ws + j.L.chunk_off);
        B.csr = d_csr;
        B.out = d_out;
        B.lo = lo;
        B.span = hi - lo;
        B.write = true;
        HIP_OK(launch_batch(B, st));
    }
    if ((!j.longp.empty() || !j.singlep.empty()) && !h_csr)
        return err(SM_EINVAL, "single-pattern searches need the host offsets");
    // one search each, into the window's part of its slice. Identical patterns have
    // identical position lists (short patterns over a small alphabet necessarily repeat
    // in a large batch): a pattern whose ranks in this window were already written for an
    // identical one is copied from there, device to device, instead of searched again.
    std::unordered_map<std::string_view, uint32_t> written;  // pattern bytes -> written index
    for (const auto *list : {&j.longp, &j.singlep}) {
        for (uint32_t i : *list) {
            const uint64_t a = std::max(h_csr[i], lo), b = std::min(h_csr[i + 1], hi);
            if (a >= b) continue;
            const uint64_t m = j.pat_off[i + 1] - j.pat_off[i];
            const std::string_view key(reinterpret_cast<const char *>(j.pats + j.pat_off[i]), (size_t)m);
            const auto it = written.find(key);
            if (it != written.end()) {
                // rank a - h_csr[i] of this pattern is CSR entry src of the written one
                const uint64_t src = h_csr[it->second] + (a - h_csr[i]);
                if (src >= lo && src + (b - a) <= hi) {
                    HIP_OK(hipMemcpyAsync(d_out + (a - lo), d_out + (src - lo), (b - a) * sizeof(int64_t),
                                          hipMemcpyDeviceToDevice, st));
                    continue;
                }
            }
            int r = corpus_find_window_async(j.c, j.pats + j.pat_off[i], m, d_out + (a - lo), a - h_csr[i], b - a,
                                             d_totals + i, ws + j.L.single, j.L.need - j.L.single, st);
            if (r) return r;
            // keep as the source the identical pattern with the most ranks in the window
            if (it == written.end()) {
                written.emplace(key, i);
            } else {
                const uint32_t w = it->second;
                const uint64_t wa = std::max(h_csr[w], lo), wb = std::min(h_csr[w + 1], hi);
                if (b - a > wb - wa) it->second = i;
            }
        }
    }
    return SM_OK;
}

// ---------------------------------------------------------------------------
// batch handle: count once, write windows
// ---------------------------------------------------------------------------
struct sm_batch {
    BatchJob j;
    PlanStaging stg;
    std::vector<uint8_t> pats;
    std::vector<uint64_t> pat_off;
    std::vector<uint64_t> csr;  // host copy, P + 1
    std::vector<uint32_t> stash_n;  // host copy: hits of each (chunk, filter group) item
    uint8_t *ws = nullptr;
    ~sm_batch()
    {
        if (ws) (void)hipFree(ws);
    }
};

extern "C" int sm_batch_open(sm_corpus *c, const uint8_t *pats, const uint64_t *pat_off, uint32_t P,
                             sm_batch **out)
{
    if (!out) return err(SM_EINVAL, "batch is NULL");
    *out = nullptr;
    TraceRange tr("batch.count");
    int r = check_corpus(c);
    if (r) return r;
    if (!pats || !pat_off) return err(SM_EINVAL, "patterns or offsets are NULL");
    for (uint32_t i = 0; i < P; i++)
        if (pat_off[i + 1] < pat_off[i]) return err(SM_EINVAL, "pattern offsets decrease at %u", i);
    std::unique_ptr<sm_batch> b(new (std::nothrow) sm_batch);
    if (!b) return err(SM_ENOMEM, "out of host memory");
    // own copy of the patterns: long patterns are read again by every write
    const uint64_t base = pat_off[0];
    b->pat_off.resize((uint64_t)P + 1);
    for (uint64_t i = 0; i <= P; i++) b->pat_off[i] = pat_off[i] - base;
    b->pats.assign(pats + base, pats + pat_off[P]);
    b->pats.resize(b->pats.size() + 16);
    if ((r = batch_plan(c, b->pats.data(), b->pat_off.data(), P, WS_WRITE, b->j))) return r;
    HIP_OK(hipMalloc((void **)&b->ws, b->j.L.need));
    uint64_t *d_tot = (uint64_t *)(b->ws + b->j.L.totals), *d_csr = (uint64_t *)(b->ws + b->j.L.csr);
    if ((r = batch_count_enqueue(b->j, b->ws, nullptr, d_tot, d_csr, true, nullptr))) return r;
    b->csr.resize((uint64_t)P + 1);
    HIP_OK(hipMemcpy(b->csr.data(), d_csr, ((uint64_t)P + 1) * 8, hipMemcpyDeviceToHost));
    const uint64_t items = batch_stash_items(b->j);
    if (items) {
        b->stash_n.resize(items);
        HIP_OK(hipMemcpy(b->stash_n.data(), b->ws + b->j.L.mqstash_n, items * 4, hipMemcpyDeviceToHost));
        b->j.h_stash_n = b->stash_n.data();
    }
    *out = b.release();
    return SM_OK;
}

extern "C" int sm_batch_offsets(const sm_batch *b, uint64_t *out_off)
{
    if (!b || !out_off) return err(SM_EINVAL, "batch or out_off is NULL");
    memcpy(out_off, b->csr.data(), b->csr.size() * 8);
    return SM_OK;
}

extern "C" int sm_batch_write_async(sm_batch *b, uint64_t lo, uint64_t hi, int64_t *d_out, void *stream)
{
    if (!b) return err(SM_EINVAL, "batch is NULL");
    const uint64_t total = b->csr.back();
    if (lo > hi || hi > total)
        return err(SM_EINVAL, "window [%llu, %llu) outside [0, %llu)", (unsigned long long)lo,
                   (unsigned long long)hi, (unsigned long long)total);
    if (hi > lo && !d_out) return err(SM_EINVAL, "d_out is NULL");
    int r = check_corpus(b->j.c);
    if (r) return r;
    if (hi == lo) return SM_OK;
    TraceRange tr("batch.write.enqueue");
    // the write plan of this window: only the patterns whose slices meet it
    if ((r = batch_write_plan(b->j, b->ws, b->csr.data(), lo, hi, (hipStream_t)stream, b->stg))) return r;
    return batch_write_enqueue(b->j, b->ws, (const uint64_t *)(b->ws + b->j.L.csr), b->csr.data(),
                               (uint64_t *)(b->ws + b->j.L.totals), d_out, lo, hi, (hipStream_t)stream);
}

extern "C" int sm_batch_close(sm_batch *b)
{
    if (!b) return SM_OK;
    if (b->ws) {  // writes still in flight read the workspace
        (void)hipSetDevice(b->j.c->dev);
        (void)hipDeviceSynchronize();
    }
    delete b;
    return SM_OK;
}

// ---------------------------------------------------------------------------
// one-call forms
// ---------------------------------------------------------------------------
extern "C" uint64_t sm_batch_workspace_size(const sm_corpus *c, const uint8_t *pats,
                                            const uint64_t *pat_off, uint32_t P)
{
    if (!c) return 0;
    BatchJob j;
    if (batch_plan(const_cast<sm_corpus *>(c), pats, pat_off, P, WS_LONG, j)) return 0;
    return j.L.need;
}

extern "C" int sm_batch_count_async(sm_corpus *c, const uint8_t *pats, const uint64_t *pat_off,
                                    uint32_t P, uint64_t *d_counts, void *d_work,
                                    uint64_t work_bytes, void *stream)
{
    int r = check_corpus(c);
    if (r) return r;
    if (P == 0) return SM_OK;
    if (!d_counts) return err(SM_EINVAL, "d_counts is NULL");
    BatchJob j;
    if ((r = batch_plan(c, pats, pat_off, P, WS_LONG, j))) return r;
    if ((r = check_ws(j, d_work, work_bytes))) return r;
    return batch_count_enqueue(j, (uint8_t *)d_work, nullptr, d_counts, nullptr, false, (hipStream_t)stream);
}

extern "C" int sm_batch_find_all_async(sm_corpus *c, const uint8_t *pats, const uint64_t *pat_off,
                                       uint32_t P, int64_t *d_out, uint64_t cap, uint64_t *d_out_off,
                                       void *d_work, uint64_t work_bytes, void *stream)
{
    int r = check_corpus(c);
    if (r) return r;
    if (P == 0) return SM_OK;
    if (!d_out_off) return err(SM_EINVAL, "d_out_off is NULL");
    if (!d_out && cap > 0) return err(SM_EINVAL, "d_out is NULL with cap > 0");
    BatchJob j;
    if ((r = batch_plan(c, pats, pat_off, P, WS_NONE, j))) return r;
    if (!j.longp.empty())
        return err(SM_EINVAL, "asynchronous batched find_all takes patterns up to %d bytes (use sm_batch_find_all)",
                   BATCH_MAX_M);
    if ((r = check_ws(j, d_work, work_bytes))) return r;
    uint8_t *ws = (uint8_t *)d_work;
    hipStream_t st = (hipStream_t)stream;
    uint64_t *d_tot = (uint64_t *)(ws + j.L.totals);
    if ((r = batch_count_enqueue(j, ws, nullptr, d_tot, d_out_off, true, st))) return r;
    // entries at or past the total are never produced, so [0, cap) is the whole prefix
    return batch_write_enqueue(j, ws, d_out_off, nullptr, d_tot, d_out, 0, cap, st);
}

extern "C" int sm_batch_count(sm_corpus *c, const uint8_t *pats, const uint64_t *pat_off, uint32_t P,
                              uint64_t *counts)
{
    int r = check_corpus(c);
    if (r) return r;
    if (P == 0) return SM_OK;
    if (!counts) return err(SM_EINVAL, "counts is NULL");
    BatchJob j;
    if ((r = batch_plan(c, pats, pat_off, P, WS_LONG, j))) return r;
    DevFree ws;
    HIP_OK(hipMalloc(&ws.p, j.L.need));
    uint64_t *d_tot = (uint64_t *)((uint8_t *)ws.p + j.L.totals);
    if ((r = batch_count_enqueue(j, (uint8_t *)ws.p, nullptr, d_tot, nullptr, false, nullptr))) return r;
    HIP_OK(hipMemcpy(counts, d_tot, (uint64_t)P * 8, hipMemcpyDeviceToHost));
    return SM_OK;
}

namespace {
constexpr uint64_t WAVE_DEFAULT = 64ull << 30;
uint64_t g_wave_bytes = WAVE_DEFAULT;  // output-wave budget of sm_batch_find_all
}

extern "C" int sm_batch_set_wave_bytes(uint64_t bytes)
{
    if (bytes != 0 && bytes < 8) return err(SM_EINVAL, "wave budget below one position");
    g_wave_bytes = bytes ? bytes : WAVE_DEFAULT;
    return SM_OK;
}

extern "C" int sm_batch_find_all(sm_corpus *c, const uint8_t *pats, const uint64_t *pat_off, uint32_t P,
                                 int64_t *out, uint64_t cap, uint64_t *out_off)
{
    int r = check_corpus(c);
    if (r) return r;
    if (!out_off) return err(SM_EINVAL, "out_off is NULL");
    if (P == 0) {
        out_off[0] = 0;
        return SM_OK;
    }
    if (!out && cap > 0) return err(SM_EINVAL, "out is NULL with cap > 0");
    sm_batch *b = nullptr;
    if ((r = sm_batch_open(c, pats, pat_off, P, &b))) return r;
    std::unique_ptr<sm_batch, int (*)(sm_batch *)> hold(b, sm_batch_close);
    memcpy(out_off, b->csr.data(), ((uint64_t)P + 1) * 8);
    const uint64_t total = out_off[P];
    const uint64_t dcap = std::min(cap, total);
    // output in waves: the device never holds more than the wave budget of positions
    size_t free_b = 0, tot_b = 0;
    HIP_OK(hipMemGetInfo(&free_b, &tot_b));
    uint64_t wave = std::min<uint64_t>(g_wave_bytes / 8, std::max<uint64_t>(free_b / 16, 1ull << 20));
    wave = std::max<uint64_t>(std::min(wave, dcap), 1);
    DevFree dbuf;
    if (dcap) HIP_OK(hipMalloc(&dbuf.p, wave * 8));
    for (uint64_t lo = 0; lo < dcap; lo += wave) {
        TraceRange tw("batch.wave (write + copy to host)");
        const uint64_t hi = std::min(dcap, lo + wave);
        if ((r = sm_batch_write_async(b, lo, hi, (int64_t *)dbuf.p, nullptr))) return r;
        HIP_OK(hipMemcpy(out + lo, dbuf.p, (hi - lo) * 8, hipMemcpyDeviceToHost));
    }
    HIP_OK(hipDeviceSynchronize());
    return total > cap ? SM_TRUNCATED : SM_OK;
}
