// C ABI of the batched multi-pattern search: planning and grouping of the
// patterns, workspace layout, launches (sm_batch.hip) and the synchronous forms.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/sm.h"
#include "sm_internal.h"

using namespace sm;

namespace {

int err(int status, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    sm_set_error(status, buf);
    return status;
}

#define HIP_OK(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return err(e_ == hipErrorOutOfMemory ? SM_ENOMEM : SM_EDEVICE, "%s: %s", #expr, \
                       hipGetErrorString(e_));                                              \
    } while (0)

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

struct HostPlan {
    std::vector<BatchPat> pats;     // batch patterns, sorted by (algo, var, m)
    std::vector<BatchGroup> groups;
    std::vector<uint32_t> longp;    // m > BATCH_MAX_M: searched one at a time
    uint64_t patbytes = 0;
    uint32_t chunk_tiles = 1;
    uint64_t nchunks = 0, ntiles = 0;
};

int build_plan(const sm_corpus *c, const uint8_t *pats, const uint64_t *pat_off, uint32_t P,
               HostPlan &hp)
{
    if (!pats || !pat_off) return err(SM_EINVAL, "patterns or offsets are NULL");
    const int sigma = corpus_sigma(c);
    uint64_t min_m = UINT64_MAX;
    for (uint32_t i = 0; i < P; i++) {
        if (pat_off[i + 1] < pat_off[i]) return err(SM_EINVAL, "pattern offsets decrease at %u", i);
        const uint64_t m = pat_off[i + 1] - pat_off[i];
        if (m == 0) return err(SM_EINVAL, "pattern %u is empty", i);
        if (m > 0xFFFFFFFFull) return err(SM_EINVAL, "pattern %u is longer than 2^32-1", i);
        if (m > c->n) continue;  // no occurrence
        if (m > (uint64_t)BATCH_MAX_M) {
            hp.longp.push_back(i);
            continue;
        }
        Plan p;
        int r = plan_pattern(pats + pat_off[i], m, sigma, p);
        if (r) return r;
        BatchPat bp;
        memset(&bp, 0, sizeof bp);
        bp.m = (uint32_t)m;
        bp.algo = (uint32_t)p.algo;
        bp.q = (uint32_t)p.q;
        bp.hbits = (uint32_t)std::min(p.hbits, BATCH_HBITS_MAX);
        bp.var = (uint32_t)var_of(p);
        bp.index = i;
        hp.pats.push_back(bp);
        min_m = std::min<uint64_t>(min_m, m);
    }
    std::stable_sort(hp.pats.begin(), hp.pats.end(), [](const BatchPat &x, const BatchPat &y) {
        if (x.algo != y.algo) return x.algo < y.algo;
        if (x.var != y.var) return x.var < y.var;
        return x.m < y.m;
    });
    uint64_t off = 0;
    for (auto &bp : hp.pats) {
        bp.pat_off = off;
        off += pat_region(bp.m);
    }
    hp.patbytes = off;
    for (uint32_t k = 0; k < hp.pats.size();) {
        const BatchPat &b = hp.pats[k];
        const uint32_t cap =
            (uint32_t)std::min<int>(BATCH_GROUP_MAX, BATCH_TABLE_BYTES / table_bytes(b.algo, b.var));
        BatchGroup g;
        memset(&g, 0, sizeof g);
        g.first = k;
        g.algo = b.algo;
        g.var = b.var;
        while (k < hp.pats.size() && g.count < cap && hp.pats[k].algo == b.algo && hp.pats[k].var == b.var) {
            g.max_m = std::max(g.max_m, hp.pats[k].m);
            g.count++;
            k++;
        }
        hp.groups.push_back(g);
    }
    if (!hp.pats.empty()) {
        hp.ntiles = (c->n - min_m + 1 + BT - 1) / BT;
        // aim for a few thousand (chunk, group) items
        uint64_t want = hp.ntiles * hp.groups.size() / 4096;
        uint32_t ct = 1;
        while ((uint64_t)ct * 2 <= want && ct < 256) ct *= 2;
        hp.chunk_tiles = ct;
        hp.nchunks = (hp.ntiles + ct - 1) / ct;
    }
    return SM_OK;
}

struct Layout {
    uint64_t pats, groups, params, patbytes, cnt, chunk_off, totals, csr, single, need;
};

uint64_t single_ws_need(const sm_corpus *c, const HostPlan &hp, const uint8_t *pats,
                        const uint64_t *pat_off)
{
    uint64_t need = 0;
    for (uint32_t i : hp.longp) {
        const uint64_t m = pat_off[i + 1] - pat_off[i];
        need = std::max(need, sm_workspace_size(c->n, m, nullptr));
    }
    (void)pats;
    return need;
}

Layout layout_of(const HostPlan &hp, uint32_t P, uint64_t single)
{
    Layout L;
    const uint64_t np = hp.pats.size();
    uint64_t o = 0;
    L.pats = o;
    o = align_up(o + np * sizeof(BatchPat), 256);
    L.groups = o;
    o = align_up(o + hp.groups.size() * sizeof(BatchGroup), 256);
    L.params = o;
    o = align_up(o + np * sizeof(Params), 256);
    L.patbytes = o;
    o = align_up(o + hp.patbytes, 256);
    L.cnt = o;
    o = align_up(o + np * hp.nchunks * 4, 256);
    L.chunk_off = o;
    o = align_up(o + np * hp.nchunks * 8, 256);
    L.totals = o;
    o = align_up(o + (uint64_t)P * 8, 256);
    L.csr = o;
    o = align_up(o + ((uint64_t)P + 1) * 8, 256);
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

// Uploads plan + pattern bytes and runs the count pass; totals -> d_totals (by
// original index, all P entries), CSR -> d_csr when not null.
int run_count(sm_corpus *c, const HostPlan &hp, const Layout &L, const uint8_t *pats,
              const uint64_t *pat_off, uint32_t P, uint8_t *ws, uint64_t *d_totals, uint64_t *d_csr,
              bool keep_chunk_off, hipStream_t st)
{
    HIP_OK(fill_u64(d_totals, P, 0, st));
    if (!hp.pats.empty()) {
        // pattern table, groups and pattern bytes: one host image, one copy
        const uint64_t img = L.cnt;  // [pats .. patbytes] precede the count array
        std::vector<uint8_t> h(img, 0);
        memcpy(h.data() + L.pats, hp.pats.data(), hp.pats.size() * sizeof(BatchPat));
        memcpy(h.data() + L.groups, hp.groups.data(), hp.groups.size() * sizeof(BatchGroup));
        for (const auto &bp : hp.pats)
            memcpy(h.data() + L.patbytes + bp.pat_off, pats + pat_off[bp.index], bp.m);
        // the params region is written by the prep kernel; copy around it
        HIP_OK(hipMemcpyAsync(ws, h.data(), L.params, hipMemcpyHostToDevice, st));
        HIP_OK(hipMemcpyAsync(ws + L.patbytes, h.data() + L.patbytes, img - L.patbytes,
                              hipMemcpyHostToDevice, st));
        BatchLaunch B;
        memset(&B, 0, sizeof B);
        B.text = c->d_text;
        B.n = c->n;
        B.pats = reinterpret_cast<const BatchPat *>(ws + L.pats);
        B.groups = reinterpret_cast<const BatchGroup *>(ws + L.groups);
        B.host_groups = hp.groups.data();
        B.params = reinterpret_cast<const Params *>(ws + L.params);
        B.patbytes = ws + L.patbytes;
        B.npats = (uint32_t)hp.pats.size();
        B.npats_total = P;
        B.ngroups = (uint32_t)hp.groups.size();
        B.chunk_tiles = hp.chunk_tiles;
        B.nchunks = hp.nchunks;
        B.ntiles = hp.ntiles;
        B.cnt = reinterpret_cast<uint32_t *>(ws + L.cnt);
        B.chunk_off_out = keep_chunk_off ? reinterpret_cast<uint64_t *>(ws + L.chunk_off) : nullptr;
        B.totals = d_totals;
        B.csr_out = nullptr;  // long patterns first, the CSR below
        B.write = false;
        B.prep = true;
        HIP_OK(launch_batch(B, st));
    }
    for (uint32_t i : hp.longp) {
        const uint64_t m = pat_off[i + 1] - pat_off[i];
        const uint64_t single = L.need - L.single;
        int r = sm_corpus_count_async(c, pats + pat_off[i], m, d_totals + i, ws + L.single, single,
                                      nullptr, st);
        if (r) return r;
    }
    if (d_csr) HIP_OK(launch_csr_scan(d_totals, P, d_csr, st));
    return SM_OK;
}

int run_write(sm_corpus *c, const HostPlan &hp, const Layout &L, uint32_t P, uint8_t *ws,
              const uint64_t *d_csr, int64_t *d_out, uint64_t cap, hipStream_t st)
{
    if (hp.pats.empty() || cap == 0) return SM_OK;
    BatchLaunch B;
    memset(&B, 0, sizeof B);
    B.text = c->d_text;
    B.n = c->n;
    B.pats = reinterpret_cast<const BatchPat *>(ws + L.pats);
    B.groups = reinterpret_cast<const BatchGroup *>(ws + L.groups);
    B.host_groups = hp.groups.data();
    B.params = reinterpret_cast<const Params *>(ws + L.params);
    B.patbytes = ws + L.patbytes;
    B.npats = (uint32_t)hp.pats.size();
    B.npats_total = P;
    B.ngroups = (uint32_t)hp.groups.size();
    B.chunk_tiles = hp.chunk_tiles;
    B.nchunks = hp.nchunks;
    B.ntiles = hp.ntiles;
    B.cnt = reinterpret_cast<uint32_t *>(ws + L.cnt);
    B.chunk_off = reinterpret_cast<const uint64_t *>(ws + L.chunk_off);
    B.csr = d_csr;
    B.out = d_out;
    B.cap = cap;
    B.write = true;
    HIP_OK(launch_batch(B, st));
    return SM_OK;
}

int check_corpus(const sm_corpus *c)
{
    if (!c) return err(SM_EINVAL, "corpus is NULL");
    if (hipSetDevice(c->dev) != hipSuccess) return err(SM_EDEVICE, "cannot select the corpus's device");
    return SM_OK;
}

}  // namespace

extern "C" uint64_t sm_batch_workspace_size(const sm_corpus *c, const uint8_t *pats,
                                            const uint64_t *pat_off, uint32_t P)
{
    if (!c) return 0;
    HostPlan hp;
    if (build_plan(c, pats, pat_off, P, hp)) return 0;
    return layout_of(hp, P, single_ws_need(c, hp, pats, pat_off)).need;
}

extern "C" int sm_batch_count_async(sm_corpus *c, const uint8_t *pats, const uint64_t *pat_off,
                                    uint32_t P, uint64_t *d_counts, void *d_work,
                                    uint64_t work_bytes, void *stream)
{
    int r = check_corpus(c);
    if (r) return r;
    if (P == 0) return SM_OK;
    if (!d_counts) return err(SM_EINVAL, "d_counts is NULL");
    HostPlan hp;
    if ((r = build_plan(c, pats, pat_off, P, hp))) return r;
    const Layout L = layout_of(hp, P, single_ws_need(c, hp, pats, pat_off));
    if (!d_work || work_bytes < L.need) return err(SM_EINVAL, "workspace too small: need %llu bytes", (unsigned long long)L.need);
    if ((uintptr_t)d_work & 255) return err(SM_EINVAL, "workspace must be 256-byte aligned");
    return run_count(c, hp, L, pats, pat_off, P, (uint8_t *)d_work, d_counts, nullptr, false,
                     (hipStream_t)stream);
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
    HostPlan hp;
    if ((r = build_plan(c, pats, pat_off, P, hp))) return r;
    if (!hp.longp.empty())
        return err(SM_EINVAL, "asynchronous batched find_all takes patterns up to %d bytes (use sm_batch_find_all)",
                   BATCH_MAX_M);
    const Layout L = layout_of(hp, P, 0);
    if (!d_work || work_bytes < L.need) return err(SM_EINVAL, "workspace too small: need %llu bytes", (unsigned long long)L.need);
    if ((uintptr_t)d_work & 255) return err(SM_EINVAL, "workspace must be 256-byte aligned");
    uint8_t *ws = (uint8_t *)d_work;
    hipStream_t st = (hipStream_t)stream;
    if ((r = run_count(c, hp, L, pats, pat_off, P, ws, (uint64_t *)(ws + L.totals), d_out_off, true, st)))
        return r;
    return run_write(c, hp, L, P, ws, d_out_off, d_out, cap, st);
}

extern "C" int sm_batch_count(sm_corpus *c, const uint8_t *pats, const uint64_t *pat_off, uint32_t P,
                              uint64_t *counts)
{
    int r = check_corpus(c);
    if (r) return r;
    if (P == 0) return SM_OK;
    if (!counts) return err(SM_EINVAL, "counts is NULL");
    HostPlan hp;
    if ((r = build_plan(c, pats, pat_off, P, hp))) return r;
    const Layout L = layout_of(hp, P, single_ws_need(c, hp, pats, pat_off));
    void *ws = nullptr;
    HIP_OK(hipMalloc(&ws, L.need));
    r = run_count(c, hp, L, pats, pat_off, P, (uint8_t *)ws, (uint64_t *)((uint8_t *)ws + L.totals),
                  nullptr, false, nullptr);
    hipError_t e = hipSuccess;
    if (!r) e = hipMemcpy(counts, (uint8_t *)ws + L.totals, (uint64_t)P * 8, hipMemcpyDeviceToHost);
    (void)hipFree(ws);
    if (r) return r;
    if (e != hipSuccess) return err(SM_EDEVICE, "copy of the counts failed: %s", hipGetErrorString(e));
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
    HostPlan hp;
    if ((r = build_plan(c, pats, pat_off, P, hp))) return r;
    const Layout L = layout_of(hp, P, single_ws_need(c, hp, pats, pat_off));
    uint8_t *ws = nullptr;
    HIP_OK(hipMalloc((void **)&ws, L.need));
    struct Free {
        void *p;
        ~Free() { (void)hipFree(p); }
    } f1{ws};
    uint64_t *d_tot = (uint64_t *)(ws + L.totals), *d_csr = (uint64_t *)(ws + L.csr);
    if ((r = run_count(c, hp, L, pats, pat_off, P, ws, d_tot, d_csr, true, nullptr))) return r;
    HIP_OK(hipMemcpy(out_off, d_csr, ((uint64_t)P + 1) * 8, hipMemcpyDeviceToHost));
    const uint64_t total = out_off[P];
    const uint64_t dcap = std::min(cap, total);
    int64_t *d_out = nullptr;
    if (dcap) HIP_OK(hipMalloc((void **)&d_out, dcap * 8));
    Free f2{d_out};
    if ((r = run_write(c, hp, L, P, ws, d_csr, d_out, dcap, nullptr))) return r;
    // long patterns: one search each, into their CSR slices
    for (uint32_t i : hp.longp) {
        const uint64_t m = pat_off[i + 1] - pat_off[i];
        if (out_off[i] >= dcap) continue;
        const uint64_t room = std::min(out_off[i + 1], dcap) - out_off[i];
        r = sm_corpus_find_all_async(c, pats + pat_off[i], m, d_out + out_off[i], room, d_tot + i,
                                     ws + L.single, L.need - L.single, nullptr, nullptr);
        if (r) return r;
    }
    if (dcap) HIP_OK(hipMemcpy(out, d_out, dcap * 8, hipMemcpyDeviceToHost));
    HIP_OK(hipDeviceSynchronize());
    return total > cap ? SM_TRUNCATED : SM_OK;
}
