// Serving layer: continuous batching of single-pattern queries over resident
// corpora.
//
// The paper times one pattern against a text already in memory (Section 2); a
// server sees a stream of such queries against a few large resident texts. The
// queues, batch formation, admission by host result memory and completion live
// in the device-independent core (sm_serve.h); this file is its HIP executor and
// the C ABI. Per pipeline slot the executor holds a HIP stream, a batch
// workspace, pinned staging and a share of the device output pool:
//
//   count step (batched count pass -> CSR offsets to the host), captured as a HIP
//   graph -> [the core admits the prefix of the batch whose positions fit the
//   pinned result arena] -> write waves of at most the slot's pool share, each a
//   windowed write + device-to-host copy into the arena, captured as graphs.
//
// The count step of one batch runs while the previous batch on another slot
// writes and copies. Graph executables are per slot and updated in place while
// the launch sequence keeps its shape (the steady state under load).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <memory>
#include <new>
#include <vector>

#include "../../include/sm.h"
#include "sm_batch_host.h"
#include "sm_serve.h"
#include "sm_trace.h"

using namespace sm;

#define err sm::batch_err

namespace {

int hip_fail(hipError_t e, const char *what)
{
    return err(e == hipErrorOutOfMemory ? SM_ENOMEM : SM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_OK(expr)                                  \
    do {                                              \
        hipError_t e_ = (expr);                       \
        if (e_ != hipSuccess) return hip_fail(e_, #expr); \
    } while (0)

int grow_dev(uint8_t **p, uint64_t *cap, uint64_t need)
{
    if (need <= *cap) return SM_OK;
    const uint64_t sz = std::max<uint64_t>(need, *cap * 2);
    if (*p) HIP_OK(hipFree(*p));
    *p = nullptr;
    *cap = 0;
    HIP_OK(hipMalloc((void **)p, sz));
    *cap = sz;
    return SM_OK;
}

template <class T>
int grow_host(T **p, uint64_t *cap, uint64_t need_bytes)
{
    if (need_bytes <= *cap) return SM_OK;
    if (*p) HIP_OK(hipHostFree(*p));
    *p = nullptr;
    const uint64_t sz = std::max<uint64_t>(need_bytes, 2 * *cap);
    *cap = 0;
    HIP_OK(hipHostMalloc((void **)p, sz, hipHostMallocDefault));
    *cap = sz;
    return SM_OK;
}

// The HIP executor of the serving core: batched count and windowed writes of one
// batch per slot, on the slot's stream.
struct HipExec {
    struct Slot {
        hipStream_t st = nullptr;
        hipEvent_t ev_count = nullptr, ev_done = nullptr;
        uint8_t *ws = nullptr;
        uint64_t ws_cap = 0;
        int64_t *pool = nullptr;  // this slot's share of the device output pool
        uint64_t pool_pos = 0;    // positions it holds
        uint8_t *h_image = nullptr;
        uint64_t h_image_cap = 0;
        uint64_t *h_csr = nullptr;
        uint64_t h_csr_cap = 0;
        uint32_t *h_stash_n = nullptr;  // hits kept per (chunk, filter group) item
        uint64_t h_stash_n_cap = 0;
        std::vector<uint8_t> pats;
        std::vector<uint64_t> pat_off;
        BatchJob job;
        std::unique_ptr<PlanStaging> stg{new PlanStaging};
        bool graphs = false, wrote = false;
        // graph executables of the count step and of a write wave
        hipGraphExec_t count_exec = nullptr, write_exec = nullptr;
    };

    int dev = 0;
    bool graphs_off = false;
    std::atomic<uint64_t> waves{0}, graph_launches{0}, graph_builds{0};

    // Enqueues work(): captured as a graph and launched through `exec` (updated in
    // place when the captured sequence has the same shape as the one it was built
    // from, else rebuilt) when use is set, else directly. A capture that fails is
    // abandoned and the work is enqueued directly (nothing of it ran).
    template <class F>
    int enqueue(hipStream_t st, hipGraphExec_t &exec, bool use, F work)
    {
        if (!use) return work();
        hipGraph_t graph = nullptr;
        if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            (void)hipGetLastError();
            return work();
        }
        const int r = work();
        hipError_t e = hipStreamEndCapture(st, &graph);
        if (r != SM_OK || e != hipSuccess || !graph) {
            if (graph) (void)hipGraphDestroy(graph);
            (void)hipGetLastError();
            return work();
        }
        bool updated = false;
        if (exec) {
            hipGraphNode_t bad = nullptr;
            hipGraphExecUpdateResult res;
            if (hipGraphExecUpdate(exec, graph, &bad, &res) == hipSuccess && res == hipGraphExecUpdateSuccess) {
                updated = true;
            } else {
                (void)hipGetLastError();
                (void)hipGraphExecDestroy(exec);
                exec = nullptr;
            }
        }
        if (!exec) {
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                exec = nullptr;
                (void)hipGraphDestroy(graph);
                return hip_fail(e, "graph instantiation");
            }
        }
        (void)hipGraphDestroy(graph);
        HIP_OK(hipGraphLaunch(exec, st));
        graph_launches++;
        if (!updated) graph_builds++;
        return SM_OK;
    }

    int count(Slot &s, void *corpus, const std::vector<SvQuery *> &qs)
    {
        TraceRange tr("serve.count.enqueue");
        HIP_OK(hipSetDevice(dev));
        sm_corpus *c = static_cast<sm_corpus *>(corpus);
        const uint32_t P = (uint32_t)qs.size();
        s.wrote = false;
        s.pats.clear();
        s.pat_off.assign(1, 0);
        for (const SvQuery *q : qs) {
            s.pats.insert(s.pats.end(), q->pat.begin(), q->pat.end());
            s.pat_off.push_back(s.pats.size());
        }
        s.pats.resize(s.pats.size() + 16);
        s.job = BatchJob();
        int r = batch_plan(c, s.pats.data(), s.pat_off.data(), P, WS_WRITE, s.job);
        if (r) return r;
        BatchJob &j = s.job;
        if ((r = grow_dev(&s.ws, &s.ws_cap, j.L.need))) return r;
        if ((r = grow_host(&s.h_image, &s.h_image_cap, std::max<uint64_t>(batch_image_bytes(j), 256)))) return r;
        if ((r = grow_host(&s.h_csr, &s.h_csr_cap, ((uint64_t)P + 1) * 8))) return r;
        const uint64_t items = batch_stash_items(j);
        if ((r = grow_host(&s.h_stash_n, &s.h_stash_n_cap, std::max<uint64_t>(items * 4, 256)))) return r;
        batch_fill_image(j, s.h_image);
        uint64_t *d_tot = (uint64_t *)(s.ws + j.L.totals), *d_csr = (uint64_t *)(s.ws + j.L.csr);
        // graphs for batches of patterns within the batch kernels' reach (longer ones
        // take the single-pattern path, whose preparation may copy from pageable memory)
        s.graphs = !graphs_off && j.longp.empty();
        r = enqueue(s.st, s.count_exec, s.graphs, [&]() -> int {
            int rr = batch_count_enqueue(j, s.ws, s.h_image, d_tot, d_csr, true, s.st);
            if (rr) return rr;
            HIP_OK(hipMemcpyAsync(s.h_csr, d_csr, ((uint64_t)P + 1) * 8, hipMemcpyDeviceToHost, s.st));
            if (items)
                HIP_OK(hipMemcpyAsync(s.h_stash_n, s.ws + j.L.mqstash_n, items * 4, hipMemcpyDeviceToHost, s.st));
            return SM_OK;
        });
        if (r) return r;
        HIP_OK(hipEventRecord(s.ev_count, s.st));
        return SM_OK;
    }

    int wait_count(Slot &s, const uint64_t **csr)
    {
        TraceRange tr("serve.count.wait");
        HIP_OK(hipSetDevice(dev));
        HIP_OK(hipEventSynchronize(s.ev_count));
        *csr = s.h_csr;
        return SM_OK;
    }

    // CSR entries [0, total) in waves of at most the slot's pool share.
    int write(Slot &s, uint64_t total, int64_t *host_out)
    {
        TraceRange tr("serve.write.enqueue");
        HIP_OK(hipSetDevice(dev));
        BatchJob &j = s.job;
        j.h_stash_n = batch_stash_items(j) ? s.h_stash_n : nullptr;
        uint64_t *d_tot = (uint64_t *)(s.ws + j.L.totals), *d_csr = (uint64_t *)(s.ws + j.L.csr);
        uint64_t nw = 0;
        int r = SM_OK;
        for (uint64_t lo = 0; lo < total; lo += s.pool_pos, nw++) {
            const uint64_t hi = std::min(total, lo + s.pool_pos);
            if ((r = batch_write_plan(j, s.ws, s.h_csr, lo, hi, s.st, *s.stg))) return r;
            // a wave with single-pattern searches launches directly, as long patterns do
            r = enqueue(s.st, s.write_exec, s.graphs && j.singlep.empty(), [&]() -> int {
                int rr = batch_write_enqueue(j, s.ws, d_csr, s.h_csr, d_tot, s.pool, lo, hi, s.st);
                if (rr) return rr;
                HIP_OK(hipMemcpyAsync(host_out + lo, s.pool, (hi - lo) * 8, hipMemcpyDeviceToHost, s.st));
                return SM_OK;
            });
            if (r) return r;
        }
        HIP_OK(hipEventRecord(s.ev_done, s.st));
        s.wrote = true;
        waves += nw;
        return SM_OK;
    }

    int wait_done(Slot &s)
    {
        if (!s.wrote) return SM_OK;  // nothing written (no positions admitted)
        TraceRange tr("serve.write.wait (writes + copies to host)");
        HIP_OK(hipSetDevice(dev));
        HIP_OK(hipEventSynchronize(s.ev_done));
        return SM_OK;
    }

    void drain(Slot &s)
    {
        (void)hipSetDevice(dev);
        (void)hipStreamSynchronize(s.st);  // whatever was enqueued before the failure
    }
};

void destroy_slots(std::vector<HipExec::Slot> &slots)
{
    for (HipExec::Slot &s : slots) {
        if (s.st) (void)hipStreamSynchronize(s.st);
        if (s.ws) (void)hipFree(s.ws);
        if (s.pool) (void)hipFree(s.pool);
        if (s.h_image) (void)hipHostFree(s.h_image);
        if (s.h_csr) (void)hipHostFree(s.h_csr);
        if (s.h_stash_n) (void)hipHostFree(s.h_stash_n);
        if (s.ev_count) (void)hipEventDestroy(s.ev_count);
        if (s.ev_done) (void)hipEventDestroy(s.ev_done);
        if (s.count_exec) (void)hipGraphExecDestroy(s.count_exec);
        if (s.write_exec) (void)hipGraphExecDestroy(s.write_exec);
        if (s.st) (void)hipStreamDestroy(s.st);
        s = HipExec::Slot();
    }
}

}  // namespace

struct sm_server {
    sm_server_config cfg{};
    HipExec exec;
    std::vector<HipExec::Slot> slots;
    uint8_t *arena = nullptr;
    std::unique_ptr<ServeCore<HipExec>> core;
};

extern "C" int64_t sm_now_ns(void) { return sv_now_ns(); }

extern "C" int sm_server_create(const sm_server_config *cfg, sm_server **out)
{
    if (!out) return err(SM_EINVAL, "server is NULL");
    *out = nullptr;
    sm_server_config c{};
    if (cfg) c = *cfg;
    if (c.pool_bytes == 0) c.pool_bytes = 16ull << 30;
    if (c.host_bytes == 0) c.host_bytes = 2ull << 30;
    if (c.max_batch == 0) c.max_batch = 256;
    if (c.slots == 0) c.slots = 2;
    if (c.max_pending == 0) c.max_pending = 1u << 20;
    if (c.slots > 8) return err(SM_EINVAL, "at most 8 pipeline slots");
    if (c.max_batch > (1u << 20)) return err(SM_EINVAL, "max_batch above 2^20");
    if (c.pool_bytes / c.slots < 8 * 1024) return err(SM_EINVAL, "output pool below 8 KiB per slot");
    if (c.host_bytes < 4096) return err(SM_EINVAL, "host result arena below 4 KiB");
    std::unique_ptr<sm_server> S(new (std::nothrow) sm_server);
    if (!S) return err(SM_ENOMEM, "out of host memory");
    S->cfg = c;
    if (hipGetDevice(&S->exec.dev) != hipSuccess) return err(SM_EDEVICE, "no HIP device");
    S->exec.graphs_off = c.graphs_off != 0;
    S->slots.resize(c.slots);
    int r = SM_OK;
    for (HipExec::Slot &s : S->slots) {
        hipError_t e;
        if ((e = hipStreamCreateWithFlags(&s.st, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&s.ev_count, hipEventDisableTiming)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&s.ev_done, hipEventDisableTiming)) != hipSuccess) {
            r = hip_fail(e, "stream/event creation");
            break;
        }
        s.pool_pos = c.pool_bytes / c.slots / 8;
        if ((e = hipMalloc((void **)&s.pool, s.pool_pos * 8)) != hipSuccess) {
            r = hip_fail(e, "output pool allocation");
            break;
        }
    }
    if (r == SM_OK) {
        hipError_t e = hipHostMalloc((void **)&S->arena, c.host_bytes, hipHostMallocDefault);
        if (e != hipSuccess) r = hip_fail(e, "pinned result arena allocation");
    }
    if (r != SM_OK) {
        destroy_slots(S->slots);
        if (S->arena) (void)hipHostFree(S->arena);
        return r;
    }
    ServeCore<HipExec>::Config cc;
    cc.max_batch = c.max_batch;
    cc.max_pending = c.max_pending;
    cc.host_bytes = c.host_bytes;
    S->core.reset(new ServeCore<HipExec>(S->exec, S->slots, S->arena, cc));
    S->core->start();
    *out = S.release();
    return SM_OK;
}

extern "C" int sm_server_add_corpus(sm_server *S, sm_corpus *c, uint32_t *id)
{
    if (!S || !c || !id) return err(SM_EINVAL, "server, corpus or id is NULL");
    if (c->dev != S->exec.dev) return err(SM_EINVAL, "corpus is on device %d, server on %d", c->dev, S->exec.dev);
    return S->core->add_corpus(c, c->n, id);
}

extern "C" int sm_server_submit(sm_server *S, uint32_t corpus, const uint8_t *pat, uint64_t m,
                                int64_t arrival_ns, uint64_t *ticket)
{
    if (!S || !ticket) return err(SM_EINVAL, "server or ticket is NULL");
    if (m == 0) return err(SM_EINVAL, "empty pattern (m = 0)");
    if (!pat) return err(SM_EINVAL, "pattern is NULL");
    if (m > 0xFFFFFFFFull) return err(SM_EINVAL, "m must be < 2^32");
    const char *why = "";
    int r;
    try {
        r = S->core->submit(corpus, pat, m, arrival_ns, ticket, &why);
    } catch (const std::bad_alloc &) {
        return err(SM_ENOMEM, "out of host memory");
    }
    if (r != SM_OK) return err(r, "%s (corpus %u)", why, corpus);
    return SM_OK;
}

extern "C" int sm_server_wait(sm_server *S, uint64_t ticket, int64_t timeout_us, sm_result *res)
{
    if (!S || !res) return err(SM_EINVAL, "server or result is NULL");
    bool filled = false;
    const int st = S->core->wait(ticket, timeout_us, [&](const SvQuery &q) {
        memset(res, 0, sizeof *res);
        res->status = q.status;
        res->corpus = q.corpus;
        res->count = q.count;
        res->positions = q.pos;
        res->arrival_ns = q.arrival_ns;
        res->start_ns = q.start_ns;
        res->done_ns = q.done_ns;
        res->batch_size = q.batch_size;
        filled = true;
    });
    if (!filled) {
        if (st == SM_EINVAL) return err(SM_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
        return SM_EBUSY;  // not an error: still running
    }
    if (st == SM_ENOMEM)
        return err(SM_ENOMEM, "query %llu: its positions alone exceed the host result arena (%llu bytes)",
                   (unsigned long long)ticket, (unsigned long long)S->cfg.host_bytes);
    if (st == SM_EBUSY) return err(SM_EBUSY, "query %llu: the server closed before it was admitted",
                                   (unsigned long long)ticket);
    if (st != SM_OK) return err(st, "query %llu failed on the device", (unsigned long long)ticket);
    return SM_OK;
}

extern "C" int sm_server_poll(sm_server *S, uint64_t ticket, sm_result *res)
{
    return sm_server_wait(S, ticket, 0, res);
}

extern "C" int sm_result_free(sm_server *S, uint64_t ticket)
{
    if (!S) return err(SM_EINVAL, "server is NULL");
    const int r = S->core->free_result(ticket);
    if (r == SM_EINVAL) return err(SM_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    if (r == SM_EBUSY) return err(SM_EBUSY, "query %llu is still running", (unsigned long long)ticket);
    return SM_OK;
}

extern "C" int sm_server_stats(sm_server *S, sm_server_metrics *st)
{
    if (!S || !st) return err(SM_EINVAL, "server or stats is NULL");
    SvCounters c;
    uint64_t npending = 0;
    S->core->snapshot(c, npending);
    memset(st, 0, sizeof *st);
    st->batches = c.batches;
    st->batched_queries = c.batched_queries;
    st->pending = npending;
    st->text_bytes = c.text_bytes;
    st->out_bytes = c.out_bytes;
    st->write_waves = S->exec.waves.load();
    st->deferred = c.deferred;
    st->graph_launches = S->exec.graph_launches.load();
    st->graph_builds = S->exec.graph_builds.load();
    st->evicted = c.evicted;
    st->evicted_bytes = c.evicted_bytes;
    st->rejected = c.rejected;
    st->mem_waits = c.mem_waits;
    st->host_peak_bytes = c.host_peak;
    st->host_arena_bytes = S->cfg.host_bytes;
    st->span_ns = c.last_done > c.first_arrival ? c.last_done - c.first_arrival : 0;
    std::vector<int64_t> &lat = c.lat_ns;
    st->completed = lat.size();
    if (!lat.empty()) {
        std::sort(lat.begin(), lat.end());
        auto pct = [&](double p) {
            size_t k = (size_t)std::ceil(p * lat.size()) - 1;
            return lat[std::min(k, lat.size() - 1)];
        };
        st->p50_ns = pct(0.50);
        st->p99_ns = pct(0.99);
        st->p999_ns = pct(0.999);
        st->max_ns = lat.back();
        double s = 0;
        for (int64_t v : lat) s += (double)v;
        st->mean_ns = s / lat.size();
        if (st->span_ns) st->qps = lat.size() * 1e9 / st->span_ns;
    }
    return SM_OK;
}

extern "C" int sm_server_reset_stats(sm_server *S)
{
    if (!S) return err(SM_EINVAL, "server is NULL");
    S->core->reset_stats();
    S->exec.waves = 0;
    S->exec.graph_launches = 0;
    S->exec.graph_builds = 0;
    return SM_OK;
}

extern "C" int sm_server_destroy(sm_server *S)
{
    if (!S) return SM_OK;
    S->core->stop();  // queued queries are dropped; dispatched batches finish
    S->core->clear();
    destroy_slots(S->slots);
    if (S->arena) (void)hipHostFree(S->arena);
    delete S;
    return SM_OK;
}
