// Serving layer: continuous batching of single-pattern queries over resident
// corpora.
//
// The paper times one pattern against a text already in memory (Section 2); a
// server sees a stream of such queries against a few large resident texts. The
// scheduler thread groups the queued queries of one corpus into a batch (the
// corpus whose oldest query arrived first goes next) and runs it through the
// batched search on one of several pipeline slots, each with its own HIP stream,
// workspace and share of the device output pool:
//
//   count step -> CSR offsets to the host (the exact output size of every query)
//   -> admission: host result space (pinned arena; a dedicated pinned buffer
//      when the arena cannot hold it) and write waves of at most the slot's
//      pool share -> windowed writes + device-to-host copies -> done event.
//
// While the scheduler waits for batch j+1's counts on one slot, batch j's writes
// and copies run on another, so the count pass of one batch overlaps the output
// traffic of the previous one. The count step and each write wave are captured
// as HIP graphs and replayed through per-slot executables that are updated in
// place while the launch sequence keeps its shape (steady state under load). A completion thread waits for each slot's done
// event in dispatch order and publishes the results. Queries past the queue
// limit are refused at submission (SM_EBUSY).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <ctime>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/sm.h"
#include "sm_batch_host.h"
#include "sm_ring.h"
#include "sm_sched.h"

using namespace sm;

#define err sm::batch_err

namespace {

int64_t now_ns()
{
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (int64_t)ts.tv_sec * 1000000000ll + ts.tv_nsec;
}

// Host result memory of one batch: a region of the pinned arena or a dedicated
// pinned buffer; released when the last of its queries' results is freed.
struct Region {
    std::shared_ptr<RingRegion> ring;
    int64_t *dedicated = nullptr;
    uint32_t refs = 0;
};

struct Arena {
    uint8_t *base = nullptr;
    Ring ring;
};

struct Query {
    uint64_t ticket = 0;
    uint32_t corpus = 0;
    std::vector<uint8_t> pat;
    int64_t arrival_ns = 0, start_ns = 0, done_ns = 0;
    int status = SM_EBUSY;  // SM_EBUSY until done
    bool done = false;
    uint64_t count = 0;
    const int64_t *pos = nullptr;
    uint32_t batch_size = 0;
    std::shared_ptr<Region> region;
};

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
    // the batch in flight
    std::vector<Query *> qs;
    std::vector<uint8_t> pats;
    std::vector<uint64_t> pat_off;
    BatchJob job;
    std::unique_ptr<PlanStaging> stg{new PlanStaging};
    std::shared_ptr<Region> region;
    int64_t *host_out = nullptr;
    int status = SM_OK;
    bool busy = false;
    // graph executables of the count step and of a write wave, updated in place
    // while the captured launch sequence keeps its shape
    hipGraphExec_t count_exec = nullptr, write_exec = nullptr;
};

}  // namespace

struct sm_server {
    int dev = 0;
    sm_server_config cfg{};
    std::vector<sm_corpus *> corpora;
    std::vector<std::deque<Query *>> pending;  // per corpus
    std::unordered_map<uint64_t, std::unique_ptr<Query>> queries;
    uint64_t next_ticket = 1;
    uint64_t npending = 0;
    std::vector<Slot> slots;
    std::deque<Slot *> inflight;  // dispatch order, for the completion thread
    Arena arena;
    std::mutex mu;
    std::condition_variable cv_work, cv_slot, cv_done, cv_inflight;
    bool stop = false;
    std::thread sched, compl_thr;
    // statistics since the last reset
    std::vector<int64_t> lat_ns;
    uint64_t batches = 0, batched_queries = 0, text_bytes = 0, out_bytes = 0, overflow_allocs = 0;
    uint64_t waves = 0, graph_launches = 0, graph_builds = 0;
    int64_t first_arrival = 0, last_done = 0;
    std::atomic<int> fatal{SM_OK};
};

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

// Enqueues work(): captured as a graph and launched through `exec` (updated in
// place when the captured sequence has the same shape as the one it was built
// from, else rebuilt) when use is set, else directly. A capture that fails is
// abandoned and the work is enqueued directly (nothing of it ran).
template <class F>
int enqueue_graph(sm_server *S, hipStream_t st, hipGraphExec_t &exec, bool use, F work)
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
    std::lock_guard<std::mutex> g(S->mu);
    S->graph_launches++;
    if (!updated) S->graph_builds++;
    return SM_OK;
}

// Count, admission, windowed writes and copies of one batch on slot s. Runs on
// the scheduler thread with the server lock released; returns after the writes
// are enqueued (the completion thread waits for them).
int run_batch(sm_server *S, Slot &s, sm_corpus *c)
{
    const uint32_t P = (uint32_t)s.qs.size();
    s.pats.clear();
    s.pat_off.assign(1, 0);
    for (Query *q : s.qs) {
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
    batch_fill_image(j, s.h_image);
    uint64_t *d_tot = (uint64_t *)(s.ws + j.L.totals), *d_csr = (uint64_t *)(s.ws + j.L.csr);
    // graphs for batches of patterns within the batch kernels' reach (longer ones
    // take the single-pattern path, whose preparation may copy from pageable memory)
    const bool graphs = !S->cfg.graphs_off && j.longp.empty();
    r = enqueue_graph(S, s.st, s.count_exec, graphs, [&]() -> int {
        int rr = batch_count_enqueue(j, s.ws, s.h_image, d_tot, d_csr, true, s.st);
        if (rr) return rr;
        HIP_OK(hipMemcpyAsync(s.h_csr, d_csr, ((uint64_t)P + 1) * 8, hipMemcpyDeviceToHost, s.st));
        return SM_OK;
    });
    if (r) return r;
    HIP_OK(hipEventRecord(s.ev_count, s.st));
    HIP_OK(hipEventSynchronize(s.ev_count));
    const uint64_t total = s.h_csr[P];
    // admission: host space for exactly `total` positions
    s.region.reset();
    s.host_out = nullptr;
    if (total) {
        {
            std::lock_guard<std::mutex> g(S->mu);
            auto rr = S->arena.ring.alloc(total * 8);
            if (rr) {
                s.region = std::make_shared<Region>();
                s.region->ring = rr;
                s.host_out = (int64_t *)(S->arena.base + rr->off);
            }
        }
        if (!s.region) {
            int64_t *d = nullptr;
            HIP_OK(hipHostMalloc((void **)&d, total * 8, hipHostMallocDefault));
            s.region = std::make_shared<Region>();
            s.region->dedicated = d;
            s.host_out = d;
            std::lock_guard<std::mutex> g(S->mu);
            S->overflow_allocs++;
        }
        s.region->refs = P;
    }
    // output waves of at most the slot's pool share
    uint64_t nw = 0;
    for (uint64_t lo = 0; lo < total; lo += s.pool_pos, nw++) {
        const uint64_t hi = std::min(total, lo + s.pool_pos);
        if ((r = batch_write_plan(j, s.ws, s.h_csr, lo, hi, s.st, *s.stg))) return r;
        // a wave with single-pattern searches launches directly, as long patterns do
        r = enqueue_graph(S, s.st, s.write_exec, graphs && j.singlep.empty(), [&]() -> int {
            int rr = batch_write_enqueue(j, s.ws, d_csr, s.h_csr, d_tot, s.pool, lo, hi, s.st);
            if (rr) return rr;
            HIP_OK(hipMemcpyAsync(s.host_out + lo, s.pool, (hi - lo) * 8, hipMemcpyDeviceToHost, s.st));
            return SM_OK;
        });
        if (r) return r;
    }
    HIP_OK(hipEventRecord(s.ev_done, s.st));
    std::lock_guard<std::mutex> g(S->mu);
    S->waves += nw;
    S->out_bytes += total * 8;
    return SM_OK;
}

void scheduler(sm_server *S)
{
    (void)hipSetDevice(S->dev);
    size_t next = 0;
    for (;;) {
        Slot &s = S->slots[next];
        sm_corpus *c = nullptr;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_slot.wait(lk, [&] { return S->stop || !s.busy; });
            S->cv_work.wait(lk, [&] { return S->stop || S->npending > 0; });
            if (S->stop) return;
            // the corpus whose oldest query arrived first, up to max_batch of its queries
            const size_t best = sched_pick(S->pending);
            sched_take(S->pending[best], S->cfg.max_batch, s.qs);
            const int64_t t = now_ns();
            for (Query *q : s.qs) q->start_ns = t;
            S->npending -= s.qs.size();
            for (Query *q : s.qs) q->batch_size = (uint32_t)s.qs.size();
            c = S->corpora[best];
            s.busy = true;
        }
        s.status = run_batch(S, s, c);
        {
            std::lock_guard<std::mutex> g(S->mu);
            S->batches++;
            S->batched_queries += s.qs.size();
            S->text_bytes += c->n * s.qs.size();
            S->inflight.push_back(&s);
        }
        S->cv_inflight.notify_one();
        next = (next + 1) % S->slots.size();
    }
}

void completer(sm_server *S)
{
    (void)hipSetDevice(S->dev);
    for (;;) {
        Slot *s = nullptr;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_inflight.wait(lk, [&] { return !S->inflight.empty() || S->stop; });
            if (S->inflight.empty()) return;  // stopping and drained
            s = S->inflight.front();
        }
        int st = s->status;
        if (st == SM_OK) {
            hipError_t e = hipEventSynchronize(s->ev_done);
            if (e != hipSuccess) st = hip_fail(e, "batch");
        } else {
            (void)hipStreamSynchronize(s->st);  // whatever was enqueued before the failure
        }
        const int64_t t = now_ns();
        {
            std::lock_guard<std::mutex> g(S->mu);
            S->inflight.pop_front();
            for (size_t i = 0; i < s->qs.size(); i++) {
                Query *q = s->qs[i];
                q->done_ns = t;
                q->status = st;
                if (st == SM_OK) {
                    q->count = s->h_csr[i + 1] - s->h_csr[i];
                    q->pos = s->host_out ? s->host_out + s->h_csr[i] : nullptr;
                    q->region = s->region;
                    S->lat_ns.push_back(t - q->arrival_ns);
                    if (S->first_arrival == 0 || q->arrival_ns < S->first_arrival) S->first_arrival = q->arrival_ns;
                    S->last_done = t;
                } else if (s->region) {
                    q->region = s->region;
                }
                q->done = true;
            }
            if (st != SM_OK) S->fatal = st;
            s->qs.clear();
            s->region.reset();
            s->busy = false;
        }
        S->cv_done.notify_all();
        S->cv_slot.notify_all();
    }
}

void release_region(sm_server *S, const std::shared_ptr<Region> &r)
{
    if (!r || --r->refs > 0) return;
    if (r->dedicated) {
        (void)hipHostFree(r->dedicated);
        r->dedicated = nullptr;
    } else {
        S->arena.ring.release(r->ring);
    }
}

void destroy_resources(sm_server *S)
{
    for (Slot &s : S->slots) {
        if (s.st) (void)hipStreamSynchronize(s.st);
        if (s.ws) (void)hipFree(s.ws);
        if (s.pool) (void)hipFree(s.pool);
        if (s.h_image) (void)hipHostFree(s.h_image);
        if (s.h_csr) (void)hipHostFree(s.h_csr);
        if (s.ev_count) (void)hipEventDestroy(s.ev_count);
        if (s.ev_done) (void)hipEventDestroy(s.ev_done);
        if (s.count_exec) (void)hipGraphExecDestroy(s.count_exec);
        if (s.write_exec) (void)hipGraphExecDestroy(s.write_exec);
        if (s.st) (void)hipStreamDestroy(s.st);
    }
    for (auto &kv : S->queries)
        if (kv.second->region && kv.second->region->dedicated) {
            (void)hipHostFree(kv.second->region->dedicated);
            kv.second->region->dedicated = nullptr;
        }
    if (S->arena.base) (void)hipHostFree(S->arena.base);
}

}  // namespace

extern "C" int64_t sm_now_ns(void) { return now_ns(); }

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
    std::unique_ptr<sm_server> S(new (std::nothrow) sm_server);
    if (!S) return err(SM_ENOMEM, "out of host memory");
    S->cfg = c;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return err(SM_EDEVICE, "no HIP device");
    S->dev = dev;
    S->slots.resize(c.slots);
    int r = SM_OK;
    for (Slot &s : S->slots) {
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
        hipError_t e = hipHostMalloc((void **)&S->arena.base, c.host_bytes, hipHostMallocDefault);
        if (e != hipSuccess) r = hip_fail(e, "pinned result arena allocation");
        S->arena.ring.cap = c.host_bytes;
    }
    if (r != SM_OK) {
        destroy_resources(S.get());
        return r;
    }
    sm_server *raw = S.get();
    raw->sched = std::thread(scheduler, raw);
    raw->compl_thr = std::thread(completer, raw);
    *out = S.release();
    return SM_OK;
}

extern "C" int sm_server_add_corpus(sm_server *S, sm_corpus *c, uint32_t *id)
{
    if (!S || !c || !id) return err(SM_EINVAL, "server, corpus or id is NULL");
    if (c->dev != S->dev) return err(SM_EINVAL, "corpus is on device %d, server on %d", c->dev, S->dev);
    std::lock_guard<std::mutex> g(S->mu);
    *id = (uint32_t)S->corpora.size();
    S->corpora.push_back(c);
    S->pending.emplace_back();
    return SM_OK;
}

extern "C" int sm_server_submit(sm_server *S, uint32_t corpus, const uint8_t *pat, uint64_t m,
                                int64_t arrival_ns, uint64_t *ticket)
{
    if (!S || !ticket) return err(SM_EINVAL, "server or ticket is NULL");
    if (m == 0) return err(SM_EINVAL, "empty pattern (m = 0)");
    if (!pat) return err(SM_EINVAL, "pattern is NULL");
    if (m > 0xFFFFFFFFull) return err(SM_EINVAL, "m must be < 2^32");
    auto q = std::unique_ptr<Query>(new (std::nothrow) Query);
    if (!q) return err(SM_ENOMEM, "out of host memory");
    q->pat.assign(pat, pat + m);
    q->arrival_ns = arrival_ns > 0 ? arrival_ns : now_ns();
    {
        std::lock_guard<std::mutex> g(S->mu);
        if (S->stop) return err(SM_EBUSY, "server is closing");
        if (S->fatal != SM_OK) return err(S->fatal, "server stopped after a device failure");
        if (corpus >= S->corpora.size()) return err(SM_EINVAL, "no corpus %u", corpus);
        if (S->npending >= S->cfg.max_pending) return err(SM_EBUSY, "queue full (%u queries)", S->cfg.max_pending);
        q->ticket = S->next_ticket++;
        q->corpus = corpus;
        *ticket = q->ticket;
        S->pending[corpus].push_back(q.get());
        S->npending++;
        S->queries.emplace(q->ticket, std::move(q));
    }
    S->cv_work.notify_one();
    return SM_OK;
}

namespace {
void fill_result(const Query *q, sm_result *res)
{
    memset(res, 0, sizeof *res);
    res->status = q->status;
    res->corpus = q->corpus;
    res->count = q->count;
    res->positions = q->pos;
    res->arrival_ns = q->arrival_ns;
    res->start_ns = q->start_ns;
    res->done_ns = q->done_ns;
    res->batch_size = q->batch_size;
}
}  // namespace

extern "C" int sm_server_wait(sm_server *S, uint64_t ticket, int64_t timeout_us, sm_result *res)
{
    if (!S || !res) return err(SM_EINVAL, "server or result is NULL");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->queries.find(ticket);
    if (it == S->queries.end()) return err(SM_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    Query *q = it->second.get();
    auto ready = [&] { return q->done; };
    if (timeout_us < 0)
        S->cv_done.wait(lk, ready);
    else if (!S->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready))
        return SM_EBUSY;  // not an error: still running
    fill_result(q, res);
    if (q->status != SM_OK) return err(q->status, "query failed on the device");
    return SM_OK;
}

extern "C" int sm_server_poll(sm_server *S, uint64_t ticket, sm_result *res)
{
    return sm_server_wait(S, ticket, 0, res);
}

extern "C" int sm_result_free(sm_server *S, uint64_t ticket)
{
    if (!S) return err(SM_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->queries.find(ticket);
    if (it == S->queries.end()) return err(SM_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    if (!it->second->done) return err(SM_EBUSY, "query %llu is still running", (unsigned long long)ticket);
    release_region(S, it->second->region);
    S->queries.erase(it);
    return SM_OK;
}

extern "C" int sm_server_stats(sm_server *S, sm_server_metrics *st)
{
    if (!S || !st) return err(SM_EINVAL, "server or stats is NULL");
    std::vector<int64_t> lat;
    memset(st, 0, sizeof *st);
    {
        std::lock_guard<std::mutex> g(S->mu);
        lat = S->lat_ns;
        st->batches = S->batches;
        st->batched_queries = S->batched_queries;
        st->pending = S->npending;
        st->text_bytes = S->text_bytes;
        st->out_bytes = S->out_bytes;
        st->write_waves = S->waves;
        st->overflow_allocs = S->overflow_allocs;
        st->graph_launches = S->graph_launches;
        st->graph_builds = S->graph_builds;
        st->span_ns = S->last_done > S->first_arrival ? S->last_done - S->first_arrival : 0;
    }
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
    std::lock_guard<std::mutex> g(S->mu);
    S->lat_ns.clear();
    S->batches = S->batched_queries = S->text_bytes = S->out_bytes = S->overflow_allocs = S->waves = 0;
    S->graph_launches = S->graph_builds = 0;
    S->first_arrival = S->last_done = 0;
    return SM_OK;
}

extern "C" int sm_server_destroy(sm_server *S)
{
    if (!S) return SM_OK;
    {
        std::lock_guard<std::mutex> g(S->mu);
        S->stop = true;  // queued queries are dropped; dispatched batches finish
    }
    S->cv_work.notify_all();
    S->cv_slot.notify_all();
    if (S->sched.joinable()) S->sched.join();
    S->cv_inflight.notify_all();  // the completer drains what was dispatched, then exits
    if (S->compl_thr.joinable()) S->compl_thr.join();
    destroy_resources(S);
    delete S;
    return SM_OK;
}
