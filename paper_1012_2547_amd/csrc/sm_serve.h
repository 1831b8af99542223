// Serving core of the query server (host code only, no HIP): per-corpus queues,
// batch formation, admission by host result memory, and completion in dispatch
// order. The device work of a batch is delegated to an executor X (the HIP
// executor in sm_server.cpp; a mock one in the CPU tests):
//
//   struct X::Slot;                                  per-slot executor state
//   int  X::count(Slot&, void *corpus, const std::vector<SvQuery *>&)
//            enqueue the count step of a batch (must not wait for the device)
//   int  X::wait_count(Slot&, const uint64_t **csr)  wait for it; csr has P + 1
//            entries (query i's positions are entries csr[i] .. csr[i+1])
//   int  X::write(Slot&, uint64_t total, int64_t *host_out)
//            enqueue the writes of CSR entries [0, total) to host_out
//   int  X::wait_done(Slot&)                         wait for the writes
//   void X::drain(Slot&)                             wait for whatever was enqueued
//
// Three threads move a batch along:
//   scheduler: the corpus whose oldest queued query arrived first, up to max_batch
//     of its queries, on any free slot -> X::count; the next batch can be formed
//     while this one counts.
//   admitter (batches in dispatch order): X::wait_count gives the exact output of
//     every query; the longest prefix of the batch whose positions fit the pinned
//     result arena now is admitted and written (X::write), the rest goes back to
//     the front of its queue (deferred, counted again later). When not even the
//     first query fits, completed results that no caller holds yet are moved from
//     the arena to pageable memory (eviction), oldest first; if that is not
//     enough the admitter waits until results are freed or batches complete. A
//     query whose positions alone exceed the arena fails with SM_ENOMEM.
//   completer (dispatch order): X::wait_done, then publishes the results.
//
// The arena (host_bytes) is therefore the only pinned memory results ever take.
// Progress: when the first query of the oldest admitted-but-waiting batch does
// not fit, every completed region is evictable except those holding a result a
// caller has received (wait/poll) and not freed; a caller that frees what it
// received before waiting for the next result never blocks admission for good.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <ctime>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/sm.h"
#include "sm_ring.h"
#include "sm_sched.h"

namespace sm {

inline int64_t sv_now_ns()
{
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (int64_t)ts.tv_sec * 1000000000ll + ts.tv_nsec;
}

struct SvRegion;

struct SvQuery {
    uint64_t ticket = 0;
    uint32_t corpus = 0;
    std::vector<uint8_t> pat;
    int64_t arrival_ns = 0, start_ns = 0, done_ns = 0;
    int status = SM_EBUSY;  // SM_EBUSY until done
    bool done = false;
    bool handed = false;    // wait/poll returned its positions: they may not move
    uint64_t count = 0;
    const int64_t *pos = nullptr;
    uint32_t batch_size = 0;
    std::shared_ptr<SvRegion> region;  // arena memory holding pos (null once moved)
    std::vector<int64_t> moved;        // pos after eviction from the arena
};

// Arena memory of one admitted batch.
struct SvRegion {
    std::shared_ptr<RingRegion> ring;
    int64_t *base = nullptr;      // host address of the batch's CSR entry 0
    uint32_t refs = 0;            // results not yet freed or moved
    bool done = false;            // its positions are on the host
    std::vector<uint64_t> tickets;  // its queries (freed ones are gone from the ticket map)
};

struct SvCounters {
    uint64_t batches = 0, batched_queries = 0, text_bytes = 0, out_bytes = 0;
    uint64_t deferred = 0, evicted = 0, evicted_bytes = 0, rejected = 0, mem_waits = 0;
    uint64_t host_peak = 0;
    std::vector<int64_t> lat_ns;
    int64_t first_arrival = 0, last_done = 0;
};

template <class X>
class ServeCore {
public:
    struct Config {
        uint32_t max_batch = 256, max_pending = 1u << 20;
        uint64_t host_bytes = 0;  // arena size
    };

    // exec and its slots outlive the core; arena_base holds host_bytes.
    ServeCore(X &exec, std::vector<typename X::Slot> &xslots, uint8_t *arena_base, const Config &cfg)
        : exec_(exec), cfg_(cfg), arena_base_(arena_base)
    {
        ring_.cap = cfg.host_bytes;
        slots_.resize(xslots.size());
        for (size_t k = 0; k < xslots.size(); k++) slots_[k].x = &xslots[k];
    }

    void start()
    {
        sched_ = std::thread([this] { scheduler(); });
        admit_ = std::thread([this] { admitter(); });
        compl_ = std::thread([this] { completer(); });
    }

    // Queued queries are dropped; dispatched batches finish (a batch still waiting
    // for arena memory fails with SM_EBUSY). Joins the threads.
    void stop()
    {
        {
            std::lock_guard<std::mutex> g(mu_);
            stop_ = true;
        }
        notify_all();
        if (sched_.joinable()) sched_.join();
        {
            std::lock_guard<std::mutex> g(mu_);
            sched_done_ = true;
        }
        notify_all();
        if (admit_.joinable()) admit_.join();
        {
            std::lock_guard<std::mutex> g(mu_);
            admit_done_ = true;
        }
        notify_all();
        if (compl_.joinable()) compl_.join();
    }

    int add_corpus(void *handle, uint64_t n, uint32_t *id)
    {
        std::lock_guard<std::mutex> g(mu_);
        *id = (uint32_t)corpora_.size();
        corpora_.push_back({handle, n});
        pending_.emplace_back();
        return SM_OK;
    }

    // SM_OK with *ticket, or an error status and a message in *why.
    int submit(uint32_t corpus, const uint8_t *pat, uint64_t m, int64_t arrival_ns, uint64_t *ticket,
               const char **why)
    {
        std::unique_ptr<SvQuery> q(new SvQuery);
        q->pat.assign(pat, pat + m);
        q->arrival_ns = arrival_ns > 0 ? arrival_ns : sv_now_ns();
        {
            std::lock_guard<std::mutex> g(mu_);
            if (stop_) return *why = "server is closing", SM_EBUSY;
            if (fatal_ != SM_OK) return *why = "server stopped after a device failure", fatal_;
            if (corpus >= corpora_.size()) return *why = "no such corpus", SM_EINVAL;
            if (npending_ >= cfg_.max_pending) return *why = "queue full", SM_EBUSY;
            q->ticket = next_ticket_++;
            q->corpus = corpus;
            *ticket = q->ticket;
            pending_[corpus].push_back(q.get());
            npending_++;
            queries_.emplace(q->ticket, std::move(q));
        }
        cv_sched_.notify_one();
        return SM_OK;
    }

    // Fills the result fields through fill(const SvQuery &). SM_EBUSY on timeout
    // (still running), SM_EINVAL for an unknown ticket, else the query's status.
    template <class F>
    int wait(uint64_t ticket, int64_t timeout_us, F fill)
    {
        std::unique_lock<std::mutex> lk(mu_);
        auto it = queries_.find(ticket);
        if (it == queries_.end()) return SM_EINVAL;
        SvQuery *q = it->second.get();
        auto ready = [&] { return q->done; };
        if (timeout_us < 0)
            cv_done_.wait(lk, ready);
        else if (!cv_done_.wait_for(lk, std::chrono::microseconds(timeout_us), ready))
            return SM_EBUSY;
        if (q->status == SM_OK) q->handed = true;
        fill(*q);
        return q->status;
    }

    // SM_OK, SM_EINVAL (unknown ticket) or SM_EBUSY (still running).
    int free_result(uint64_t ticket)
    {
        {
            std::lock_guard<std::mutex> g(mu_);
            auto it = queries_.find(ticket);
            if (it == queries_.end()) return SM_EINVAL;
            if (!it->second->done) return SM_EBUSY;
            release(it->second->region);
            queries_.erase(it);
        }
        cv_mem_.notify_all();
        return SM_OK;
    }

    // Copies the counters and latencies; npending is queued queries.
    void snapshot(SvCounters &c, uint64_t &npending)
    {
        std::lock_guard<std::mutex> g(mu_);
        c = ctr_;
        npending = npending_;
    }

    void reset_stats()
    {
        std::lock_guard<std::mutex> g(mu_);
        ctr_ = SvCounters();
        ctr_.host_peak = ring_.used;
    }

    uint64_t arena_used()
    {
        std::lock_guard<std::mutex> g(mu_);
        return ring_.used;
    }

    // Frees what is left (after stop()).
    void clear()
    {
        std::lock_guard<std::mutex> g(mu_);
        queries_.clear();
        regions_.clear();
    }

private:
    struct Slot {
        typename X::Slot *x = nullptr;
        std::vector<SvQuery *> qs;
        uint32_t corpus = 0;
        void *handle = nullptr;
        const uint64_t *csr = nullptr;
        std::vector<int> qst;  // per-query status
        std::shared_ptr<SvRegion> region;
        int status = SM_OK;
        bool busy = false;
    };

    void notify_all()
    {
        cv_sched_.notify_all();
        cv_count_.notify_all();
        cv_inflight_.notify_all();
        cv_mem_.notify_all();
        cv_done_.notify_all();
    }

    Slot *free_slot()
    {
        for (Slot &s : slots_)
            if (!s.busy) return &s;
        return nullptr;
    }

    void scheduler()
    {
        for (;;) {
            Slot *s = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_sched_.wait(lk, [&] { return stop_ || (npending_ > 0 && free_slot()); });
                if (stop_) return;
                s = free_slot();
                const size_t best = sched_pick(pending_);
                sched_take(pending_[best], cfg_.max_batch, s->qs);
                npending_ -= s->qs.size();
                const int64_t t = sv_now_ns();
                for (SvQuery *q : s->qs) {
                    q->start_ns = t;
                    q->batch_size = (uint32_t)s->qs.size();
                }
                s->corpus = (uint32_t)best;
                s->handle = corpora_[best].handle;
                s->busy = true;
            }
            s->status = exec_.count(*s->x, s->handle, s->qs);
            {
                std::lock_guard<std::mutex> g(mu_);
                counting_.push_back(s);
            }
            cv_count_.notify_one();
        }
    }

    // Largest k <= P whose first k queries' positions fit the arena now.
    uint64_t fit_prefix(const uint64_t *csr, uint64_t P) const
    {
        uint64_t lo = 0, hi = P;  // csr[lo] fits
        while (lo < hi) {
            const uint64_t mid = hi - (hi - lo) / 2;
            if (ring_.fits(csr[mid] * 8)) lo = mid;
            else hi = mid - 1;
        }
        return lo;
    }

    // Moves completed results that no caller holds from the arena to pageable
    // memory, oldest region first, until `bytes` fit. Caller holds mu_.
    bool evict_for(uint64_t bytes)
    {
        bool moved = false;
        while (!ring_.fits(bytes)) {
            while (!regions_.empty() && (!regions_.front()->ring || regions_.front()->ring->freed))
                regions_.pop_front();
            if (regions_.empty()) break;
            SvRegion *r = regions_.front().get();
            if (!r->done) break;  // its batch is still being written: wait for it
            std::vector<SvQuery *> live;
            bool held = false;
            for (uint64_t tk : r->tickets) {
                auto it = queries_.find(tk);
                if (it == queries_.end() || it->second->region.get() != r) continue;
                live.push_back(it->second.get());
                held = held || it->second->handed;
            }
            if (held) break;  // a caller reads it: wait until it is freed
            for (SvQuery *q : live) {
                q->moved.assign(q->pos, q->pos + q->count);
                q->pos = q->moved.empty() ? nullptr : q->moved.data();
                ctr_.evicted++;
                ctr_.evicted_bytes += q->count * 8;
                q->region.reset();
            }
            r->refs = 0;
            ring_.release(r->ring);
            regions_.pop_front();
            moved = true;
        }
        return moved;
    }

    void release(std::shared_ptr<SvRegion> &r)
    {
        if (!r) return;
        if (r->refs > 0 && --r->refs == 0) ring_.release(r->ring);
        r.reset();
    }

    // Admission of one counted batch: the prefix that fits is written, the rest
    // requeued. Runs on the admitter thread.
    int admit_batch(Slot &s)
    {
        const uint64_t *csr = nullptr;
        int r = exec_.wait_count(*s.x, &csr);
        if (r) return r;
        s.csr = csr;
        const uint64_t P = s.qs.size();
        s.qst.assign(P, SM_OK);
        uint64_t total = 0;
        {
            std::unique_lock<std::mutex> lk(mu_);
            uint64_t k = 0;
            for (;;) {
                k = fit_prefix(csr, P);
                if (k > 0) break;
                const uint64_t b0 = csr[1] * 8;
                if (!ring_.ever_fits(b0)) {  // can never fit: refuse this query alone
                    s.qst[0] = SM_ENOMEM;
                    ctr_.rejected++;
                    k = 1;
                    break;
                }
                if (evict_for(b0)) continue;
                if (stop_) {
                    for (uint64_t i = 0; i < P; i++) s.qst[i] = SM_EBUSY;
                    k = P;
                    break;
                }
                ctr_.mem_waits++;
                cv_mem_.wait(lk);
            }
            if (k < P) {  // the rest waits for memory: back to the front of its queue
                auto &dq = pending_[s.corpus];
                for (uint64_t i = P; i-- > k;) dq.push_front(s.qs[i]);
                npending_ += P - k;
                ctr_.deferred += P - k;
                s.qs.resize(k);
                s.qst.resize(k);
            }
            const bool wrote = s.qst[0] == SM_OK;
            total = wrote ? csr[k] : 0;
            s.region.reset();
            if (total) {
                auto rr = ring_.alloc(total * 8);  // fits: checked under this lock
                if (!rr) return SM_ENOMEM;
                s.region = std::make_shared<SvRegion>();
                s.region->ring = rr;
                s.region->base = (int64_t *)(arena_base_ + rr->off);
                s.region->refs = (uint32_t)k;
                s.region->tickets.reserve(k);
                for (SvQuery *q : s.qs) s.region->tickets.push_back(q->ticket);
                while (!regions_.empty() && regions_.front()->ring->freed) regions_.pop_front();
                regions_.push_back(s.region);
                ctr_.host_peak = std::max(ctr_.host_peak, ring_.used);
            }
            ctr_.batches++;
            ctr_.batched_queries += k;
            ctr_.text_bytes += corpora_[s.corpus].n * k;
            ctr_.out_bytes += total * 8;
        }
        if (P > s.qs.size()) cv_sched_.notify_one();
        if (total) return exec_.write(*s.x, total, s.region->base);
        return SM_OK;
    }

    void admitter()
    {
        for (;;) {
            Slot *s = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_count_.wait(lk, [&] { return !counting_.empty() || sched_done_; });
                if (counting_.empty()) return;  // scheduler stopped and every batch admitted
                s = counting_.front();
            }
            if (s->status == SM_OK) s->status = admit_batch(*s);
            {
                std::lock_guard<std::mutex> g(mu_);
                counting_.pop_front();
                inflight_.push_back(s);
            }
            cv_inflight_.notify_one();
        }
    }

    void completer()
    {
        for (;;) {
            Slot *s = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_inflight_.wait(lk, [&] { return !inflight_.empty() || admit_done_; });
                if (inflight_.empty()) return;
                s = inflight_.front();
            }
            int st = s->status;
            if (st == SM_OK) st = exec_.wait_done(*s->x);
            else exec_.drain(*s->x);
            const int64_t t = sv_now_ns();
            {
                std::lock_guard<std::mutex> g(mu_);
                inflight_.pop_front();
                for (size_t i = 0; i < s->qs.size(); i++) {
                    SvQuery *q = s->qs[i];
                    q->done_ns = t;
                    q->status = st != SM_OK ? st : (i < s->qst.size() ? s->qst[i] : SM_OK);
                    q->region = s->region;  // dropped by free_result (refs counts every query)
                    if (q->status == SM_OK) {
                        q->count = s->csr[i + 1] - s->csr[i];
                        q->pos = s->region ? s->region->base + s->csr[i] : nullptr;
                        ctr_.lat_ns.push_back(t - q->arrival_ns);
                        if (ctr_.first_arrival == 0 || q->arrival_ns < ctr_.first_arrival)
                            ctr_.first_arrival = q->arrival_ns;
                        ctr_.last_done = t;
                    }
                    q->done = true;
                }
                if (s->region) s->region->done = true;
                if (st != SM_OK) fatal_ = st;
                s->qs.clear();
                s->qst.clear();
                s->region.reset();
                s->busy = false;
            }
            cv_done_.notify_all();
            cv_sched_.notify_all();
            cv_mem_.notify_all();
        }
    }

    struct CorpusRef {
        void *handle;
        uint64_t n;
    };

    X &exec_;
    Config cfg_;
    uint8_t *arena_base_;
    Ring ring_;
    std::deque<std::shared_ptr<SvRegion>> regions_;  // allocation order
    std::vector<CorpusRef> corpora_;
    std::vector<std::deque<SvQuery *>> pending_;
    std::unordered_map<uint64_t, std::unique_ptr<SvQuery>> queries_;
    uint64_t next_ticket_ = 1, npending_ = 0;
    std::vector<Slot> slots_;
    std::deque<Slot *> counting_, inflight_;
    std::mutex mu_;
    std::condition_variable cv_sched_, cv_count_, cv_inflight_, cv_mem_, cv_done_;
    bool stop_ = false, sched_done_ = false, admit_done_ = false;
    int fatal_ = SM_OK;
    SvCounters ctr_;
    std::thread sched_, admit_, compl_;
};

}  // namespace sm
