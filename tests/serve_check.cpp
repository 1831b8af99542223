// The server's serving core (sm_serve.h) driven by a mock executor on the CPU:
// every query's pattern encodes its id and its number of positions, the mock
// "count step" reads them back, and the mock "writes" fill position j of query
// id with id * 1000003 + j when the batch completes. Producer threads submit
// queries for three corpora; consumer threads wait for them, check every
// position, and free the results.
//
// Checked, for a small result arena (so that most batches are cut, deferred and
// counted again, completed results are evicted to pageable memory, and queries
// larger than the arena are refused):
//   - every query completes exactly once with the right positions, or with
//     SM_ENOMEM exactly when its positions alone exceed the arena;
//   - the arena never holds more than its size (peak counter);
//   - nothing deadlocks: a consumer waiting in ticket order, and consumers that
//     hold a result for a while in random order, both finish (a watchdog fails
//     the run after 120 s);
//   - stop() with queries still queued or waiting for memory returns.
// Built with -fsanitize=thread in the test as well.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <thread>
#include <vector>

#include "sm_serve.h"

using sm::ServeCore;
using sm::SvQuery;

struct MockExec {
    struct Slot {
        std::vector<uint64_t> csr, ids;
        uint64_t total = 0;
        int64_t *out = nullptr;
        bool wrote = false;
        unsigned seed = 1;
    };
    std::atomic<uint64_t> counts{0}, writes{0};

    static void nap(Slot &s, int max_us)
    {
        s.seed = s.seed * 1103515245u + 12345u;
        std::this_thread::sleep_for(std::chrono::microseconds((s.seed >> 8) % (unsigned)max_us));
    }
    int count(Slot &s, void *, const std::vector<SvQuery *> &qs)
    {
        s.csr.assign(qs.size() + 1, 0);
        s.ids.assign(qs.size(), 0);
        for (size_t i = 0; i < qs.size(); i++) {
            uint64_t id, cnt;
            std::memcpy(&id, qs[i]->pat.data(), 8);
            std::memcpy(&cnt, qs[i]->pat.data() + 8, 8);
            s.ids[i] = id;
            s.csr[i + 1] = s.csr[i] + cnt;
        }
        s.wrote = false;
        counts++;
        return SM_OK;
    }
    int wait_count(Slot &s, const uint64_t **csr)
    {
        nap(s, 300);
        *csr = s.csr.data();
        return SM_OK;
    }
    int write(Slot &s, uint64_t total, int64_t *out)
    {
        s.total = total;
        s.out = out;
        s.wrote = true;
        writes++;
        return SM_OK;
    }
    int wait_done(Slot &s)
    {
        if (!s.wrote) return SM_OK;
        nap(s, 400);
        for (size_t i = 0; i + 1 < s.csr.size() && s.csr[i + 1] <= s.total; i++)
            for (uint64_t j = 0; j < s.csr[i + 1] - s.csr[i]; j++)
                s.out[s.csr[i] + j] = (int64_t)(s.ids[i] * 1000003ull + j);
        return SM_OK;
    }
    void drain(Slot &) {}
};

static std::atomic<bool> g_bad{false};
static void fail(const char *what, unsigned long long a = 0, unsigned long long b = 0)
{
    if (!g_bad.exchange(true)) std::printf("FAIL %s (%llu, %llu)\n", what, a, b);
}

// counts: mostly small, some large, a few larger than a 1 MiB arena
static uint64_t draw_count(std::mt19937_64 &rng)
{
    const uint64_t ref = (1u << 20) / 8;  // positions in 1 MiB
    const uint64_t r = rng() % 1000;
    if (r < 5) return ref + 1 + rng() % 1000;
    if (r < 150) return ref / 8 + rng() % (ref / 3);
    if (r < 300) return 0;
    return rng() % 2000;
}

struct Run {
    uint64_t completed = 0, refused = 0, expect_refused = 0;
    sm::SvCounters c;
};

// mode 0: one consumer in ticket order; mode 1: four consumers in random order,
// each holding its result for a while before freeing it.
static Run run(int mode, uint64_t arena_bytes, int nq, uint32_t max_batch, int nslots)
{
    MockExec ex;
    std::vector<MockExec::Slot> xs(nslots);
    for (int k = 0; k < nslots; k++) xs[k].seed = 7 + k;
    std::vector<uint8_t> arena(arena_bytes);
    ServeCore<MockExec>::Config cfg;
    cfg.max_batch = max_batch;
    cfg.host_bytes = arena_bytes;
    ServeCore<MockExec> core(ex, xs, arena.data(), cfg);
    int corpus_tag[3];
    uint32_t ids[3];
    for (int c = 0; c < 3; c++) core.add_corpus(&corpus_tag[c], 1000 + c, &ids[c]);
    core.start();

    std::vector<uint64_t> tickets(nq, 0), counts(nq, 0);
    std::vector<std::atomic<int>> ready(nq);
    for (auto &r : ready) r = 0;
    std::atomic<int> submitted{0};
    const int NP = 3;
    std::vector<std::thread> prod;
    for (int p = 0; p < NP; p++)
        prod.emplace_back([&, p] {
            std::mt19937_64 rng(1000 + p + 17 * mode);
            for (int i = p; i < nq; i += NP) {
                const uint64_t cnt = draw_count(rng);
                counts[i] = cnt;
                uint8_t pat[16];
                const uint64_t id = (uint64_t)i;
                std::memcpy(pat, &id, 8);
                std::memcpy(pat + 8, &cnt, 8);
                uint64_t tk = 0;
                const char *why = "";
                int r;
                while ((r = core.submit(ids[rng() % 3], pat, 16, 0, &tk, &why)) == SM_EBUSY)
                    std::this_thread::yield();
                if (r != SM_OK) fail("submit", (unsigned long long)r);
                tickets[i] = tk;
                ready[i].store(1, std::memory_order_release);
                submitted++;
                if (rng() % 8 == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 200));
            }
        });

    std::atomic<uint64_t> completed{0}, refused{0};
    auto check_one = [&](int i, std::mt19937_64 &rng, int hold_us) {
        while (!ready[i].load(std::memory_order_acquire)) std::this_thread::yield();
        const int64_t *pos = nullptr;
        uint64_t got = 0;
        int st = core.wait(tickets[i], -1, [&](const SvQuery &q) {
            pos = q.pos;
            got = q.count;
        });
        const bool too_big = counts[i] * 8 > arena_bytes;
        if (st == SM_ENOMEM) {
            if (!too_big) fail("refused a query that fits the arena", i, counts[i]);
            refused++;
        } else if (st != SM_OK) {
            fail("query status", i, (unsigned long long)(-st));
        } else {
            if (too_big) fail("admitted a query larger than the arena", i, counts[i]);
            if (got != counts[i]) fail("count", i, got);
            for (uint64_t j = 0; j < got; j++)
                if (pos[j] != (int64_t)((uint64_t)i * 1000003ull + j)) {
                    fail("position", i, j);
                    break;
                }
        }
        if (hold_us) std::this_thread::sleep_for(std::chrono::microseconds(rng() % hold_us));
        if (core.free_result(tickets[i]) != SM_OK) fail("free", i);
        completed++;
    };
    std::vector<std::thread> cons;
    std::vector<int> order(nq);
    if (mode == 0) {
        cons.emplace_back([&] {
            std::mt19937_64 rng(5);
            for (int i = 0; i < nq; i++) check_one(i, rng, 0);
        });
    } else {
        for (int i = 0; i < nq; i++) order[i] = i;
        std::mt19937_64 sh(9);
        std::shuffle(order.begin(), order.end(), sh);
        const int NC = 4;
        for (int c = 0; c < NC; c++)
            cons.emplace_back([&, c] {
                std::mt19937_64 rng(50 + c);
                for (int k = c; k < nq; k += NC) check_one(order[k], rng, 300);
            });
    }
    // watchdog
    std::atomic<bool> finished{false};
    std::thread dog([&] {
        for (int t = 0; t < 1200 && !finished; t++) std::this_thread::sleep_for(std::chrono::milliseconds(100));
        if (!finished) {
            std::printf("FAIL no progress for 120 s (mode %d): %llu of %d completed\n", mode,
                        (unsigned long long)completed.load(), nq);
            std::fflush(stdout);
            std::_Exit(3);
        }
    });
    for (auto &t : prod) t.join();
    for (auto &t : cons) t.join();
    finished = true;
    dog.join();
    Run out;
    uint64_t np = 0;
    core.snapshot(out.c, np);
    core.stop();
    core.clear();
    out.completed = completed;
    out.refused = refused;
    for (int i = 0; i < nq; i++) out.expect_refused += counts[i] * 8 > arena_bytes;
    if (np != 0) fail("queries left queued", np);
    if (out.c.host_peak > arena_bytes) fail("arena peak above its size", out.c.host_peak, arena_bytes);
    if (out.refused != out.expect_refused || out.c.rejected != out.expect_refused)
        fail("refused count", out.refused, out.expect_refused);
    if (out.completed != (uint64_t)nq) fail("completed", out.completed, nq);
    return out;
}

// stop() while queries are queued and a batch waits for memory held by a
// caller: returns, and the waiting queries fail with SM_EBUSY.
static void stop_while_waiting()
{
    MockExec ex;
    std::vector<MockExec::Slot> xs(2);
    const uint64_t arena_bytes = 64 * 1024;
    std::vector<uint8_t> arena(arena_bytes);
    ServeCore<MockExec>::Config cfg;
    cfg.host_bytes = arena_bytes;
    cfg.max_batch = 4;
    ServeCore<MockExec> core(ex, xs, arena.data(), cfg);
    int tag;
    uint32_t id;
    core.add_corpus(&tag, 10, &id);
    core.start();
    auto submit = [&](uint64_t qid, uint64_t cnt) {
        uint8_t pat[16];
        std::memcpy(pat, &qid, 8);
        std::memcpy(pat + 8, &cnt, 8);
        uint64_t tk = 0;
        const char *why = "";
        if (core.submit(id, pat, 16, 0, &tk, &why) != SM_OK) fail("submit (stop test)");
        return tk;
    };
    // the first result takes 3/4 of the arena and is held (received, not freed)
    const uint64_t t0 = submit(0, arena_bytes / 8 * 3 / 4);
    if (core.wait(t0, -1, [](const SvQuery &) {}) != SM_OK) fail("first query");
    std::vector<uint64_t> rest;
    for (int i = 1; i < 20; i++) rest.push_back(submit(i, arena_bytes / 8 / 2));
    std::this_thread::sleep_for(std::chrono::milliseconds(50));
    sm::SvCounters c;
    uint64_t np = 0;
    core.snapshot(c, np);
    if (c.mem_waits == 0) fail("no batch waited for memory");
    core.stop();  // must return
    for (uint64_t tk : rest) {
        const int st = core.wait(tk, 0, [](const SvQuery &) {});
        if (st != SM_EBUSY) fail("a query admitted while the arena was held", tk, (unsigned long long)(-st));
    }
    core.clear();
}

int main()
{
    const Run a = run(0, 1 << 20, 3000, 64, 2);
    std::printf("in order: batches %llu, deferred %llu, evicted %llu, refused %llu, mem waits %llu, peak %llu of %d\n",
                (unsigned long long)a.c.batches, (unsigned long long)a.c.deferred,
                (unsigned long long)a.c.evicted, (unsigned long long)a.refused,
                (unsigned long long)a.c.mem_waits, (unsigned long long)a.c.host_peak, 1 << 20);
    if (a.c.deferred == 0) fail("no query was deferred: the arena did not bind");
    if (a.c.evicted == 0) fail("no result was evicted");
    const Run b = run(1, 1 << 20, 3000, 32, 3);
    std::printf("random order: batches %llu, deferred %llu, evicted %llu, refused %llu, mem waits %llu, peak %llu\n",
                (unsigned long long)b.c.batches, (unsigned long long)b.c.deferred,
                (unsigned long long)b.c.evicted, (unsigned long long)b.refused,
                (unsigned long long)b.c.mem_waits, (unsigned long long)b.c.host_peak);
    // an arena that holds every result at once never binds
    const Run c = run(0, 256 << 20, 1000, 256, 2);
    if (c.c.deferred || c.c.evicted || c.c.mem_waits || c.refused) fail("memory pressure with a large arena");
    stop_while_waiting();
    if (g_bad) return 1;
    std::printf("ok\n");
    return 0;
}
