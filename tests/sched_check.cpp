// The server's batch formation (sm_sched.h) driven by a mock executor on the CPU:
// producer threads queue queries for random corpora under one lock, as
// sm_server_submit does; a scheduler thread forms batches with sched_pick /
// sched_take, as the server's scheduler does, and a mock executor "runs" them.
// Checked: every query runs exactly once, a batch holds one corpus's queries in
// arrival order and at most max_batch of them, and the chosen corpus held the
// oldest queued query. Built with -fsanitize=thread in the test as well.
#include <condition_variable>
#include <cstdio>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "sm_sched.h"

struct Q {
    int64_t arrival_ns;
    uint64_t ticket;
    uint32_t corpus;
};

int main()
{
    const int NC = 3, NP = 4, PER = 3000;
    const size_t MAXB = 37;
    std::vector<std::deque<Q *>> pending(NC);
    std::vector<Q> all((size_t)NP * PER);
    std::mutex mu;
    std::condition_variable cv;
    uint64_t next_ticket = 1;
    int64_t clock = 0;
    int producers_left = NP;  // guarded by mu
    std::vector<int> ran(all.size() + 1, 0);
    bool bad = false;
    auto fail = [&](const char *why) {
        if (!bad) std::printf("FAIL %s\n", why);
        bad = true;
    };
    std::vector<std::thread> prod;
    for (int p = 0; p < NP; p++)
        prod.emplace_back([&, p] {
            std::mt19937 rng(100 + p);
            for (int i = 0; i < PER; i++) {
                Q *q = &all[(size_t)p * PER + i];
                {
                    std::lock_guard<std::mutex> g(mu);
                    q->ticket = next_ticket++;
                    q->arrival_ns = ++clock;  // arrival order = submission order
                    q->corpus = rng() % NC;
                    pending[q->corpus].push_back(q);
                }
                cv.notify_one();
                if (rng() % 64 == 0) std::this_thread::yield();
            }
            {
                std::lock_guard<std::mutex> g(mu);
                producers_left--;
            }
            cv.notify_one();
        });
    std::thread sched([&] {
        std::vector<Q *> batch;
        std::vector<int64_t> last_arrival(NC, 0);
        for (;;) {
            size_t c;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return producers_left == 0 || sm::sched_pick(pending) != SIZE_MAX; });
                c = sm::sched_pick(pending);
                if (c == SIZE_MAX) return;  // producers done and every queue empty
                // the chosen corpus holds the oldest queued query
                for (int k = 0; k < NC; k++)
                    if (!pending[k].empty() && pending[k].front()->arrival_ns < pending[c].front()->arrival_ns)
                        fail("picked a corpus whose head is not the oldest");
                sm::sched_take(pending[c], MAXB, batch);
            }
            // mock executor: run the batch outside the lock
            if (batch.empty() || batch.size() > MAXB) fail("batch size");
            for (size_t i = 0; i < batch.size(); i++) {
                if (batch[i]->corpus != c) fail("mixed corpora in a batch");
                if (batch[i]->arrival_ns <= last_arrival[c]) fail("out of arrival order");
                last_arrival[c] = batch[i]->arrival_ns;
                ran[batch[i]->ticket]++;
            }
        }
    });
    for (auto &t : prod) t.join();
    sched.join();
    for (size_t t = 1; t <= all.size(); t++)
        if (ran[t] != 1) fail("a query ran other than once");
    if (bad) return 1;
    std::printf("ok\n");
    return 0;
}
