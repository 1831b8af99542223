// Batch formation of the query server (host code only, no HIP): queries wait in
// one FIFO queue per corpus; the next batch takes the corpus whose oldest queued
// query arrived first (ties: the lower ticket) and up to max_batch of its queries
// in arrival order. Q is any type with arrival_ns and ticket members.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <deque>
#include <vector>

namespace sm {

// Index of the corpus to serve next, or SIZE_MAX when every queue is empty.
template <class Q>
size_t sched_pick(const std::vector<std::deque<Q *>> &pending)
{
    size_t best = SIZE_MAX;
    int64_t best_t = INT64_MAX;
    uint64_t best_tk = UINT64_MAX;
    for (size_t k = 0; k < pending.size(); k++) {
        if (pending[k].empty()) continue;
        const Q *q = pending[k].front();
        if (q->arrival_ns < best_t || (q->arrival_ns == best_t && q->ticket < best_tk)) {
            best = k;
            best_t = q->arrival_ns;
            best_tk = q->ticket;
        }
    }
    return best;
}

// Moves up to max_batch queries from the front of dq to out (cleared first).
template <class Q>
void sched_take(std::deque<Q *> &dq, size_t max_batch, std::vector<Q *> &out)
{
    out.clear();
    while (!dq.empty() && out.size() < max_batch) {
        out.push_back(dq.front());
        dq.pop_front();
    }
}

}  // namespace sm
