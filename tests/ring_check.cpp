// Randomised check of the server's result-arena ring allocator (host code).
// Exits non-zero with a message on the first violated property.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "sm_ring.h"

static int fail(const char *what, int step)
{
    std::printf("FAIL %s at step %d\n", what, step);
    return 1;
}

int main()
{
    std::mt19937_64 rng(12345);
    for (uint64_t cap : {256ull * 17, 4096ull, 1ull << 20}) {
        sm::Ring ring;
        ring.cap = cap;
        std::vector<std::shared_ptr<sm::RingRegion>> live;
        std::vector<uint64_t> want;  // requested bytes per live region
        for (int step = 0; step < 200000; step++) {
            const bool do_alloc = live.empty() || (rng() % 100) < 52;
            if (do_alloc) {
                const uint64_t req = 1 + rng() % (cap / 4);
                const uint64_t held = ring.used;  // live regions and freed ones not yet passed by the tail
                auto r = ring.alloc(req);
                // with at most half the ring held, a request of at most a quarter
                // always fits (one side of the split free space is big enough)
                if (!r && held <= cap / 2 && ((req + 255) & ~255ull) <= cap / 4)
                    return fail("refused a request that fits", step);
                if (!r) continue;
                const uint64_t rb = (req + 255) & ~255ull;
                if (r->off % 256 || r->off + rb > cap) return fail("region outside the ring", step);
                for (auto &o : live) {  // no overlap with any live region's payload
                    const uint64_t a0 = r->off, a1 = r->off + rb;
                    const uint64_t b0 = o->off, b1 = o->off + want[&o - &live[0]];
                    if (a0 < b1 && b0 < a1) return fail("overlapping regions", step);
                }
                live.push_back(r);
                want.push_back(rb);
            } else {
                const size_t k = rng() % live.size();
                ring.release(live[k]);
                live.erase(live.begin() + k);
                want.erase(want.begin() + k);
            }
            if (ring.used > cap) return fail("more than the ring in use", step);
        }
        for (auto &r : live) ring.release(r);
        if (ring.used != 0 || ring.head != 0) return fail("not empty after releasing all", -1);
        if (!ring.alloc(cap)) return fail("whole ring refused when empty", -1);
    }
    std::printf("ok\n");
    return 0;
}
