// Ring allocator for the server's pinned host result arena (host code only, no
// HIP): regions are taken at the head in allocation order and may be given back
// in any order; the tail advances over the freed prefix. A region that would
// cross the end of the ring starts at offset 0 instead, and the skipped end is
// charged to it until it is released.
#pragma once

#include <stdint.h>

#include <deque>
#include <memory>

namespace sm {

struct RingRegion {
    uint64_t off = 0, bytes = 0;  // bytes includes the skipped end, if any
    bool freed = false;
};

struct Ring {
    uint64_t cap = 0, head = 0, used = 0;
    std::deque<std::shared_ptr<RingRegion>> live;  // allocation order

    // Whether alloc(bytes) would succeed now (always for 0 bytes, which need no region).
    bool fits(uint64_t bytes) const
    {
        bytes = (bytes + 255) & ~255ull;
        if (bytes == 0) return true;
        if (bytes > cap) return false;
        const uint64_t pad = head + bytes > cap ? cap - head : 0;
        return used + pad + bytes <= cap;
    }

    // Whether a region of `bytes` fits the ring at all (when nothing else is held).
    bool ever_fits(uint64_t bytes) const { return ((bytes + 255) & ~255ull) <= cap; }

    // A region of at least `bytes` (rounded up to 256), or null if it does not fit now.
    std::shared_ptr<RingRegion> alloc(uint64_t bytes)
    {
        bytes = (bytes + 255) & ~255ull;
        if (bytes == 0 || bytes > cap) return nullptr;
        uint64_t pad = 0;
        if (head + bytes > cap) pad = cap - head;  // wrap: skip the end of the ring
        if (used + pad + bytes > cap) return nullptr;
        auto r = std::make_shared<RingRegion>();
        r->off = (head + pad) % cap;
        r->bytes = pad + bytes;
        head = (r->off + bytes) % cap;
        used += r->bytes;
        live.push_back(r);
        return r;
    }

    void release(const std::shared_ptr<RingRegion> &r)
    {
        r->freed = true;
        while (!live.empty() && live.front()->freed) {
            used -= live.front()->bytes;
            live.pop_front();
        }
        if (live.empty()) head = used = 0;
    }
};

}  // namespace sm
