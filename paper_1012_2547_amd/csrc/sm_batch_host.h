// Host side of the batched search, shared by the batch C ABI (sm_batch.cpp) and
// the server (sm_server.cpp): the plan of a batch (sorted patterns, groups, text
// chunking), its workspace layout, and the two enqueue steps (count, then
// writes of any window of the CSR output).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "sm_internal.h"

namespace sm {

struct BatchLayout {  // byte offsets inside the batch workspace
    uint64_t pats, groups, cgroups, mqgroups, mqtabs, mqwtabs, params, patbytes, cnt, chunk_off, totals,
        csr, wgroups, wroute, mqwlist, hqgroups, hqtabs, mqstash, mqstash_n, single, need;
};

struct BatchJob {
    sm_corpus *c = nullptr;
    uint32_t P = 0;
    const uint8_t *pats = nullptr;    // host pattern bytes, valid for the job's life
    const uint64_t *pat_off = nullptr;
    std::vector<BatchPat> bpats;      // patterns searched inside batch launches, sorted
    std::vector<BatchGroup> groups;   // write pass: all batch patterns
    std::vector<BatchGroup> cgroups;  // count pass: patterns outside the prefix filter
    std::vector<MqGroup> mq;          // count pass: prefix filter groups
    std::vector<uint8_t> mqtab;       // their tables (MQ_TAB_BYTES each)
    std::vector<uint8_t> mqwtab;      // the same groups' write tables (every pattern with its slot)
    std::vector<int32_t> mq_of;       // sorted pattern -> its filter group, or -1
    uint32_t mq_max_m = 0;
    // the count pass keeps each (chunk, filter group) item's hits when they fit
    // (MQ_STASH); after the count, h_stash_n (nchunks x mq.size(), host, set by the
    // caller) tells which items kept them
    bool stash = false;
    const uint32_t *h_stash_n = nullptr;
    // write plan, built from the counts (batch_write_plan); without one the write
    // pass runs every pattern's own scanner (groups)
    bool wplan = false;
    std::vector<BatchGroup> wgroups;  // per-pattern write groups
    // per sorted pattern: 2 = written from the filter's kept hits (a pass over its count
    // group's items), 4 = by a filter pass over the text with the window's other such
    // patterns (hq groups); 1 own scanner, 3 single-pattern pipeline
    std::vector<uint8_t> wroute;
    std::vector<uint32_t> mqwlist;    // count groups with route-2 patterns in the window
    std::vector<MqGroup> hq;          // route-4 patterns of the window, by q-class and length
    std::vector<uint8_t> hqtab;       // their tables
    uint32_t max_hq = 0;              // hq groups the layout has room for
    std::vector<uint32_t> longp;      // m > BATCH_MAX_M: searched one pattern at a time
    // write plan: patterns of the window dense enough that the single-pattern
    // pipeline (bitmap form, coalesced emit) beats a batch rescan; possible when the
    // workspace holds single-pattern scratch for every m up to single_max_m
    std::vector<uint32_t> singlep;
    uint32_t single_max_m = 0;
    uint64_t patbytes = 0;
    uint32_t chunk_tiles = 1;
    uint64_t nchunks = 0, ntiles = 0;
    BatchLayout L{};
};

// Single-pattern scratch reserved in a batch workspace: none (asynchronous
// find_all), for the long patterns (counting), or also for the dense patterns of
// the write waves (handle, synchronous find_all, server).
enum BatchWs { WS_NONE = 0, WS_LONG = 1, WS_WRITE = 2 };

// Validates and plans P patterns against the corpus (host only), with the
// workspace scratch of kind ws (BatchWs).
int batch_plan(sm_corpus *c, const uint8_t *pats, const uint64_t *pat_off, uint32_t P, int ws,
               BatchJob &j);

// Bytes of the host image uploaded by the count step (pattern table, groups and
// pattern bytes), and its contents.
uint64_t batch_image_bytes(const BatchJob &j);
// (chunk, filter group) items whose hit counts the count step leaves at L.mqstash_n
// (u32 each) for the write plan; 0 when the job keeps no hits.
uint64_t batch_stash_items(const BatchJob &j);
void batch_fill_image(const BatchJob &j, uint8_t *dst);

// Count step: uploads the image (h_image: batch_fill_image's output, pinned or
// pageable; null = built here), builds the tables, counts every pattern ->
// d_totals[0..P) (caller order) and, when d_csr is not null, the exclusive scan
// -> d_csr[0..P]. keep_chunk_off keeps what a later write step needs.
int batch_count_enqueue(BatchJob &j, uint8_t *ws, const uint8_t *h_image, uint64_t *d_totals,
                        uint64_t *d_csr, bool keep_chunk_off, hipStream_t st);

// Pinned staging for write-plan uploads: refilled only after the previous
// upload from it has completed (its event).
struct PlanStaging {
    uint8_t *host = nullptr;
    uint64_t cap = 0;
    hipEvent_t ev = nullptr;
    bool pending = false;
    ~PlanStaging();
};

// Routes every pattern with occurrences in the CSR window [lo, hi) to its own
// scanner or to a shared prefix filter write group, from the host copy of the
// CSR offsets, and uploads the plan into the workspace through stg (enqueued on
// st). The next write uses it.
int batch_write_plan(BatchJob &j, uint8_t *ws, const uint64_t *h_csr, uint64_t lo, uint64_t hi,
                     hipStream_t st, PlanStaging &stg);

// Write step: CSR entries [lo, hi) -> d_out[0 .. hi - lo). Needs the count
// step's workspace (keep_chunk_off) and d_csr; h_csr (host copy of d_csr) is
// needed only when the job has long patterns or the plan routes patterns to the
// single-pattern pipeline.
int batch_write_enqueue(BatchJob &j, uint8_t *ws, const uint64_t *d_csr, const uint64_t *h_csr,
                        uint64_t *d_totals, int64_t *d_out, uint64_t lo, uint64_t hi,
                        hipStream_t st);

int batch_err(int status, const char *fmt, ...);

}  // namespace sm
