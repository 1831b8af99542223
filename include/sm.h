/*
 * sm.h -- C ABI of an MI355X (gfx950) library for online exact string matching.
 *
 * The operation (Faro & Lecroq, "The Exact String Matching Problem: a
 * Comprehensive Experimental Evaluation", Section 1): given a text t of length n
 * and a pattern p of length m over an alphabet of size sigma, find ALL
 * occurrences of p in t. Here:
 *   - t and p are raw bytes (0..255); sigma is a property of the data, never an
 *     argument; there is no case folding and no sentinel;
 *   - an occurrence is a 0-based offset i with 0 <= i <= n-m and
 *     t[i+k] == p[k] for 0 <= k < m; overlapping occurrences all count;
 *   - positions are reported as int64 in strictly ascending order.
 *
 * Conventions shared by every entry point
 *   - m == 0 is invalid (SM_EINVAL). m > n or n == 0 gives zero occurrences
 *     (SM_OK). m must be < 2^32.
 *   - `count` receives the TOTAL number of occurrences on SM_OK and on
 *     SM_TRUNCATED. When the total exceeds `cap`, exactly the first `cap`
 *     positions (the sorted prefix) are written and SM_TRUNCATED is returned.
 *     Count first, then size the output, is the intended two-call pattern.
 *   - Arguments are validated before any device work; a NULL text with n > 0, a
 *     NULL pattern, a NULL count, or a NULL output with cap > 0 is SM_EINVAL.
 *   - The caller owns every buffer passed in; the library keeps no caller
 *     pointer after a call returns (a corpus opened with text_on_device borrows
 *     its device text until sm_corpus_close).
 *   - Results do not depend on the algorithm, tile size, q or any other tuning
 *     choice: every algorithm is exact and results are bit-identical.
 *   - Calls are reentrant. On failure, sm_last_error() returns a thread-local
 *     message describing the last non-OK status of the calling thread.
 *   - Device pointers are HIP device addresses on the current HIP device;
 *     `stream` is a hipStream_t (NULL = the default stream).
 */
#ifndef SM_H
#define SM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum sm_status {
    SM_OK = 0,
    SM_TRUNCATED = 1,   /* not an error: more occurrences than `cap` */
    SM_EINVAL = -1,     /* invalid argument; nothing was launched */
    SM_ENOMEM = -2,     /* a device or host allocation failed */
    SM_EDEVICE = -3,    /* a HIP call failed, or the device is not gfx950 */
    SM_EBUSY = -4       /* the resource is in use (server queue full, closing) */
};

/* A device-resident text (see sm_corpus_open). */
typedef struct sm_corpus sm_corpus;

/* Scan algorithms (paper, Figs. 1 and 3). SM_ALGO_AUTO lets the planner choose. */
enum sm_algo {
    SM_ALGO_AUTO = 0,
    SM_ALGO_SHIFT_AND = 1, /* Shift-And / Shift-Or, bit-parallel (Fig. 3), one step per text byte;
                              for m > 49 the pattern's last 17 bytes are scanned (its last 49
                              when its smallest period lies in 18..49) and the rest verified (a
                              start one period after an occurrence, the period inside the
                              scanned suffix, without reading): linear on texts of one symbol,
                              where the planner takes it for every m */
    SM_ALGO_BNDM = 2,      /* Backward Nondeterministic DAWG Matching, m <= 64 (Fig. 3); with q = 2 or 4
                              the window's last q bytes are read at once (BNDMq, Fig. 3) */
    SM_ALGO_SBNDM = 3,     /* Simplified BNDM (Fig. 3); any m: for m > 64 its factor form, in which
                              the pattern's last 64 bytes are searched and the first m - 64 of each
                              start found are verified (after the factor's own occurrences the
                              window shifts by the factor's period) */
    SM_ALGO_HASHQ = 4,     /* Hash-q: hashed q-gram skip + verification, any m >= q (Fig. 1) */
    SM_ALGO_BLOCK = 5,     /* 16-byte block fingerprint filter after SSEF (Fig. 1), 144 <= m <= 4096:
                              one aligned 16-byte block per S text bytes (S the largest multiple of 16
                              <= m - 15) is read and looked up among
                              the pattern's blocks, candidates verified byte-exactly */
    SM_ALGO_BRUTE = 6,     /* brute force (Fig. 1, BF) over packed bytes, m <= 8: the four starts of a
                              text word are compared with the pattern at once, byte-parallel */
    SM_ALGO_FSBNDM = 7     /* Forward SBNDM (Fig. 3), m <= 63: SBNDM for the pattern followed by one
                              position that matches any byte, so the byte after the window is read
                              first as a look-ahead */
};

/*
 * Tuning options. A NULL sm_opts*, or zero in a field, means "planner's choice".
 * Options change speed only, never results. Invalid combinations (BNDM with
 * m > 64, FSBNDM with m > 63, the block filter with m outside [144, 4096], brute force with
 * m > 8, q > m or
 * q > 16, lane_bytes not in {16,32,64,128}, hbits outside [8,12]) are SM_EINVAL.
 * lane_bytes, q and hbits do not apply to the block filter (its tile is the
 * starts of 256 sampled blocks).
 */
typedef struct sm_opts {
    int32_t algo;         /* enum sm_algo */
    int32_t lane_bytes;   /* candidate starts per lane; a tile is 256 * lane_bytes starts */
    int32_t q;            /* Hash-q gram length, 1..16; for SBNDM the q-gram read at once, 1, 2, 4 or 8;
                             for BNDM 1, 2 or 4 */
    int32_t sigma_hint;   /* expected alphabet size of the text (planner input only) */
    int32_t tiles_per_wg; /* consecutive tiles per workgroup, >= 1 */
    int32_t hbits;        /* Hash-q table has 2^hbits buckets */
    int32_t reserved[2];  /* must be zero */
} sm_opts;

/* What the planner chose for a pattern of length m (introspection). suffix: for
 * Shift-And with m > 49, the length of the pattern's suffix the scan matches (17, or
 * 49 when the pattern's smallest period lies in 18..49 or m exceeds 2^24), else 0. */
typedef struct sm_plan_info {
    int32_t algo, lane_bytes, q, hbits, tiles_per_wg, suffix;
} sm_plan_info;

const char *sm_version(void);
const char *sm_last_error(void);

/*
 * sm_find_all -- all occurrences, host buffers, synchronous.
 *   text[n], pat[m]: host bytes.  out_pos[cap]: host int64 output.
 *   *count: total number of occurrences.
 * The text is copied to the device for the call (PCIe included); use a corpus or
 * the *_dev / *_async forms for device-resident texts.
 */
int sm_find_all(const uint8_t *text, uint64_t n, const uint8_t *pat, uint64_t m,
                int64_t *out_pos, uint64_t cap, uint64_t *count);

/* sm_count -- number of occurrences only (host buffers, synchronous). */
int sm_count(const uint8_t *text, uint64_t n, const uint8_t *pat, uint64_t m, uint64_t *count);

/*
 * Device-resident text and output, synchronous with respect to `count`:
 *   d_text[n]: device bytes (any alignment).  pat[m]: HOST bytes.
 *   d_out[cap]: device int64.  *count: host.  Work is enqueued on `stream`, which
 *   is synchronized before returning. A scratch workspace is allocated and cached
 *   per calling thread.
 */
int sm_find_all_dev(const uint8_t *d_text, uint64_t n, const uint8_t *pat, uint64_t m,
                    int64_t *d_out, uint64_t cap, uint64_t *count, void *stream);
int sm_count_dev(const uint8_t *d_text, uint64_t n, const uint8_t *pat, uint64_t m,
                 uint64_t *count, void *stream);

/*
 * Asynchronous form: no host synchronization, no allocation. The total is
 * written to *d_count (device uint64) in stream order; d_out receives the first
 * min(cap, total) positions. d_work is a caller-owned device workspace of at
 * least sm_workspace_size(n, m, opts) bytes, 256-byte aligned, with no required
 * initial contents; it must not be used by two calls that may run concurrently. The pattern (host) is
 * captured into kernel arguments when m <= 3072 bytes, so the host buffer may be
 * reused as soon as the call returns; longer patterns are copied with a
 * host-blocking hipMemcpyAsync.
 *
 * find_all runs three kernels: a count pass over the text (which also keeps the
 * hit offsets of tiles with few hits), a scan of the per-tile counts, and an
 * emit pass that writes positions. Tiles with many hits are re-read by the emit
 * pass, except in Shift-And scans with lanes of >= 32 starts, where the count
 * pass keeps their hits as a bitmap of starts. count
 * runs the first kernel only; its workspace may be smaller.
 *
 * The size depends on m: for m <= 64 it holds that bitmap (n bits), fewer tiles
 * are needed as m grows, and the lane width (hence the tile count) the planner
 * may pick differs between lengths. sm_workspace_size_upto(n, M, opts) is the
 * size of a workspace that serves every pattern length 1..M under the same
 * options (the maximum of sm_workspace_size over those lengths, or a bound
 * above it for M > 4097, where the planner's lanes no longer depend on m under
 * the built-in table).
 */
uint64_t sm_workspace_size(uint64_t n, uint64_t m, const sm_opts *opts);
uint64_t sm_workspace_size_upto(uint64_t n, uint64_t m_max, const sm_opts *opts);
int sm_find_all_async(const uint8_t *d_text, uint64_t n, const uint8_t *pat, uint64_t m,
                      int64_t *d_out, uint64_t cap, uint64_t *d_count, void *d_work,
                      uint64_t work_bytes, const sm_opts *opts, void *stream);
int sm_count_async(const uint8_t *d_text, uint64_t n, const uint8_t *pat, uint64_t m,
                   uint64_t *d_count, void *d_work, uint64_t work_bytes, const sm_opts *opts,
                   void *stream);

/*
 * sm_find_all_noalloc -- for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same search as sm_find_all_async, with the workspace taken from a static device
 * array of SM_NOALLOC_SCRATCH_BYTES held by the library on every device it runs on
 * until the process ends. The call makes no hipMalloc, hipFree, pinned-memory or
 * other allocating call; it only enqueues kernels on `stream`.
 *   d_text[n]: device bytes.  pat[m]: HOST bytes, m <= 3072 (captured into kernel
 *   arguments, so the host buffer may be reused at once).  d_out[cap]: device
 *   int64, the first min(cap, total) positions.  *d_count: device uint64, the
 *   total, written in stream order.  opts: as sm_find_all_async (NULL = planner).
 * Errors: the arguments of sm_find_all_async; m > 3072, or an (n, m, lanes) whose
 * workspace (sm_workspace_size) exceeds SM_NOALLOC_SCRATCH_BYTES, is SM_EINVAL
 * before any device work (at the planner's lanes, n up to 2^30 fits every m).
 * Every call on one device shares that device's array and leaves its contents
 * behind (the next call needs none of them): two calls that may overlap in time
 * on the same device -- different streams, threads or graph replays running
 * concurrently -- race on it and give wrong results. Serialize them (one stream,
 * or events between them).
 */
#define SM_NOALLOC_SCRATCH_BYTES (256ull << 20)
int sm_find_all_noalloc(const uint8_t *d_text, uint64_t n, const uint8_t *pat, uint64_t m,
                        int64_t *d_out, uint64_t cap, uint64_t *d_count, const sm_opts *opts,
                        void *stream);

/*
 * Batched search: P patterns against one corpus, the text streamed once per
 * group of patterns instead of once per pattern (kernels and grouping in the
 * package's csrc/sm_batch.*). Patterns are concatenated in pats; pattern i is
 * pats[pat_off[i] .. pat_off[i+1]) (pat_off has P + 1 entries, non-decreasing,
 * no empty pattern: SM_EINVAL). Results are exactly the single-pattern results.
 *
 * sm_batch_count: counts[i] = number of occurrences of pattern i (host array).
 * sm_batch_find_all: CSR output. out_off[i] = sum of the counts of patterns
 *   < i (P + 1 entries, always complete); pattern i's positions, ascending, go
 *   to out[out_off[i] .. out_off[i+1]) for the entries below cap. Returns
 *   SM_TRUNCATED when out_off[P] > cap.
 * *_async: device outputs (d_counts / d_out, d_out_off), caller workspace of
 *   sm_batch_workspace_size bytes (256-byte aligned), enqueued on `stream`; the
 *   pattern bytes are copied from the host during the call. The asynchronous
 *   find_all takes patterns up to 2048 bytes; the synchronous forms take any m.
 */
uint64_t sm_batch_workspace_size(const sm_corpus *corpus, const uint8_t *pats,
                                 const uint64_t *pat_off, uint32_t P);
int sm_batch_count(sm_corpus *corpus, const uint8_t *pats, const uint64_t *pat_off, uint32_t P,
                   uint64_t *counts);
int sm_batch_find_all(sm_corpus *corpus, const uint8_t *pats, const uint64_t *pat_off, uint32_t P,
                      int64_t *out, uint64_t cap, uint64_t *out_off);
int sm_batch_count_async(sm_corpus *corpus, const uint8_t *pats, const uint64_t *pat_off,
                         uint32_t P, uint64_t *d_counts, void *d_work, uint64_t work_bytes,
                         void *stream);
int sm_batch_find_all_async(sm_corpus *corpus, const uint8_t *pats, const uint64_t *pat_off,
                            uint32_t P, int64_t *d_out, uint64_t cap, uint64_t *d_out_off,
                            void *d_work, uint64_t work_bytes, void *stream);

/*
 * Batch handle: the count step of a batched find_all, kept so that the output
 * can be written in windows (waves) of any size. sm_batch_open plans the
 * patterns (as sm_batch_find_all), allocates the batch's workspace, counts
 * every pattern and keeps the CSR offsets (synchronous). sm_batch_offsets
 * copies them (P + 1 entries) to the host. sm_batch_write_async writes the CSR
 * entries [lo, hi) (0 <= lo <= hi <= total) to the device buffer d_out[0 ..
 * hi - lo), enqueued on `stream`: pattern i's positions are entries out_off[i]
 * .. out_off[i+1], ascending. Writes on one batch share its workspace and must
 * not overlap in time (one stream, or waits between them). The library copies
 * the patterns at open; sm_batch_close waits for the device and frees the batch.
 *
 * sm_batch_find_all writes through the same windows, in waves of at most the
 * budget set by sm_batch_set_wave_bytes (default 64 GiB, 0 restores it; it is
 * also kept below half of the free device memory), so the device never holds
 * the whole output.
 */
typedef struct sm_batch sm_batch;
int sm_batch_open(sm_corpus *corpus, const uint8_t *pats, const uint64_t *pat_off, uint32_t P,
                  sm_batch **batch);
int sm_batch_offsets(const sm_batch *batch, uint64_t *out_off);
int sm_batch_write_async(sm_batch *batch, uint64_t lo, uint64_t hi, int64_t *d_out, void *stream);
int sm_batch_close(sm_batch *batch);
int sm_batch_set_wave_bytes(uint64_t bytes);
/* How the write pass of sm_batch_open, sm_batch_find_all and the server finds the
 * positions of each pattern with occurrences (speed only, never results):
 * 0 = automatic (from the counts of the window: the single-pattern pipeline for
 * patterns of at most 64 bytes with at least one occurrence per 384 text bytes; the
 * shared prefix-filter pass of the pattern's count group -- which copies out the
 * hits the count step kept, up to 2048 per text chunk and group, and scans the
 * other chunks again -- when the group kept every chunk's hits or its patterns would
 * otherwise rescan most of the text; each pattern's own scanner for the rest),
 * 1 = every pattern's own scanner, 2 = the shared pass for every pattern of a
 * filter group sparse enough for it (at most 16 occurrences per 4096 text bytes),
 * 3 = the single-pattern pipeline for every pattern of at most 64 bytes. Patterns
 * longer than 2048 bytes always take the single-pattern pipeline. Process-wide;
 * SM_EINVAL outside 0..3. */
int sm_batch_set_write_policy(int policy);

/*
 * Server: continuous batching of single-pattern queries over resident corpora
 * (the paper's workload, Section 2, one pattern per query, served many at a
 * time). Queries are queued per corpus; a scheduler thread batches the queued
 * queries of one corpus (oldest first, at most max_batch) onto any free one of
 * `slots` pipeline slots (own HIP stream, workspace and pool_bytes / slots of
 * device output staging) and starts the batch's count step; the next batch can be
 * formed and counted while earlier ones are written and copied.
 *
 * Admission by memory: the count step gives every query's exact number of
 * positions. Results live in one pinned host arena of host_bytes, the only
 * pinned memory results ever take. Batches are admitted in dispatch order: the
 * longest prefix of the batch whose positions fit the arena is written (in waves
 * of at most the slot's staging size), the rest goes back to the front of its
 * queue and is counted again later (`deferred`). When not even the first query
 * fits, completed results that no caller has received yet are moved from the
 * arena to pageable memory (`evicted`), oldest first; if that is not enough,
 * admission waits until results are freed or batches complete. A query whose
 * positions alone exceed host_bytes fails with SM_ENOMEM (`rejected`). A result
 * returned by wait/poll stays where it is until sm_result_free; a caller that
 * frees each result before waiting for the next never stalls admission for good.
 *
 * sm_server_create: zero fields take defaults (pool 16 GiB, host arena 2 GiB,
 *   max_batch 256, 2 slots, max_pending 2^20 queued queries, HIP graphs on); the
 *   server runs on the current HIP device. With graphs on, each batch's count step
 *   and write waves are captured as HIP graphs and replayed through per-slot
 *   executables, updated in place while the launch sequence keeps its shape
 *   (batches with patterns over 2048 bytes launch directly).
 * sm_server_add_corpus: registers an open corpus (borrowed: keep it open until
 *   sm_server_destroy); ids are 0, 1, ...
 * sm_server_submit: copies the pattern and queues the query; arrival_ns is its
 *   arrival time on sm_now_ns's clock (<= 0: now) and latency is measured from
 *   it. SM_EBUSY when max_pending queries are queued. Thread-safe.
 * sm_server_wait: waits up to timeout_us (< 0: forever) for the query; SM_OK
 *   with *res filled, SM_EBUSY if it is still running, or the query's error
 *   (SM_ENOMEM: its positions exceed the arena).
 *   res->positions (res->count entries, ascending) is library-owned host memory,
 *   valid until sm_result_free(ticket). sm_server_poll = wait with timeout 0.
 * sm_server_stats: latency percentiles (arrival to positions on the host) of
 *   the queries completed since the last reset, throughput and memory counters.
 * sm_server_destroy: drops queued queries, finishes dispatched ones (a batch still
 *   waiting for arena memory fails with SM_EBUSY), frees all.
 */
typedef struct sm_server sm_server;
typedef struct sm_server_config {
    uint64_t pool_bytes;   /* device output staging, split across the slots */
    uint64_t host_bytes;   /* pinned host result arena */
    uint32_t max_batch;    /* queries per batch */
    uint32_t slots;        /* pipeline slots (streams), 1..8 */
    uint32_t max_pending;  /* queued queries before submit returns SM_EBUSY */
    uint32_t graphs_off;   /* nonzero: launch directly instead of through HIP graphs */
    uint32_t reserved[4];  /* must be zero */
} sm_server_config;
typedef struct sm_result {
    int32_t status;
    uint32_t corpus;
    uint64_t count;             /* occurrences */
    const int64_t *positions;   /* count ascending positions (host, library-owned) */
    int64_t arrival_ns, start_ns, done_ns;  /* arrival, batch dispatch, results on host */
    uint32_t batch_size;        /* queries in its batch */
    uint32_t reserved;
} sm_result;
typedef struct sm_server_metrics {
    uint64_t completed, pending, batches, batched_queries;
    uint64_t text_bytes;        /* sum over admitted batches of n x queries (pattern-bytes) */
    uint64_t out_bytes;         /* positions written, bytes */
    uint64_t write_waves;
    uint64_t deferred;          /* queries sent back to their queue: their positions did not fit the arena */
    int64_t p50_ns, p99_ns, p999_ns, max_ns;
    double mean_ns;
    int64_t span_ns;            /* first arrival to last completion */
    double qps;                 /* completed / span */
    uint64_t graph_launches;    /* graph launches (count steps and write waves) */
    uint64_t graph_builds;      /* of which needed a new executable (shape changed) */
    uint64_t evicted;           /* results moved from the arena to pageable memory */
    uint64_t evicted_bytes;
    uint64_t rejected;          /* queries failed with SM_ENOMEM (positions alone exceed the arena) */
    uint64_t mem_waits;         /* times admission waited for arena memory */
    uint64_t host_peak_bytes;   /* most arena bytes held at once since the last reset */
    uint64_t host_arena_bytes;  /* the arena's size (host_bytes) */
} sm_server_metrics;
int64_t sm_now_ns(void);
int sm_server_create(const sm_server_config *cfg, sm_server **server);
int sm_server_add_corpus(sm_server *server, sm_corpus *corpus, uint32_t *corpus_id);
int sm_server_submit(sm_server *server, uint32_t corpus_id, const uint8_t *pat, uint64_t m,
                     int64_t arrival_ns, uint64_t *ticket);
int sm_server_wait(sm_server *server, uint64_t ticket, int64_t timeout_us, sm_result *res);
int sm_server_poll(sm_server *server, uint64_t ticket, sm_result *res);
int sm_result_free(sm_server *server, uint64_t ticket);
int sm_server_stats(sm_server *server, sm_server_metrics *stats);
int sm_server_reset_stats(sm_server *server);
int sm_server_destroy(sm_server *server);

/*
 * Planner tuning table. The planner picks the first entry whose alphabet-size
 * range and pattern-length range contain (sigma, m); sigma is the corpus's
 * sigma_eff, opts->sigma_hint, or an estimate from the pattern's byte counts.
 * Zero fields mean "planner default". Entries whose algorithm cannot handle m
 * are skipped. The library carries a table measured on MI355X (see the package's
 * tune module); sm_tune_set replaces it (count = 0 restores it).
 */
typedef struct sm_tune_entry {
    int32_t sigma_lo, sigma_hi;
    uint32_t m_lo, m_hi;
    int32_t algo, lane_bytes, q, tiles_per_wg, hbits, reserved;
} sm_tune_entry;
int sm_tune_set(const sm_tune_entry *entries, uint32_t count);
int sm_tune_get(sm_tune_entry *entries, uint32_t cap, uint32_t *count);

/* Planner introspection: the plan a call with these arguments would use. The
 * pattern is read on the host only (its byte statistics inform the planner). */
int sm_plan_query(const uint8_t *pat, uint64_t m, const sm_opts *opts, sm_plan_info *info);

/*
 * Corpus: a device-resident text reused across queries (the paper's fixed text
 * buffers, Section 2). sm_corpus_open copies a host text to the device
 * (text_on_device = 0) or borrows a device pointer (text_on_device = 1; the
 * caller keeps it alive until close), and probes its byte histogram once; the
 * planner then uses the measured alphabet size. A corpus is immutable after
 * open; concurrent queries on it are allowed.
 */
int sm_corpus_open(const uint8_t *text, uint64_t n, int text_on_device, sm_corpus **corpus);
int sm_corpus_close(sm_corpus *corpus);
/* host output, synchronous */
int sm_corpus_find_all(sm_corpus *corpus, const uint8_t *pat, uint64_t m, int64_t *out_pos,
                       uint64_t cap, uint64_t *count);
int sm_corpus_count(sm_corpus *corpus, const uint8_t *pat, uint64_t m, uint64_t *count);
/* histogram[256], number of distinct bytes (sigma) and the effective alphabet size
 * sigma_eff = 1 / sum_c p_c^2 (the size of the uniform alphabet with the same
 * probability that two random bytes are equal); any pointer may be NULL. */
int sm_corpus_stats(const sm_corpus *corpus, uint64_t *histogram, int32_t *sigma,
                    double *sigma_eff);
/* Asynchronous corpus queries: as sm_find_all_async / sm_count_async on the
 * corpus text, planned with the corpus's measured sigma_eff. */
int sm_corpus_find_all_async(sm_corpus *corpus, const uint8_t *pat, uint64_t m, int64_t *d_out,
                             uint64_t cap, uint64_t *d_count, void *d_work, uint64_t work_bytes,
                             const sm_opts *opts, void *stream);
int sm_corpus_count_async(sm_corpus *corpus, const uint8_t *pat, uint64_t m, uint64_t *d_count,
                          void *d_work, uint64_t work_bytes, const sm_opts *opts, void *stream);
/* device address of the corpus text and its length */
int sm_corpus_text(const sm_corpus *corpus, const uint8_t **d_text, uint64_t *n);

/*
 * Kernel timing (profiling aid). sm_prof_enable(k), k >= 1: every k-th
 * *_async/_dev call from now on (the first, then every k-th after it, in issue
 * order) records HIP events on its stream around its kernels (each event costs
 * the stream a few microseconds, so a stride keeps timed loops close to their
 * unprofiled speed); 0 turns recording off, a negative k is SM_EINVAL.
 * sm_prof_collect waits for the recorded events, returns the accumulated times
 * of the recorded calls and clears them.
 */
typedef struct sm_prof {
    uint64_t calls;        /* calls recorded */
    double count_ms;       /* count kernel (the pass over the text; the dominant kernel) */
    double emit_ms;        /* tile scan + emit kernels (find_all only) */
    double total_ms;       /* whole calls: pattern preparation + all kernels */
    uint64_t text_bytes;   /* sum of n over the calls */
    uint64_t sampled_calls;   /* of the calls, those whose count pass is the block filter, */
    double sampled_count_ms;  /* which reads one 16-byte block per about m - 15 bytes, and its time */
    /* batched count passes (sm_batch_count*, sm_batch_open): while recording is on,
     * every pass not captured into a HIP graph is recorded, whatever the stride */
    uint64_t batch_calls;          /* passes recorded */
    double batch_ms;               /* their whole time: preparation, scanner groups, filter, scans */
    uint64_t filter_launches;      /* shared multi-pattern filter launches (mq_count_kernel) in them */
    double filter_ms;              /* time of those launches */
    uint64_t filter_pattern_bytes; /* sum over the passes of n x patterns in the filter's groups */
} sm_prof;
int sm_prof_enable(int every);
int sm_prof_collect(sm_prof *out);

#ifdef __cplusplus
}
#endif

#endif /* SM_H */
