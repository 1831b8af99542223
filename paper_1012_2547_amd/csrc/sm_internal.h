// Internal declarations shared by the host library and the HIP kernels.
// Not part of the public C ABI (include/sm.h).
#pragma once
#include <stdint.h>
#include <stddef.h>
#include <hip/hip_runtime.h>

struct sm_opts;  // include/sm.h

namespace sm {

// Scan algorithms (values match SM_ALGO_* in include/sm.h).
enum Algo : int32_t {
    ALGO_AUTO = 0,
    ALGO_SHIFT_AND = 1,  // bit-parallel prefix automaton, m <= 64 (Fig. 3, SA/SO)
    ALGO_BNDM = 2,       // bit-parallel backward factor automaton, m <= 64 (Fig. 3, BNDM)
    ALGO_SBNDM = 3,      // BNDM without prefix tracking (Fig. 3, SBNDM); for m > 64 its factor
                         // form: the pattern's last 64 bytes scanned, the rest verified
    ALGO_HASHQ = 4,      // hashed q-gram skip filter + verification, any m >= q (Fig. 1, HASHq)
    ALGO_BLOCK = 5,      // 16-byte block fingerprint filter, BF_MIN_M <= m <= BF_MAX_M (after
                         // SSEF, Fig. 1): reads one aligned block per bf_stride(m) text bytes
    ALGO_BRUTE = 6,      // brute force over packed bytes, m <= BRUTE_MAX_M (Fig. 1, BF)
    ALGO_FSBNDM = 7,     // SBNDM with the character after the window read first, m <= 63 (Fig. 3, FSBNDM)
    ALGO_COUNT_ = 8
};
constexpr int BRUTE_MAX_M = 8;

constexpr int BLOCK = 256;         // threads per workgroup (4 wave64)
constexpr int BP_MAX_M = 64;       // bit-parallel state lives in one 64-bit lane register
constexpr int FSBNDM_MAX_M = BP_MAX_M - 1;  // FSBNDM: the pattern and one look-ahead position fit 64 bits
constexpr int SA_SUFFIX = 49;      // Shift-And for m > SA_SUFFIX scans the pattern's last 49 bytes
constexpr int SA_SHORT = 17;       // ... or its last 17 bytes (32-bit state) when no period of the
                                   // pattern lies in (SA_SHORT, SA_SUFFIX]
constexpr int SA_STAGE_MAX = 1024 + SA_SUFFIX;  // its tiles stage whole windows up to this m
constexpr int Q_MAX = 16;          // longest hashed q-gram
constexpr int H_MIN = 8;           // hash table bits range
constexpr int H_MAX = 12;
constexpr int PREP_INLINE = 3072;  // pattern bytes carried in the prep kernel's arguments
constexpr uint32_t PERIOD_MAX = 64;  // periods searched by the prep kernel
constexpr int BF_H = 12;             // block filter: bucket bits of the block hash
constexpr int BF_MIN_M = 144;        // block filter pattern lengths (a tile of 256 blocks then
                                     // holds more starts than one of the widest lanes, 128)
constexpr int BF_MAX_M = 4096;
// Block filter stride: starts owned per sampled block, a multiple of 16 so that every
// sampled block is one aligned 16-byte chunk. The block of start 0 lies up to 15
// bytes early (BF_LEAD), which may take one more tile.
inline uint64_t bf_stride(uint64_t m) { return 16 * ((m - 15) / 16); }
constexpr uint64_t BF_LEAD = 15;

constexpr uint32_t STASH_K = 256;  // hits per tile kept as u16 offsets by the count pass
constexpr uint32_t EMIT_GRID = 4096;  // workgroups of the emit kernel (grid-stride over tiles)
constexpr int EMIT_SUB = 4096;       // starts per sub-tile when a dense tile is rescanned
constexpr uint64_t SCAN_CHUNK = 4096;  // tile counts per workgroup of the tile-count scan (4 per thread)
constexpr int SUPER_SHIFT = 6;        // tiles per super-chunk total: 64
constexpr int SUPER_NZ_SHIFT = 40;    // super-chunk total: (tiles with hits << 40) | hits
constexpr int AUTO_MIN_LANE = 64;    // lane_bytes of the planner's heuristic (no table entry)

// Device-side parameter block at the start of the caller's workspace; the
// pattern follows it (16-byte aligned, zero padded).
struct alignas(16) Params {
    uint32_t m, algo, q, hbits;
    uint32_t sh1;        // Hash-q: shift after a verified window
    uint32_t period;     // smallest period of p if it is <= PERIOD_MAX or p has none (= m); else 0
    uint32_t period_lb;  // lower bound on the smallest period
    uint32_t pad0;
    uint64_t mask[256];          // Shift-And (complemented form) or BNDM masks
    uint8_t shift[1 << H_MAX];   // Hash-q shift per hash bucket (capped at 255)
    // Block filter: the alignments j < m - 15 of the pattern's 16-byte blocks
    // p[j, j + 16), bucketed by the block's hash, each bucket in descending j;
    // bucket h holds bf_js[bf_start[h] .. bf_start[h + 1]).
    uint16_t bf_start[(1 << BF_H) + 1];
    uint16_t bf_js[BF_MAX_M - 15];
};
static_assert(sizeof(Params) % 16 == 0, "Params must keep the pattern 16-byte aligned");

// Host-side plan: everything the launches need that is known on the host.
struct Plan {
    int32_t algo;
    int32_t lane_bytes;   // L: candidate starts per lane; tile = BLOCK * L starts (block
                          // filter: bf_stride(m), the starts of one sampled block)
    int32_t q;            // Hash-q gram length
    int32_t hbits;        // Hash-q table bits
    int32_t tiles_per_wg; // consecutive tiles per workgroup (count kernel)
    int32_t slots;        // find: keep lanes' first hits while counting (tiles expected sparse)
    uint64_t m;
    int32_t sfx = 0;      // Shift-And, m > SA_SUFFIX: the suffix scanned (SA_SUFFIX or SA_SHORT)
};

// A tile with hits, as the tile-count scan lists it for the emit pass.
struct TileEntry {
    uint32_t t;    // tile index
    uint32_t cnt;  // its hits
    uint64_t off;  // hit number of its first hit
};
static_assert(sizeof(TileEntry) == 16, "one 16-byte load per entry");

// Workspace layout (offsets in bytes from the workspace base):
// [Params][pattern][tile_cnt u32][super u64 per 64 tiles][list TileEntry][nlist u64]
// [stash u16 x STASH_K per tile][bits: one bit per start, when the plan keeps hit
// bitmaps: m <= BP_MAX_M, or Shift-And's suffix form]
struct WsLayout {
    uint64_t params, pat, tile_cnt, super, list, nlist, stash, bits;
    uint64_t need;        // minimum workspace size for find_all
    uint64_t need_count;  // minimum workspace size for count (params, pattern, tile_cnt)
    uint64_t ntiles;
};

inline uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

inline uint64_t tile_starts(const Plan &p) { return (uint64_t)BLOCK * (uint64_t)p.lane_bytes; }

inline uint64_t num_tiles(uint64_t n, uint64_t m, uint64_t tile)
{
    if (m == 0 || m > n) return 0;
    return (n - m + 1 + tile - 1) / tile;
}

inline uint64_t num_super(uint64_t ntiles) { return (ntiles + (1ull << SUPER_SHIFT) - 1) >> SUPER_SHIFT; }

// lead: starts before start 0 that the first tile may cover (the block filter's BF_LEAD)
inline WsLayout ws_layout(uint64_t n, uint64_t m, uint64_t tile, bool bitmap, uint64_t lead = 0)
{
    WsLayout w;
    w.ntiles = (m == 0 || m > n) ? 0 : num_tiles(n + lead, m, tile);
    uint64_t o = 0;
    w.params = o;
    o = align_up(o + sizeof(Params), 256);
    w.pat = o;
    o = align_up(o + m + 64, 256);
    w.tile_cnt = o;
    o = align_up(o + 4 * w.ntiles, 256);
    w.super = o;
    o = align_up(o + 8 * num_super(w.ntiles), 256);
    w.need_count = align_up(o, 256);
    w.list = o;
    o = align_up(o + sizeof(TileEntry) * w.ntiles, 256);
    w.nlist = o;
    o = align_up(o + 8, 256);
    w.stash = o;
    o = align_up(o + 2ull * STASH_K * w.ntiles, 256);
    // hit bitmaps of dense Shift-And tiles: tile t at bit t * tile; whatever the
    // tile (at most BLOCK * 128 starts), the last one ends before bit n + BLOCK * 128
    w.bits = 0;
    if ((bitmap || m <= (uint64_t)BP_MAX_M) && w.ntiles) {
        w.bits = o;
        o = align_up(o + (n + (uint64_t)BLOCK * 128) / 8 + 8, 256);
    }
    w.need = o;
    return w;
}

// Device pointers of the find_all workspace.
struct FindWs {
    uint32_t *tile_cnt;
    uint64_t *super;  // per 64 tiles: (tiles with hits << 40) | hits, added by the count pass
    TileEntry *list;
    uint64_t *nlist;
    uint16_t *stash;
    uint32_t *bits;  // null when the layout has no bitmap region
    uint64_t ntiles;
};

// ---------------------------------------------------------------------------
// Batched multi-pattern search (sm_batch.hip / sm_batch.cpp)
// ---------------------------------------------------------------------------
constexpr int BATCH_LANE = 64;           // starts per lane
constexpr int BATCH_MAX_M = 2048;        // longest pattern handled inside a batch launch
constexpr int BATCH_TABLE_BYTES = 32768; // LDS for a group's tables
constexpr int BATCH_GROUP_MAX = 32;      // patterns per group
constexpr int BATCH_HBITS_MAX = 10;      // Hash-q table bits inside a batch (1 KB per pattern)
// Batch write waves. Cost model (seconds, measured on MI355X at n = 2^32): a
// single-pattern search costs one count pass over the text (about 1/6.1e12 s per
// byte, launches included) and 2.7 ps per position for its coalesced emit; one
// prefix-filter write pass of a group costs about 1/0.8e12 s per text byte; a
// position written from a batch pass (the filter's sorted tile lists, or a
// lane-direct store of a pattern's own scanner) costs 40 to 60 ps. So a pattern
// of at most SINGLE_ROUTE_MAX_M bytes with at least one occurrence per
// SINGLE_ROUTE_DENSITY text bytes takes the single-pattern pipeline (break-even
// near one per 300 to 400 bytes).
constexpr uint32_t SINGLE_ROUTE_MAX_M = 64;
constexpr double SINGLE_ROUTE_DENSITY = 384.0;
constexpr double SINGLE_COST_PER_BYTE = 1.0 / 6.1e12;
constexpr double SINGLE_COST_PER_POS = 8.0 / 3.0e12;
constexpr double FILTER_COST_PER_BYTE = 1.0 / 0.8e12;

// Multi-pattern prefix filter of the batched count pass. The patterns of one
// q-class (q = min(m, MQ_QMAX)) are cut into groups of at most MQ_G. A group keeps
// a bitmap over MQ_H-bit hashes of its patterns' first q bytes; a set bit leads
// (through the bucket's rank) to the slots of the distinct q-byte prefixes with
// that hash, and a slot to its patterns. Patterns with m == q are counted once
// per slot; longer ones are checked on bytes [q, q + 8) from a per-pattern copy
// and beyond that against the pattern itself.
constexpr int MQ_H = 16;                    // hash bits (bitmap of 2^16 bits)
constexpr int MQ_WORDS = 1 << (MQ_H - 5);   // bitmap words
constexpr int MQ_G = 1024;                  // patterns per group
constexpr int MQ_QMAX = 8;                  // longest prefix gram (two 32-bit words)
constexpr int MQ_MIN = 3;                   // smallest q-class sent to the filter
constexpr uint32_t MQ_NONE = 0xFFFF;
// The filter's count pass keeps the hits of each (chunk, group) item -- counter id
// << MQ_REL_BITS | start relative to the chunk -- of every counter with at most
// MQ_CAP hits in the chunk, MQ_STASH entries per item at most, so that the write
// pass copies them out instead of scanning the chunk again. A pattern is served
// from the stash in a chunk when the item kept its entries (stash_n <= MQ_STASH)
// and its count there is at most MQ_CAP.
constexpr uint32_t MQ_STASH = 4096;
constexpr uint32_t MQ_CAP = 64;
constexpr int MQ_REL_BITS = 22;  // a chunk is at most 256 tiles of BLOCK * BATCH_LANE starts

// Table of one group (byte offsets; the part below MQ_LDS_BYTES is staged in LDS).
constexpr uint32_t MQ_OFF_BITS = 0;                                // u32[MQ_WORDS]
constexpr uint32_t MQ_OFF_RANK = MQ_OFF_BITS + 4 * MQ_WORDS;       // u16[MQ_WORDS]: set bits before the word
constexpr uint32_t MQ_OFF_BSTART = MQ_OFF_RANK + 2 * MQ_WORDS;     // u16[MQ_G + 8]: bucket -> first slot
constexpr uint32_t MQ_OFF_SPRE = MQ_OFF_BSTART + 2 * (MQ_G + 8);   // uint2[MQ_G]: slot prefix (q bytes)
constexpr uint32_t MQ_OFF_SSTART = MQ_OFF_SPRE + 8 * MQ_G;         // u16[MQ_G + 8]: slot -> first long pattern
constexpr uint32_t MQ_OFF_SREP = MQ_OFF_SSTART + 2 * (MQ_G + 8);   // u16[MQ_G]: slot's counter for m == q, or MQ_NONE
constexpr uint32_t MQ_OFF_PID = MQ_OFF_SREP + 2 * MQ_G;            // u16[MQ_G]: patterns with m > q, by slot
constexpr uint32_t MQ_OFF_M = MQ_OFF_PID + 2 * MQ_G;               // u16[MQ_G]: lengths
constexpr uint32_t MQ_OFF_PRE2 = MQ_OFF_M + 2 * MQ_G;              // uint2[MQ_G]: bytes [q, q + 8) (masked)
constexpr uint32_t MQ_LDS_BYTES = MQ_OFF_PRE2 + 8 * MQ_G;
constexpr uint32_t MQ_OFF_SPI = MQ_LDS_BYTES;                      // u32[MQ_G]: sorted pattern index
constexpr uint32_t MQ_OFF_POFF = MQ_OFF_SPI + 4 * MQ_G;            // u32[MQ_G]: byte offset of the pattern
constexpr uint32_t MQ_OFF_CID = MQ_OFF_POFF + 4 * MQ_G;            // u16[MQ_G]: counter holding its count
constexpr uint32_t MQ_TAB_BYTES = MQ_OFF_CID + 2 * MQ_G;

struct MqGroup {
    uint32_t count, q, min_m, max_m;
    uint32_t flat;     // every pattern has m == q and every bucket holds one slot
    uint32_t pad;
    uint64_t tab_off;  // byte offset of the group's table
};

// Hash of a q-gram packed little-endian into (lo, hi) with the bytes past q
// zero. q <= 2 keys are used directly (exact); longer ones are hashed. Host and
// device use the same functions.
__host__ __device__ inline uint32_t mq_hash(uint32_t lo, uint32_t hi)
{
    return ((lo * 0x9E3779B1u) ^ (hi * 0x85EBCA77u)) >> (32 - MQ_H);
}
__host__ __device__ inline uint32_t mq_key(uint32_t lo, uint32_t hi, uint32_t q)
{
    return q <= 2 ? lo : mq_hash(lo, hi);
}

struct BatchPat {      // one pattern, in the batch's sorted order
    uint64_t pat_off;  // offset of its bytes in the device pattern buffer (16-byte aligned)
    uint32_t m, algo, var, q, hbits;
    uint32_t index;    // position in the caller's list
};

struct BatchGroup {    // consecutive sorted patterns that share a kernel variant
    uint32_t first, count, algo, var, max_m, pad;
};

struct BatchLaunch {
    const uint8_t *text;
    uint64_t n;
    const BatchPat *pats;
    const BatchGroup *groups;       // write pass: every pattern
    const BatchGroup *host_groups;
    const BatchGroup *cgroups;      // count pass, per-pattern scanners (patterns outside the filter)
    const BatchGroup *host_cgroups;
    uint32_t ncgroups;
    const MqGroup *mqgroups;        // count pass, prefix filter (ordered by q)
    const MqGroup *host_mq;
    // write pass, prefix filter: the count groups listed in mqwlist (ascending, so
    // the q <= 2 groups come first), with their write tables (every pattern listed
    // with its slot), for the patterns with wroute[sorted] == 2
    const uint8_t *mqwtabs;
    const uint32_t *mqwlist;
    const uint32_t *host_mqwlist;
    uint32_t nmqw;
    const uint8_t *wroute;
    // write pass, filter pass over the text for the window's route-4 patterns
    const MqGroup *hqgroups;
    const MqGroup *host_hq;
    const uint8_t *hqtabs;
    uint32_t nhq;
    uint32_t *mqstash;              // [chunk][group] MQ_STASH hits each (count pass writes)
    uint32_t *mqstash_n;            // [chunk][group] hits (more than MQ_STASH: not kept)
    const uint8_t *mqtabs;
    uint32_t nmq, mq_max_m;
    const Params *params;
    const uint8_t *patbytes;
    uint32_t npats;        // patterns in this launch set (sorted)
    uint32_t npats_total;  // entries of totals / csr (caller's P)
    uint32_t ngroups;
    uint32_t chunk_tiles;
    uint64_t nchunks, ntiles;
    uint32_t *cnt;
    const uint64_t *chunk_off;  // write: per (pattern, chunk) offsets
    uint64_t *chunk_off_out;    // count: where the segmented scan writes them (may be null)
    uint64_t *totals;           // count: per original index
    uint64_t *csr_out;          // count: exclusive scan of totals, P + 1 entries (may be null)
    const uint64_t *csr;        // write: CSR offsets by original index
    int64_t *out;               // write: CSR entry k goes to out[k - lo]
    uint64_t lo, span;          // write: window [lo, lo + span) of CSR entries
    bool write, prep;
};
hipError_t launch_batch(const BatchLaunch &L, hipStream_t stream);

// Kernel timing of batched count passes (sm_prof_*): while recording is on, every
// count pass of launch_batch that is not being captured into a graph records
// events at its start (e0), around its shared-filter launches (e1, e2) and at its
// end (e3).
struct BatchProfRec {
    hipEvent_t e0, e1, e2, e3;
    uint64_t filter_pattern_bytes;  // n x patterns in the filter groups
    uint32_t filter_launches;
};
// true: the events are created and e0 is recorded on st
bool prof_batch_begin(hipStream_t st, BatchProfRec &r);
// hands a finished record (e3 recorded) to sm_prof_collect
void prof_batch_push(const BatchProfRec &r);
// destroys the events of a record that will not be finished
void prof_batch_discard(BatchProfRec &r);
// csr[0..P] = exclusive scan of totals[0..P)
hipError_t launch_csr_scan(const uint64_t *totals, uint64_t P, uint64_t *csr, hipStream_t stream);

}  // namespace sm

// A device-resident text (see sm_corpus_open).
struct sm_corpus {
    const uint8_t *d_text = nullptr;
    uint64_t n = 0;
    bool owned = false;
    uint64_t hist[256];
    int32_t sigma = 0;        // distinct bytes
    double sigma_eff = 0;     // 1 / sum_c p_c^2: alphabet size with the same collision rate
    int dev = 0;
};

namespace sm {
// The corpus's sigma_eff rounded to [1, 256] (planner input).
int corpus_sigma(const sm_corpus *c);

// Single-pattern find_all of hit numbers [first, first + cap) into d_out[0 ..)
// (a window of the sorted list); total -> *d_count.
int corpus_find_window_async(sm_corpus *c, const uint8_t *pat, uint64_t m, int64_t *d_out,
                             uint64_t first, uint64_t cap, uint64_t *d_count, void *d_work,
                             uint64_t work_bytes, hipStream_t stream);

// Plan one pattern as the single-pattern path would (sigma from the corpus), or
// with explicit options.
int plan_pattern(const uint8_t *pat, uint64_t m, int sigma, Plan &p);
int plan_pattern_opts(const uint8_t *pat, uint64_t m, const ::sm_opts *o, Plan &p);
const char *sm_set_error(int status, const char *msg);

// Kernel launchers (sm_kernels.hip). All are asynchronous on `stream` and
// return the HIP error of the launch.
// Builds the pattern's tables in d_params; zeroes *d_zero when not null, and the
// nsuper super-chunk totals at d_super.
hipError_t launch_prep(const Plan &plan, const uint8_t *pat_host, Params *d_params,
                       uint8_t *d_pat, uint64_t *d_zero, uint64_t *d_super, uint64_t nsuper,
                       hipStream_t stream);
// count -> sum: total -> *d_total (uses w.tile_cnt only).
// `after_count` (may be null) is recorded after the count kernel.
hipError_t launch_count(const Plan &plan, const uint8_t *d_text, uint64_t n,
                        const Params *d_params, const uint8_t *d_pat, const FindWs &w,
                        uint64_t *d_total, hipStream_t stream, hipEvent_t after_count);
// count -> scan -> emit: hit numbers [first, first + cap) -> d_out[0 .. ), total -> *d_total.
// `after_count` (may be null) is recorded after the count kernel.
hipError_t launch_find(const Plan &plan, const uint8_t *d_text, uint64_t n, const Params *d_params,
                       const uint8_t *d_pat, const FindWs &w, int64_t *d_out, uint64_t first,
                       uint64_t cap, uint64_t *d_total, hipStream_t stream, hipEvent_t after_count);
hipError_t launch_set_u64(uint64_t *d_dst, uint64_t value, hipStream_t stream);
hipError_t launch_histogram(const uint8_t *d_text, uint64_t n, uint64_t *d_hist256,
                            hipStream_t stream);

}  // namespace sm
