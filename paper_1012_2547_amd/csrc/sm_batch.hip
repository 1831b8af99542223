// Batched multi-pattern search: P patterns against one resident text.
//
// The paper's experiments search one pattern at a time (Section 2); serving many
// patterns over the same text on a GPU wants the text read once for many
// patterns instead. Patterns are sorted by kernel variant (algorithm, state width
// or q-gram words) and length, and cut into groups whose tables fit a fixed LDS
// budget. A work item is (text chunk, group): one workgroup loads the group's
// tables into LDS once, then streams the chunk's tiles through LDS and runs every
// pattern of the group over each staged tile with the same per-lane scanners as
// the single-pattern path. Items are ordered chunk-major, so the groups of a
// chunk run close together and the chunk is served from L2 / Infinity Cache
// after its first read.
//
// Counting writes one count per (pattern, chunk); a segmented scan gives each
// pattern its total and per-chunk offsets; the write pass re-runs the items that
// have hits and writes each pattern's positions into its CSR slice in order.
#include <hip/hip_runtime.h>

#include <cstring>

#include "sm_internal.h"
#include "sm_device.h"

namespace sm {
namespace {
using namespace dev;

constexpr int BL = BATCH_LANE;                 // starts per lane
constexpr int BT = BLOCK * BATCH_LANE;         // starts per tile
// staged bytes: tile + halo of the group's longest pattern + misalignment + word reads
constexpr int B_CHUNKS = (((BT + BATCH_MAX_M + 48 + 15) / 16 + 1) + 7) & ~7;
constexpr int B_PER = (B_CHUNKS + BLOCK - 1) / BLOCK;

struct PatInfo {
    uint32_t m, q, hbits, sh1, period, period_lb;
    uint64_t pat_off;
};

struct BatchArgs {
    const uint8_t *text;
    uint64_t n;
    const BatchPat *pats;      // sorted order
    const BatchGroup *groups;
    const Params *params;      // per sorted pattern
    const uint8_t *patbytes;
    uint32_t group_lo, ngroups;  // groups handled by this launch
    uint32_t chunk_tiles;
    uint64_t nchunks, ntiles;
    uint32_t *cnt;             // [sorted pattern][chunk]
    const uint64_t *chunk_off; // [sorted pattern][chunk] (write)
    const uint64_t *csr;       // [original index] (write)
    int64_t *out;              // write: CSR entry k goes to out[k - lo]
    uint64_t lo, span;         // write: window [lo, lo + span) of CSR entries
};

template <int ALGO, int VAR>
struct BatchShared {
    uint4 text[B_CHUNKS];
    uint64_t tab[BATCH_TABLE_BYTES / 8];
    PatInfo info[BATCH_GROUP_MAX];
    uint32_t acc[BATCH_GROUP_MAX];
    uint64_t run[BATCH_GROUP_MAX];
    uint32_t w[BLOCK / 64];
};

// bytes of one pattern's table in LDS
template <int ALGO, int VAR>
__host__ __device__ __forceinline__ constexpr int tab_bytes()
{
    return ALGO == ALGO_HASHQ ? (1 << BATCH_HBITS_MAX) : ((ALGO == ALGO_SHIFT_AND && VAR == 0) ? 1024 : 2048);
}

template <int ALGO, int VAR>
__device__ __forceinline__ void load_group_tables(BatchShared<ALGO, VAR> &S, const BatchArgs &a,
                                                  const BatchGroup &g)
{
    constexpr int TB = tab_bytes<ALGO, VAR>();
    const int tid = threadIdx.x;
    for (uint32_t j = 0; j < g.count; j++) {
        const Params *P = a.params + g.first + j;
        uint8_t *dst = reinterpret_cast<uint8_t *>(S.tab) + j * TB;
        if (ALGO == ALGO_HASHQ) {
            const uint32_t nb = 1u << a.pats[g.first + j].hbits;
            for (uint32_t k = tid; k < nb / 16; k += BLOCK)
                reinterpret_cast<uint4 *>(dst)[k] = reinterpret_cast<const uint4 *>(P->shift)[k];
        } else if (ALGO == ALGO_SHIFT_AND && VAR == 0) {
            reinterpret_cast<uint32_t *>(dst)[tid] = (uint32_t)P->mask[tid];
        } else {
            reinterpret_cast<uint64_t *>(dst)[tid] = P->mask[tid];
        }
    }
    if (tid < (int)g.count) {
        const BatchPat &bp = a.pats[g.first + tid];
        const Params *P = a.params + g.first + tid;
        PatInfo in;
        in.m = bp.m;
        in.q = bp.q;
        in.hbits = bp.hbits;
        in.sh1 = P->sh1;
        in.period = P->period;
        in.period_lb = P->period_lb;
        in.pat_off = bp.pat_off;
        S.info[tid] = in;
        S.acc[tid] = 0;
    }
}

// Scan pattern j of the group over the staged tile (all threads call it).
template <int ALGO, int VAR, bool WRITE, class E>
__device__ __forceinline__ uint32_t batch_lane(BatchShared<ALGO, VAR> &S, const BatchArgs &a, int j,
                                               uint64_t s, int boff, int lo, int hi, E &o)
{
    constexpr int TB = tab_bytes<ALGO, VAR>();
    const PatInfo in = S.info[j];
    const int m = (int)in.m;
    const uint8_t *tab = reinterpret_cast<const uint8_t *>(S.tab) + j * TB;
    if (ALGO == ALGO_SHIFT_AND) {
        if (lo > hi) return 0u;
        if (VAR == 0)
            return lane_shift_and<uint32_t, 16, WRITE>(S.text, reinterpret_cast<const uint32_t *>(tab), m,
                                                       boff, lo, hi, o);
        if (VAR == 1)
            return lane_shift_and<uint64_t, 16, WRITE>(S.text, reinterpret_cast<const uint64_t *>(tab), m,
                                                       boff, lo, hi, o);
        if (VAR == 2)
            return lane_shift_and<uint64_t, 4, WRITE>(S.text, reinterpret_cast<const uint64_t *>(tab), m,
                                                      boff, lo, hi, o);
        return lane_shift_and<uint64_t, 1, WRITE>(S.text, reinterpret_cast<const uint64_t *>(tab), m,
                                                  boff, lo, hi, o);
    } else if (ALGO == ALGO_BNDM) {
        if (lo > hi) return 0u;
        return lane_bndm<1, WRITE>(reinterpret_cast<const uint8_t *>(S.text),
                                reinterpret_cast<const uint64_t *>(tab), m, boff, lo, hi, o);
    } else if (ALGO == ALGO_SBNDM) {
        if (lo > hi) return 0u;
        return lane_sbndm<1, WRITE>(reinterpret_cast<const uint8_t *>(S.text),
                                 reinterpret_cast<const uint64_t *>(tab), m, (int)in.period, boff, lo,
                                 hi, o);
    } else {
        // wave-cooperative: every lane takes part, lanes without starts have lo > hi
        return lane_hashq<VAR, WRITE>(reinterpret_cast<const uint32_t *>(S.text), tab, m, (int)in.q,
                                      (int)in.hbits, (int)in.sh1, (int)in.period, (int)in.period_lb,
                                      boff, lo, hi, a.text, s, a.patbytes + in.pat_off, o);
    }
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// Stage tile t: text positions [s, s + BT + max_m - 1) clipped to n.
template <int ALGO, int VAR>
__device__ __forceinline__ int batch_stage(BatchShared<ALGO, VAR> &S, const BatchArgs &a, uint64_t s,
                                           uint32_t max_m)
{
    uint64_t x1 = s + (uint64_t)BT + max_m - 1;
    if (x1 > a.n) x1 = a.n;
    Staged<B_PER> st;
    stage_issue(st, a.text, s, x1);
    stage_commit<ALGO == ALGO_SHIFT_AND>(st, S.text);
    return st.boff;
}

template <int ALGO, int VAR, bool WRITE>
__global__ __launch_bounds__(BLOCK) void batch_kernel(BatchArgs a)
{
    __shared__ BatchShared<ALGO, VAR> S;
    const uint64_t item = blockIdx.x;
    const uint64_t chunk = item / a.ngroups;
    const BatchGroup g = a.groups[a.group_lo + item % a.ngroups];
    const int tid = threadIdx.x;

    const uint64_t wend = a.lo + a.span;
    if (WRITE) {  // skip items without hits in the window (uniform: all threads read the same)
        bool any = false;
        for (uint32_t j = 0; j < g.count; j++) {
            const uint64_t sp = g.first + j;
            const uint32_t c = a.cnt[sp * a.nchunks + chunk];
            if (c == 0) continue;
            const uint64_t r0 = a.csr[a.pats[sp].index] + a.chunk_off[sp * a.nchunks + chunk];
            any |= r0 < wend && r0 + c > a.lo;
        }
        if (!any) return;
    }
    load_group_tables<ALGO, VAR>(S, a, g);
    if (WRITE && tid < (int)g.count) {
        const uint64_t sp = g.first + tid;
        const uint32_t c = a.cnt[sp * a.nchunks + chunk];
        const uint64_t r0 = a.csr[a.pats[sp].index] + a.chunk_off[sp * a.nchunks + chunk];
        S.acc[tid] = (r0 < wend && r0 + c > a.lo) ? c : 0u;  // nonzero: hits in the window
        S.run[tid] = r0;
    }
    const uint64_t t0 = chunk * a.chunk_tiles;
    uint64_t t1 = t0 + a.chunk_tiles;
    if (t1 > a.ntiles) t1 = a.ntiles;
    for (uint64_t t = t0; t < t1; t++) {
        const uint64_t s = t * (uint64_t)BT;
        __syncthreads();  // previous tile's readers are done; tables and info visible
        const int boff = batch_stage<ALGO, VAR>(S, a, s, g.max_m);
        __syncthreads();
        for (uint32_t j = 0; j < g.count; j++) {
            const uint64_t m = S.info[j].m;
            if (m > a.n || s > a.n - m) continue;  // no start of this pattern in the tile
            if (WRITE && S.acc[j] == 0) continue;  // no hit of this pattern in the chunk
            const uint64_t lim = a.n - m - s;
            const int hi_rel = lim >= (uint64_t)(BT - 1) ? BT - 1 : (int)lim;
            const int lo = tid * BL;
            const int hi = (lo + BL - 1) < hi_rel ? (lo + BL - 1) : hi_rel;
            NoEmit ne;
            const uint32_t c = batch_lane<ALGO, VAR, false>(S, a, (int)j, s, boff, lo, hi, ne);
            if (!WRITE) {
                const uint32_t wsum = wave_sum(c);
                if ((tid & 63) == 0 && wsum) atomicAdd(&S.acc[j], wsum);
            } else {
                uint32_t tot;
                const uint32_t before = block_excl_scan(c, S.w, tot);
                if (tot) {  // uniform
                    const uint64_t r0 = S.run[j];
                    if (r0 < wend && r0 + tot > a.lo) {
                        PosEmit pe;
                        pe.out = a.out;
                        pe.lo = a.lo;
                        pe.span = a.span;
                        pe.base = s;
                        pe.idx = r0 + before;
                        batch_lane<ALGO, VAR, true>(S, a, (int)j, s, boff, lo, hi, pe);
                    }
                    __syncthreads();
                    if (tid == 0) {
                        S.run[j] = r0 + tot;
                        if (r0 + tot >= wend) S.acc[j] = 0;  // the rest of the chunk is past the window
                    }
                }
            }
        }
    }
    if (!WRITE) {
        __syncthreads();
        if (tid < (int)g.count) a.cnt[(uint64_t)(g.first + tid) * a.nchunks + chunk] = S.acc[tid];
    }
}

// ---------------------------------------------------------------------------
// Prefix filter count pass: one work item = (text chunk, filter group).
// ---------------------------------------------------------------------------
struct MqArgs {
    const uint8_t *text;
    uint64_t n;
    const MqGroup *groups;
    const uint8_t *tabs;
    const uint8_t *patbytes;
    uint32_t ngroups, chunk_tiles;
    uint64_t nchunks, ntiles;
    uint32_t *cnt;             // [sorted pattern][chunk]
    // count pass: the hits of each (chunk, group) item, group index group_base + the
    // launch's group, nmq groups in all (null: not kept)
    uint32_t *stash, *stash_n;
    uint32_t group_base, nmq;
};
static_assert(256 * BT <= (1 << MQ_REL_BITS), "a chunk's relative starts fit MQ_REL_BITS");
static_assert(MQ_G <= (1 << (32 - MQ_REL_BITS)), "counter ids fit above the relative start");

// The filter's count pass scans each tile in MQ_SUB sub-tiles of MQ_BT starts: it reads
// at most 20 bytes past a start from LDS (the q-gram key, then bytes [q, q + 8) of a
// candidate; longer patterns are checked from global memory), so a sub-tile stages
// MQ_BT + 32 bytes, and the smaller LDS tile lets three workgroups share a CU (two
// with whole tiles).
constexpr int MQ_SUB = 2;
constexpr int MQ_BT = BT / MQ_SUB, MQ_BL = BL / MQ_SUB;
constexpr int MQ_STAGE = MQ_BT + 32;
constexpr int MQ_CHUNKS = (((MQ_STAGE + 15) / 16 + 1) + 7) & ~7;
constexpr int MQ_PER = (MQ_CHUNKS + BLOCK - 1) / BLOCK;

struct MqShared {
    uint4 text[MQ_CHUNKS];
    uint4 tab[MQ_LDS_BYTES / 16];
    uint32_t acc[MQ_G];
    uint32_t nst;  // hits of the item so far (the stash keeps the first MQ_STASH)
};

// k entries of this lane for the item's stash: the index of the first, or
// MQ_STASH when the item already holds more than MQ_STASH (then it is not kept;
// the count goes on only until then, so the counter stays small)
__device__ __forceinline__ uint32_t mq_stash_take(MqShared &S, uint32_t k)
{
    if (k == 0 || *(volatile uint32_t *)&S.nst > MQ_STASH) return MQ_STASH;
    return atomicAdd(&S.nst, k);
}

// Word k (bytes [4k, 4k + 4)) of the swizzled LDS tile.
__device__ __forceinline__ uint32_t tile_word(const uint4 *text, uint32_t k)
{
    return reinterpret_cast<const uint32_t *>(text)[4 * swz(k >> 2) + (k & 3)];
}

// A start whose q-gram hash bit is set: the slots of its bucket whose prefix
// equals the key (lo, hi) are taken. A slot's m == q patterns (when the table
// keeps them apart) go to one counter, on_slot(rep); every other pattern j of the
// slot is checked on bytes [q, q + 8) from its copy in the table and beyond that
// against the pattern in global memory, then on_hit(j).
// text/T: the LDS tile and table; x: LDS byte index of the start; g: its global position.
template <class OnSlot, class OnHit>
__device__ __forceinline__ void mq_slots(const uint4 *text, const uint8_t *T, const MqArgs &a,
                                         const uint32_t *poff, uint32_t h, uint32_t wbits, uint32_t lo,
                                         uint32_t hi, uint32_t x, uint64_t g, uint32_t q, OnSlot on_slot,
                                         OnHit on_hit)
{
    const uint16_t *rank = reinterpret_cast<const uint16_t *>(T + MQ_OFF_RANK);
    const uint16_t *bstart = reinterpret_cast<const uint16_t *>(T + MQ_OFF_BSTART);
    const uint2 *spre = reinterpret_cast<const uint2 *>(T + MQ_OFF_SPRE);
    const uint16_t *sstart = reinterpret_cast<const uint16_t *>(T + MQ_OFF_SSTART);
    const uint16_t *srep = reinterpret_cast<const uint16_t *>(T + MQ_OFF_SREP);
    const uint16_t *pid = reinterpret_cast<const uint16_t *>(T + MQ_OFF_PID);
    const uint16_t *m16 = reinterpret_cast<const uint16_t *>(T + MQ_OFF_M);
    const uint2 *pre2 = reinterpret_cast<const uint2 *>(T + MQ_OFF_PRE2);
    const uint32_t k = (uint32_t)rank[h >> 5] + (uint32_t)__builtin_popcount(wbits & ((1u << (h & 31)) - 1u));
    const uint32_t s1 = bstart[k + 1];
    for (uint32_t sl = bstart[k]; sl < s1; sl++) {
        const uint2 p = spre[sl];
        if ((p.x ^ lo) | (p.y ^ hi)) continue;
        const uint32_t rep = srep[sl];
        if (rep != MQ_NONE) on_slot(rep);  // the slot's patterns with m == q
        const uint32_t e1 = sstart[sl + 1];
        if (sstart[sl] == e1) continue;
        // bytes [q, q + 8) of the text at this start, from the tile
        const uint32_t y = x + q, wi = y >> 2, sb = y & 3;
        const uint32_t w0 = tile_word(text, wi), w1 = tile_word(text, wi + 1), w2 = tile_word(text, wi + 2);
        const uint32_t t0 = alignbyte(w1, w0, sb), t1 = alignbyte(w2, w1, sb);
        for (uint32_t e = sstart[sl]; e < e1; e++) {
            const uint32_t j = pid[e];
            const uint32_t m = m16[j];
            if (g + m > a.n) continue;
            const uint32_t nb = m - q < 8 ? m - q : 8;
            const uint2 p2 = pre2[j];
            if (((t0 ^ p2.x) & byte_mask(nb < 4 ? (int)nb : 4)) | ((t1 ^ p2.y) & byte_mask(nb > 4 ? (int)nb - 4 : 0)))
                continue;
            bool ok = true;
            if (m > q + 8) {  // the rest of the pattern, 16 bytes at a time, from global memory
                const uint8_t *pat = a.patbytes + poff[j];
                const uint8_t *tl = a.text + g + m - 1, *pl = pat + m + 15;
                for (uint32_t off = q + 8; off < m && ok; off += 16)
                    ok = diff16(load16(a.text + g + off, tl), load16(pat + off, pl), m - off < 16 ? m - off : 16) == 0;
            }
            if (ok) on_hit(j);
        }
    }
}

// The 16 starts of LDS chunk u: their q-gram hashes and bitmap words, and the
// mask of starts whose hash bit is set.
template <bool EXACT>
__device__ __forceinline__ uint32_t mq_filter16(const uint4 cu, const uint4 nx, const uint32_t *bits,
                                                uint32_t mlo, uint32_t mhi, uint32_t *hh, uint32_t *wb)
{
    const uint32_t W[8] = {cu.x, cu.y, cu.z, cu.w, nx.x, nx.y, nx.z, nx.w};
#pragma unroll
    for (int b = 0; b < 16; b++) {
        const int i = b >> 2, sh = b & 3;
        const uint32_t klo = (sh ? alignbyte(W[i + 1], W[i], sh) : W[i]) & mlo;
        const uint32_t khi = EXACT ? 0u : ((sh ? alignbyte(W[i + 2], W[i + 1], sh) : W[i + 1]) & mhi);
        hh[b] = EXACT ? klo : mq_hash(klo, khi);
        wb[b] = bits[hh[b] >> 5];
    }
    uint32_t cm = 0;
#pragma unroll
    for (int b = 0; b < 16; b++) cm |= __builtin_amdgcn_ubfe(wb[b], hh[b] & 31, 1) << b;
    return cm;
}

// The key of the start at LDS byte index x, read again from the tile.
template <bool EXACT>
__device__ __forceinline__ void mq_key_at(const uint4 *text, uint32_t x, uint32_t mlo, uint32_t mhi,
                                          uint32_t &klo, uint32_t &khi, uint32_t &h)
{
    const uint32_t wi = x >> 2, sb = x & 3;
    const uint32_t w0 = tile_word(text, wi), w1 = tile_word(text, wi + 1);
    klo = alignbyte(w1, w0, sb) & mlo;
    khi = EXACT ? 0u : (alignbyte(tile_word(text, wi + 2), w1, sb) & mhi);
    h = EXACT ? klo : mq_hash(klo, khi);
}

// EXACT: q <= 2, the key itself indexes the bitmap.
template <bool EXACT>
__global__ __launch_bounds__(BLOCK) void mq_count_kernel(MqArgs a)
{
    __shared__ MqShared S;
    const uint64_t item = blockIdx.x;
    const uint64_t chunk = item / a.ngroups;
    const MqGroup g = a.groups[item % a.ngroups];
    const int tid = threadIdx.x;
    const uint8_t *tab = a.tabs + g.tab_off;
    {   // the group's table (bitmap, ranks, buckets, slots, prefixes, lengths) and counters
        const uint4 *src = reinterpret_cast<const uint4 *>(tab);
        for (uint32_t k = tid; k < MQ_LDS_BYTES / 16; k += BLOCK) S.tab[k] = src[k];
        for (uint32_t k = tid; k < g.count; k += BLOCK) S.acc[k] = 0;
        if (tid == 0) S.nst = 0;
    }
    const uint32_t *poff = reinterpret_cast<const uint32_t *>(tab + MQ_OFF_POFF);
    const uint32_t *bits = reinterpret_cast<const uint32_t *>(S.tab);
    const uint32_t q = g.q;
    const uint32_t mlo = byte_mask(q < 4 ? (int)q : 4), mhi = byte_mask(q > 4 ? (int)q - 4 : 0);
    const uint64_t sitem = chunk * a.nmq + a.group_base + item % a.ngroups;
    uint32_t *stash = a.stash ? a.stash + sitem * MQ_STASH : nullptr;
    // the chunk's sub-tiles (MQ_BT starts each); its first start is c0
    const uint64_t c0 = chunk * a.chunk_tiles * (uint64_t)BT;
    const uint64_t t0 = chunk * a.chunk_tiles * MQ_SUB;
    uint64_t t1 = t0 + a.chunk_tiles * MQ_SUB;
    if (t1 > a.ntiles * MQ_SUB) t1 = a.ntiles * MQ_SUB;
    // sub-tiles with a start of some pattern of the group: s + min_m <= n
    const uint64_t tl = a.n >= g.min_m ? (a.n - g.min_m) / MQ_BT + 1 : 0;
    if (t1 > tl) t1 = tl;
    Staged<MQ_PER> st;
    if (t0 < t1) {
        const uint64_t x1 = t0 * (uint64_t)MQ_BT + MQ_STAGE;
        stage_issue(st, a.text, t0 * (uint64_t)MQ_BT, x1 < a.n ? x1 : a.n);
    }
    for (uint64_t t = t0; t < t1; t++) {
        const uint64_t s = t * (uint64_t)MQ_BT;
        __syncthreads();  // previous sub-tile's readers are done; tables visible
        stage_commit<true>(st, S.text);
        const int boff = st.boff;
        __syncthreads();
        if (t + 1 < t1) {  // next sub-tile's loads fly while this one is scanned
            const uint64_t s2 = s + (uint64_t)MQ_BT;
            const uint64_t x1 = s2 + MQ_STAGE;
            stage_issue(st, a.text, s2, x1 < a.n ? x1 : a.n);
        }
        const uint64_t lim = a.n - g.min_m - s;  // largest relative start of the group
        const int hi_rel = lim >= (uint64_t)(MQ_BT - 1) ? MQ_BT - 1 : (int)lim;
        const int lo = tid * MQ_BL;
        const int hi = (lo + MQ_BL - 1) < hi_rel ? (lo + MQ_BL - 1) : hi_rel;
        if (lo > hi) continue;
        const int u0 = (boff + lo) >> 4, u1 = (boff + hi) >> 4;
        uint4 nx = S.text[swz((uint32_t)u0)];
        for (int u = u0; u <= u1; u++) {
            const uint4 cu = nx;
            nx = S.text[swz((uint32_t)(u + 1))];
            uint32_t hh[16], wb[16];
            uint32_t cm = mq_filter16<EXACT>(cu, nx, bits, mlo, mhi, hh, wb);
            const int r0 = 16 * u - boff;  // relative start of byte 0 of this chunk
            if (g.flat && __ballot(__builtin_popcount(cm) >= 4)) {
                // dense candidates in a flat group: bucket = slot, all 16 starts'
                // lookups at once; a start counts when its bit is set, it lies in the
                // lane's range and its key equals the slot's prefix
                const uint8_t *T = reinterpret_cast<const uint8_t *>(S.tab);
                const uint16_t *rank = reinterpret_cast<const uint16_t *>(T + MQ_OFF_RANK);
                const uint2 *spre = reinterpret_cast<const uint2 *>(T + MQ_OFF_SPRE);
                const uint16_t *srep = reinterpret_cast<const uint16_t *>(T + MQ_OFF_SREP);
                const uint32_t W[8] = {cu.x, cu.y, cu.z, cu.w, nx.x, nx.y, nx.z, nx.w};
                uint32_t kk[16];
#pragma unroll
                for (int b = 0; b < 16; b++) {
                    const int r = r0 + b;
                    if (r < lo || r > hi) cm &= ~(1u << b);
                    const uint32_t below = wb[b] & ((1u << (hh[b] & 31)) - 1u);
                    kk[b] = ((cm >> b) & 1u) ? (uint32_t)rank[hh[b] >> 5] + (uint32_t)__builtin_popcount(below) : 0u;
                }
                uint32_t hm = 0;  // starts of this unit whose hit is kept
                uint32_t rp[16];
#pragma unroll
                for (int b = 0; b < 16; b++) {
                    const int i = b >> 2, sh = b & 3;
                    const uint32_t klo = (sh ? alignbyte(W[i + 1], W[i], sh) : W[i]) & mlo;
                    const uint32_t khi = EXACT ? 0u : ((sh ? alignbyte(W[i + 2], W[i + 1], sh) : W[i + 1]) & mhi);
                    const uint2 p = spre[kk[b]];
                    rp[b] = srep[kk[b]];
                    if (((cm >> b) & 1u) && !((p.x ^ klo) | (p.y ^ khi))) {
                        if (atomicAdd(&S.acc[rp[b]], 1u) < MQ_CAP) hm |= 1u << b;
                    }
                }
                if (stash && hm) {
                    uint32_t at = mq_stash_take(S, (uint32_t)__builtin_popcount(hm));
                    const uint32_t rel0 = (uint32_t)(s - c0) + (uint32_t)r0;
#pragma unroll
                    for (int b = 0; b < 16; b++)
                        if ((hm >> b) & 1u) {
                            if (at < MQ_STASH) stash[at] = (rp[b] << MQ_REL_BITS) | (rel0 + (uint32_t)b);
                            at++;
                        }
                }
                continue;
            }
            // this lane's candidates, one per iteration (a wave iterates as often as
            // its busiest lane); the key is read again from the tile
            while (cm) {
                const int b = __builtin_ctz(cm);
                cm &= cm - 1;
                const int r = r0 + b;
                if (r < lo || r > hi) continue;
                const uint32_t x = (uint32_t)(16 * u + b);
                uint32_t klo, khi, h;
                mq_key_at<EXACT>(S.text, x, mlo, mhi, klo, khi, h);
                const uint32_t rel = (uint32_t)(s - c0) + (uint32_t)r;
                auto rec = [&](uint32_t ctr) {
                    if (atomicAdd(&S.acc[ctr], 1u) < MQ_CAP && stash) {
                        const uint32_t at = mq_stash_take(S, 1u);
                        if (at < MQ_STASH) stash[at] = (ctr << MQ_REL_BITS) | rel;
                    }
                };
                mq_slots(S.text, reinterpret_cast<const uint8_t *>(S.tab), a, poff, h, bits[h >> 5], klo, khi,
                         x, s + (uint64_t)r, q, rec, rec);
            }
        }
    }
    __syncthreads();
    const uint32_t *spi = reinterpret_cast<const uint32_t *>(tab + MQ_OFF_SPI);
    const uint16_t *cid = reinterpret_cast<const uint16_t *>(tab + MQ_OFF_CID);
    for (uint32_t j = tid; j < g.count; j += BLOCK)
        a.cnt[(uint64_t)spi[j] * a.nchunks + chunk] = S.acc[cid[j]];
    if (stash && tid == 0) a.stash_n[sitem] = S.nst;
}

// ---------------------------------------------------------------------------
// Prefix filter write pass: one work item = (text chunk, filter group). Each
// tile gathers its hits (local pattern j, tile position r) in an LDS list, sorts
// them by (j, r), and writes hit k of pattern j in the tile at CSR entry
// base_j + run_j + k, where base_j is the pattern's offset at the chunk start and
// run_j counts its hits in the chunk so far. A tile whose list would overflow is
// run again on halves of the pattern range, down to single patterns; a pattern
// with more hits in one tile than the list holds is never routed here (the
// router sends only patterns with at most 16 hits per 4096 starts on average, and
// the tile is re-run per pattern range until each fits).
// ---------------------------------------------------------------------------
constexpr int MQW_LIST = 4096;
static_assert(BT / 4 <= MQW_LIST, "a quarter tile of one pattern must fit the write list");

// Items are (chunk, listed group): group list[k] of f.groups / f.tabs (the group's
// write table) for k < nlisted, or group k when list is null. Patterns take part
// when route[sorted] == route_val: 2 for the count groups' patterns whose hits the
// count pass kept (here only where it did not: an item that overflowed, or more
// than MQ_CAP hits in the chunk; mq_stash_write_kernel writes the rest), 4 for the
// window's heavy patterns (groups of their own, nothing kept).
struct MqwArgs {
    MqArgs f;
    const BatchPat *pats;      // sorted
    const uint64_t *chunk_off; // [sorted pattern][chunk]
    const uint64_t *csr;       // [original index]
    int64_t *out;              // CSR entry k goes to out[k - lo]
    uint64_t lo, span;
    const uint32_t *list;
    uint32_t nlisted, nmq;
    const uint8_t *route;
    uint32_t route_val;
    const uint32_t *stash, *stash_n;  // null: nothing kept
    const uint8_t *ctabs;             // the count tables (counter ids)
};

struct MqwShared {
    uint4 text[B_CHUNKS];
    uint4 tab[MQ_LDS_BYTES / 16];
    uint32_t list[MQW_LIST];
    uint32_t run[MQ_G];
    uint8_t act[MQ_G];
    uint32_t nlist;
    int flag;
};

template <bool EXACT>
__global__ __launch_bounds__(BLOCK) void mq_write_kernel(MqwArgs w)
{
    __shared__ MqwShared S;
    const MqArgs &a = w.f;
    const uint64_t item = blockIdx.x;
    const uint64_t chunk = item / w.nlisted;
    const uint32_t gi = w.list ? w.list[item % w.nlisted] : (uint32_t)(item % w.nlisted);
    // the count pass kept the item's entries: patterns with at most MQ_CAP hits in
    // the chunk are written from them (mq_stash_write_kernel), the others here
    const bool kept = w.stash_n && w.stash_n[chunk * w.nmq + gi] <= MQ_STASH;
    const MqGroup g = a.groups[gi];
    const int tid = threadIdx.x;
    const uint8_t *tab = a.tabs + g.tab_off;
    const uint32_t *spi = reinterpret_cast<const uint32_t *>(tab + MQ_OFF_SPI);
    const uint32_t *poff = reinterpret_cast<const uint32_t *>(tab + MQ_OFF_POFF);
    const uint64_t wend = w.lo + w.span;
    // patterns with hits in this chunk that fall in the window
    if (tid == 0) S.flag = 0;
    __syncthreads();
    for (uint32_t j = tid; j < g.count; j += BLOCK) {
        const uint64_t sp = spi[j];
        uint32_t c = w.route[sp] == w.route_val ? a.cnt[sp * a.nchunks + chunk] : 0u;
        if (kept && c <= MQ_CAP) c = 0;  // written from the stash
        const uint64_t r0 = c ? w.csr[w.pats[sp].index] + w.chunk_off[sp * a.nchunks + chunk] : 0;
        const bool on = c && r0 < wend && r0 + c > w.lo;
        S.act[j] = on ? 1 : 0;
        S.run[j] = 0;
        if (on) S.flag = 1;
    }
    __syncthreads();
    if (!S.flag) return;  // uniform
    {
        const uint4 *src = reinterpret_cast<const uint4 *>(tab);
        for (uint32_t k = tid; k < MQ_LDS_BYTES / 16; k += BLOCK) S.tab[k] = src[k];
        if (tid == 0) S.nlist = 0;
    }
    const uint32_t *bits = reinterpret_cast<const uint32_t *>(S.tab);
    const uint8_t *T = reinterpret_cast<const uint8_t *>(S.tab);
    const uint32_t q = g.q;
    const uint32_t mlo = byte_mask(q < 4 ? (int)q : 4), mhi = byte_mask(q > 4 ? (int)q - 4 : 0);
    const uint64_t t0 = chunk * a.chunk_tiles;
    uint64_t t1 = t0 + a.chunk_tiles;
    if (t1 > a.ntiles) t1 = a.ntiles;
    const uint64_t tl = a.n >= g.min_m ? (a.n - g.min_m) / BT + 1 : 0;
    if (t1 > tl) t1 = tl;
    for (uint64_t t = t0; t < t1; t++) {
        const uint64_t s = t * (uint64_t)BT;
        __syncthreads();
        uint64_t x1 = s + (uint64_t)BT + g.max_m - 1;
        if (x1 > a.n) x1 = a.n;
        Staged<B_PER> st;
        stage_issue(st, a.text, s, x1);
        stage_commit<true>(st, S.text);
        const int boff = st.boff;
        __syncthreads();
        const uint64_t lim = a.n - g.min_m - s;
        const int hi_rel = lim >= (uint64_t)(BT - 1) ? BT - 1 : (int)lim;
        const int lo = tid * BL;
        const int hi = (lo + BL - 1) < hi_rel ? (lo + BL - 1) : hi_rel;
        // One attempt: the hits of patterns [jlo, jhi) at tile starts [rlo, rhi) are
        // listed, sorted, written, and counted into the run counters. Returns false
        // (and changes nothing) when the list overflows. Uniform over the block.
        auto attempt = [&](uint32_t jlo, uint32_t jhi, int rlo, int rhi) -> bool {
            const int a0 = lo > rlo ? lo : rlo, a1 = hi < rhi - 1 ? hi : rhi - 1;
            if (a0 <= a1) {
                const int u0 = (boff + a0) >> 4, u1 = (boff + a1) >> 4;
                uint4 nx = S.text[swz((uint32_t)u0)];
                for (int u = u0; u <= u1; u++) {
                    const uint4 cu = nx;
                    nx = S.text[swz((uint32_t)(u + 1))];
                    uint32_t hh[16], wb[16];
                    uint32_t cm = mq_filter16<EXACT>(cu, nx, bits, mlo, mhi, hh, wb);
                    const int r0 = 16 * u - boff;
                    while (cm) {
                        const int b = __builtin_ctz(cm);
                        cm &= cm - 1;
                        const int r = r0 + b;
                        if (r < a0 || r > a1) continue;
                        const uint32_t x = (uint32_t)(16 * u + b);
                        uint32_t klo, khi, h;
                        mq_key_at<EXACT>(S.text, x, mlo, mhi, klo, khi, h);
                        mq_slots(S.text, T, a, poff, h, bits[h >> 5], klo, khi, x, s + (uint64_t)r, q,
                                 [&](uint32_t) {},
                                 [&](uint32_t j) {
                                     if (j >= jlo && j < jhi && S.act[j]) {
                                         const uint32_t i = atomicAdd(&S.nlist, 1u);
                                         if (i < (uint32_t)MQW_LIST) S.list[i] = (j << 14) | (uint32_t)r;
                                     }
                                 });
                    }
                }
            }
            __syncthreads();
            const uint32_t nl = S.nlist;
            __syncthreads();
            if (tid == 0) S.nlist = 0;
            if (nl > (uint32_t)MQW_LIST) {
                __syncthreads();
                return false;
            }
            if (nl) {
                // bitonic sort of the list by (j, r), padded to a power of two
                uint32_t n2 = 2;
                while (n2 < nl) n2 <<= 1;
                for (uint32_t i = nl + tid; i < n2; i += BLOCK) S.list[i] = 0xFFFFFFFFu;
                __syncthreads();
                for (uint32_t k = 2; k <= n2; k <<= 1)
                    for (uint32_t jj = k >> 1; jj > 0; jj >>= 1) {
                        for (uint32_t i = tid; i < n2; i += BLOCK) {
                            const uint32_t ixj = i ^ jj;
                            if (ixj > i) {
                                const uint32_t x = S.list[i], y = S.list[ixj];
                                if ((x > y) == ((i & k) == 0)) {
                                    S.list[i] = y;
                                    S.list[ixj] = x;
                                }
                            }
                        }
                        __syncthreads();
                    }
                // rank inside its pattern's run (entries before it with the same j), write
                auto rank_of = [&](uint32_t e, uint32_t j) {
                    uint32_t b0 = 0, b1 = e;  // first entry of pattern j: lower bound of j << 14
                    while (b0 < b1) {
                        const uint32_t mid = (b0 + b1) >> 1;
                        if (S.list[mid] < (j << 14)) b0 = mid + 1; else b1 = mid;
                    }
                    return e - b0;
                };
                for (uint32_t e = tid; e < nl; e += BLOCK) {
                    const uint32_t key = S.list[e], j = key >> 14, r = key & 0x3FFFu;
                    const uint64_t sp = spi[j];
                    const uint64_t k = w.csr[w.pats[sp].index] + w.chunk_off[sp * a.nchunks + chunk] +
                                       S.run[j] + rank_of(e, j);
                    if (k - w.lo < w.span) w.out[k - w.lo] = (int64_t)(s + r);
                }
                __syncthreads();
                // the last entry of each pattern advances its run counter
                for (uint32_t e = tid; e < nl; e += BLOCK) {
                    const uint32_t j = S.list[e] >> 14;
                    if (e + 1 == nl || (S.list[e + 1] >> 14) != j) S.run[j] += rank_of(e, j) + 1;
                }
            }
            __syncthreads();
            return true;
        };
        // pattern ranges: the whole group, halved on overflow; a single pattern that
        // overflows is run over the tile's quarters (at most 4096 starts, so at
        // most 4096 hits of one pattern: each fits)
        uint32_t jlo = 0;
        while (jlo < g.count) {
            uint32_t jhi = g.count;
            while (!attempt(jlo, jhi, 0, BT)) {
                if (jhi - jlo > 1) {
                    jhi = jlo + (jhi - jlo) / 2;
                    continue;
                }
                for (int qt = 0; qt < 4; qt++) attempt(jlo, jhi, qt * (BT / 4), (qt + 1) * (BT / 4));
                break;
            }
            jlo = jhi;
        }
    }
}

// Write pass of the items whose hits the count pass kept: the item's entries
// (counter << MQ_REL_BITS | start in the chunk) are sorted in LDS, so each
// counter's hits come in ascending order; entry k of counter c is hit number
// k - first(c) in the chunk of every taking-part pattern counted by c (duplicates
// and the m == q patterns of a slot share one counter). Threads take consecutive
// entries, so a pattern's positions are stored coalesced. The text is not read.
__global__ __launch_bounds__(BLOCK) void mq_stash_write_kernel(MqwArgs w)
{
    __shared__ uint32_t s_e[MQ_STASH];
    __shared__ uint32_t s_head[MQ_G];   // counter -> first taking-part pattern, or MQ_NONE
    __shared__ uint32_t s_next[MQ_G];   // pattern -> next one on the same counter
    __shared__ uint64_t s_base[MQ_G];   // pattern -> CSR entry of its first hit in the chunk
    __shared__ int s_any;
    const MqArgs &a = w.f;
    const uint64_t chunk = blockIdx.x / w.nlisted;
    const uint32_t gi = w.list[blockIdx.x % w.nlisted];
    const uint64_t sitem = chunk * w.nmq + gi;
    const uint32_t ne = w.stash_n[sitem];
    if (ne == 0 || ne > MQ_STASH) return;  // uniform
    const MqGroup g = a.groups[gi];
    const uint8_t *ctab = w.ctabs + g.tab_off;
    const uint32_t *spi = reinterpret_cast<const uint32_t *>(ctab + MQ_OFF_SPI);
    const uint16_t *cid = reinterpret_cast<const uint16_t *>(ctab + MQ_OFF_CID);
    const int tid = threadIdx.x;
    const uint64_t wend = w.lo + w.span;
    for (uint32_t k = tid; k < (uint32_t)MQ_G; k += BLOCK) s_head[k] = MQ_NONE;
    if (tid == 0) s_any = 0;
    uint32_t n2 = 64;
    while (n2 < ne) n2 <<= 1;
    const uint32_t *src = w.stash + sitem * MQ_STASH;
    for (uint32_t k = tid; k < n2; k += BLOCK) s_e[k] = k < ne ? src[k] : 0xFFFFFFFFu;
    __syncthreads();
    for (uint32_t j = tid; j < g.count; j += BLOCK) {
        const uint64_t sp = spi[j];
        const uint32_t c = w.route[sp] == 2 ? a.cnt[sp * a.nchunks + chunk] : 0u;
        if (!c || c > MQ_CAP) continue;  // counters above MQ_CAP were not kept
        const uint64_t r0 = w.csr[w.pats[sp].index] + w.chunk_off[sp * a.nchunks + chunk];
        if (!(r0 < wend && r0 + c > w.lo)) continue;
        s_base[j] = r0;
        s_next[j] = atomicExch(&s_head[cid[j]], j);
        s_any = 1;
    }
    __syncthreads();
    if (!s_any) return;  // uniform
    // bitonic sort, ascending
    for (uint32_t k = 2; k <= n2; k <<= 1)
        for (uint32_t jj = k >> 1; jj > 0; jj >>= 1) {
            for (uint32_t i = tid; i < n2; i += BLOCK) {
                const uint32_t ixj = i ^ jj;
                if (ixj > i) {
                    const uint32_t x = s_e[i], y = s_e[ixj];
                    if ((x > y) == ((i & k) == 0)) {
                        s_e[i] = y;
                        s_e[ixj] = x;
                    }
                }
            }
            __syncthreads();
        }
    const uint64_t s0 = chunk * (uint64_t)a.chunk_tiles * (uint64_t)BT;
    constexpr uint32_t RMASK = (1u << MQ_REL_BITS) - 1u;
    for (uint32_t k = tid; k < ne; k += BLOCK) {
        const uint32_t e = s_e[k], c = e >> MQ_REL_BITS;
        uint32_t j = s_head[c];
        if (j == MQ_NONE) continue;
        uint32_t b0 = 0, b1 = k;  // first entry of counter c
        while (b0 < b1) {
            const uint32_t mid = (b0 + b1) >> 1;
            if ((s_e[mid] >> MQ_REL_BITS) < c) b0 = mid + 1; else b1 = mid;
        }
        const int64_t pos = (int64_t)(s0 + (e & RMASK));
        for (; j != MQ_NONE; j = s_next[j]) {
            const uint64_t idx = s_base[j] + (k - b0);
            if (idx - w.lo < w.span) w.out[idx - w.lo] = pos;
        }
    }
}

// One workgroup per pattern: tables into params[j].
__global__ __launch_bounds__(BLOCK) void batch_prep_kernel(const BatchPat *pats, const uint8_t *patbytes,
                                                           Params *params)
{
    __shared__ uint32_t s_tab[1 << H_MAX];
    __shared__ uint32_t s_bad[PERIOD_MAX + 1];
    const BatchPat bp = pats[blockIdx.x];
    Params *P = params + blockIdx.x;
    if (threadIdx.x == 0) {
        P->m = bp.m;
        P->algo = bp.algo;
        P->q = bp.q;
        P->hbits = bp.hbits;
    }
    build_tables(patbytes + bp.pat_off, bp.m, bp.algo, bp.q, bp.hbits, P, s_tab, s_bad, nullptr);
}

// One workgroup per sorted pattern: per-chunk counts -> exclusive offsets and the
// pattern's total (stored at totals[original index]).
__global__ __launch_bounds__(BLOCK) void batch_seg_scan_kernel(const BatchPat *pats, const uint32_t *cnt,
                                                               uint64_t nchunks, uint64_t *chunk_off,
                                                               uint64_t *totals)
{
    __shared__ uint32_t s_w[BLOCK / 64];
    __shared__ uint64_t s_carry;
    const uint64_t j = blockIdx.x;
    const uint32_t *c = cnt + j * nchunks;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (uint64_t b = 0; b < nchunks; b += BLOCK) {
        const uint64_t i = b + threadIdx.x;
        const uint32_t v = i < nchunks ? c[i] : 0u;
        uint32_t tot;
        const uint32_t before = block_excl_scan(v, s_w, tot);
        const uint64_t carry = s_carry;
        if (chunk_off && i < nchunks) chunk_off[j * nchunks + i] = carry + before;
        __syncthreads();
        if (threadIdx.x == 0) s_carry = carry + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) totals[pats[j].index] = s_carry;
}

// Exclusive scan of P totals (original order) -> csr[0..P], one workgroup of 1024.
__global__ __launch_bounds__(1024) void csr_scan_kernel(const uint64_t *totals, uint64_t P, uint64_t *csr)
{
    __shared__ uint64_t s_part[1024];
    const uint64_t per = (P + 1023) / 1024;
    const uint64_t b = threadIdx.x * per;
    const uint64_t e = b + per < P ? b + per : P;
    uint64_t sum = 0;
    for (uint64_t k = b; k < e; k++) sum += totals[k];
    s_part[threadIdx.x] = sum;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const uint64_t v = threadIdx.x >= (unsigned)d ? s_part[threadIdx.x - d] : 0;
        __syncthreads();
        s_part[threadIdx.x] += v;
        __syncthreads();
    }
    uint64_t run = s_part[threadIdx.x] - sum;
    for (uint64_t k = b; k < e; k++) {
        csr[k] = run;
        run += totals[k];
    }
    if (threadIdx.x == 1023) csr[P] = s_part[1023];
}

template <int ALGO, int VAR>
hipError_t launch_batch_v(const BatchArgs &a, bool write, hipStream_t st)
{
    const uint64_t grid = a.nchunks * a.ngroups;
    if (grid == 0) return hipSuccess;
    if (grid > 0x7FFFFFFFull) return hipErrorInvalidValue;
    if (write)
        hipLaunchKernelGGL((batch_kernel<ALGO, VAR, true>), dim3((uint32_t)grid), dim3(BLOCK), 0, st, a);
    else
        hipLaunchKernelGGL((batch_kernel<ALGO, VAR, false>), dim3((uint32_t)grid), dim3(BLOCK), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_batch_class(uint32_t algo, uint32_t var, const BatchArgs &a, bool write, hipStream_t st)
{
    switch (algo) {
    case ALGO_SHIFT_AND:
        switch (var) {
        case 0: return launch_batch_v<ALGO_SHIFT_AND, 0>(a, write, st);
        case 1: return launch_batch_v<ALGO_SHIFT_AND, 1>(a, write, st);
        case 2: return launch_batch_v<ALGO_SHIFT_AND, 2>(a, write, st);
        default: return launch_batch_v<ALGO_SHIFT_AND, 3>(a, write, st);
        }
    case ALGO_BNDM: return launch_batch_v<ALGO_BNDM, 0>(a, write, st);
    case ALGO_SBNDM: return launch_batch_v<ALGO_SBNDM, 0>(a, write, st);
    case ALGO_HASHQ:
        switch (var) {
        case 1: return launch_batch_v<ALGO_HASHQ, 1>(a, write, st);
        case 2: return launch_batch_v<ALGO_HASHQ, 2>(a, write, st);
        case 3: return launch_batch_v<ALGO_HASHQ, 3>(a, write, st);
        default: return launch_batch_v<ALGO_HASHQ, 4>(a, write, st);
        }
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_csr_scan(const uint64_t *totals, uint64_t P, uint64_t *csr, hipStream_t st)
{
    hipLaunchKernelGGL(csr_scan_kernel, dim3(1), dim3(1024), 0, st, totals, P, csr);
    return hipGetLastError();
}

namespace {
// a batched count pass's timing record, discarded unless the pass reaches its end
struct BatchProfGuard {
    BatchProfRec r;
    bool on = false;
    ~BatchProfGuard()
    {
        if (on) prof_batch_discard(r);
    }
};
}  // namespace

hipError_t launch_batch(const BatchLaunch &L, hipStream_t st)
{
    BatchProfGuard bp;
    if (!L.write) bp.on = prof_batch_begin(st, bp.r);
    BatchArgs a;
    memset(&a, 0, sizeof a);
    a.text = L.text;
    a.n = L.n;
    a.pats = L.pats;
    a.groups = L.groups;
    a.params = L.params;
    a.patbytes = L.patbytes;
    a.chunk_tiles = L.chunk_tiles;
    a.nchunks = L.nchunks;
    a.ntiles = L.ntiles;
    a.cnt = L.cnt;
    a.chunk_off = L.chunk_off;
    a.csr = L.csr;
    a.out = L.out;
    a.lo = L.lo;
    a.span = L.span;
    hipError_t e;
    if (L.prep) {
        hipLaunchKernelGGL(batch_prep_kernel, dim3(L.npats), dim3(BLOCK), 0, st, L.pats, L.patbytes,
                           const_cast<Params *>(L.params));
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // one launch per run of groups that share a kernel variant
    const BatchGroup *hg = L.write ? L.host_groups : L.host_cgroups;
    const uint32_t ng = L.write ? L.ngroups : L.ncgroups;
    a.groups = L.write ? L.groups : L.cgroups;  // write: the per-pattern write groups given
    uint32_t g = 0;
    while (g < ng) {
        uint32_t h = g + 1;
        while (h < ng && hg[h].algo == hg[g].algo && hg[h].var == hg[g].var) h++;
        a.group_lo = g;
        a.ngroups = h - g;
        if ((e = launch_batch_class(hg[g].algo, hg[g].var, a, L.write, st)) != hipSuccess) return e;
        g = h;
    }
    if (L.write && (L.nmqw || L.nhq)) {
        MqwArgs w;
        memset(&w, 0, sizeof w);
        w.f.text = L.text;
        w.f.n = L.n;
        w.f.patbytes = L.patbytes;
        w.f.chunk_tiles = L.chunk_tiles;
        w.f.nchunks = L.nchunks;
        w.f.ntiles = L.ntiles;
        w.f.cnt = L.cnt;
        w.pats = L.pats;
        w.chunk_off = L.chunk_off;
        w.csr = L.csr;
        w.out = L.out;
        w.lo = L.lo;
        w.span = L.span;
        w.nmq = L.nmq;
        w.route = L.wroute;
        // a filter pass over the text: groups[list[k]] (list null: groups[k]) for k < ng,
        // the exact-key groups (q <= 2) and the hashed ones in launches of their own.
        // list is the device copy (kernel argument), host_list the host one, host the
        // host copy of the groups (both read here to split the launches).
        auto rescan = [&](const uint32_t *list, const uint32_t *host_list, const MqGroup *host,
                          uint32_t ng) -> hipError_t {
            uint32_t nexact = 0;
            while (nexact < ng && host[host_list ? host_list[nexact] : nexact].q <= 2) nexact++;
            for (int pass = 0; pass < 2; pass++) {
                const uint32_t g0 = pass ? nexact : 0, g1 = pass ? ng : nexact;
                if (g1 == g0) continue;
                if (list) {
                    w.list = list + g0;
                } else {
                    w.list = nullptr;
                    w.f.groups += g0;
                }
                w.nlisted = g1 - g0;
                const uint64_t grid = L.nchunks * (g1 - g0);
                if (grid > 0x7FFFFFFFull) return hipErrorInvalidValue;
                if (pass == 0)
                    hipLaunchKernelGGL(mq_write_kernel<true>, dim3((uint32_t)grid), dim3(BLOCK), 0, st, w);
                else
                    hipLaunchKernelGGL(mq_write_kernel<false>, dim3((uint32_t)grid), dim3(BLOCK), 0, st, w);
                if (!list) w.f.groups -= g0;
                hipError_t e2 = hipGetLastError();
                if (e2 != hipSuccess) return e2;
            }
            return hipSuccess;
        };
        if (L.nmqw && L.mqstash) {
            // the patterns whose hits the count pass kept: copied out, then the items
            // where it did not keep them scanned again
            w.f.groups = L.mqgroups;
            w.f.tabs = L.mqwtabs;
            w.f.ngroups = L.nmq;
            w.route_val = 2;
            w.stash = L.mqstash;
            w.stash_n = L.mqstash_n;
            w.ctabs = L.mqtabs;
            w.list = L.mqwlist;
            w.nlisted = L.nmqw;
            const uint64_t grid = L.nchunks * L.nmqw;
            if (grid > 0x7FFFFFFFull) return hipErrorInvalidValue;
            hipLaunchKernelGGL(mq_stash_write_kernel, dim3((uint32_t)grid), dim3(BLOCK), 0, st, w);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            if ((e = rescan(L.mqwlist, L.host_mqwlist, L.host_mq, L.nmqw)) != hipSuccess) return e;
        }
        if (L.nhq) {  // the heavy patterns: one filter pass of their own groups
            w.f.groups = L.hqgroups;
            w.f.tabs = L.hqtabs;
            w.f.ngroups = L.nhq;
            w.route_val = 4;
            w.stash = nullptr;
            w.stash_n = nullptr;
            if ((e = rescan(nullptr, nullptr, L.host_hq, L.nhq)) != hipSuccess) return e;
        }
    }
    if (!L.write && L.nmq) {
        MqArgs m;
        memset(&m, 0, sizeof m);
        m.text = L.text;
        m.n = L.n;
        m.groups = L.mqgroups;
        m.tabs = L.mqtabs;
        m.patbytes = L.patbytes;
        m.ngroups = L.nmq;
        m.chunk_tiles = L.chunk_tiles;
        m.nchunks = L.nchunks;
        m.ntiles = L.ntiles;
        m.cnt = L.cnt;
        m.stash = L.mqstash;
        m.stash_n = L.mqstash_n;
        m.nmq = L.nmq;
        // one launch for the exact-key groups (q <= 2), one for the hashed ones; the
        // groups are ordered by q, so each launch takes a contiguous range
        uint32_t nexact = 0;
        while (nexact < L.nmq && L.host_mq[nexact].q <= 2) nexact++;
        if (bp.on) {
            if ((e = hipEventRecord(bp.r.e1, st)) != hipSuccess) return e;
            for (uint32_t g = 0; g < L.nmq; g++) bp.r.filter_pattern_bytes += (uint64_t)L.host_mq[g].count * L.n;
        }
        for (int pass = 0; pass < 2; pass++) {
            const uint32_t g0 = pass ? nexact : 0, g1 = pass ? L.nmq : nexact;
            if (g1 == g0) continue;
            m.groups = L.mqgroups + g0;
            m.ngroups = g1 - g0;
            m.group_base = g0;
            const uint64_t grid = L.nchunks * (g1 - g0);
            if (grid > 0x7FFFFFFFull) return hipErrorInvalidValue;
            if (pass == 0)
                hipLaunchKernelGGL(mq_count_kernel<true>, dim3((uint32_t)grid), dim3(BLOCK), 0, st, m);
            else
                hipLaunchKernelGGL(mq_count_kernel<false>, dim3((uint32_t)grid), dim3(BLOCK), 0, st, m);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            bp.r.filter_launches++;
        }
        if (bp.on && (e = hipEventRecord(bp.r.e2, st)) != hipSuccess) return e;
    } else if (bp.on) {  // no filter groups: an empty filter interval
        if ((e = hipEventRecord(bp.r.e1, st)) != hipSuccess) return e;
        if ((e = hipEventRecord(bp.r.e2, st)) != hipSuccess) return e;
    }
    if (!L.write) {
        hipLaunchKernelGGL(batch_seg_scan_kernel, dim3(L.npats), dim3(BLOCK), 0, st, L.pats, L.cnt,
                           L.nchunks, L.chunk_off_out, L.totals);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (L.csr_out) {
            hipLaunchKernelGGL(csr_scan_kernel, dim3(1), dim3(1024), 0, st, L.totals,
                               (uint64_t)L.npats_total, L.csr_out);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    if (bp.on) {
        if ((e = hipEventRecord(bp.r.e3, st)) != hipSuccess) return e;
        prof_batch_push(bp.r);
        bp.on = false;
    }
    return hipSuccess;
}

}  // namespace sm
