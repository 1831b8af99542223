// HIP kernels for online exact string matching on gfx950 (CDNA4).
//
// Problem (paper, Section 1): report every i with t[i .. i+m-1] = p, for a byte
// text t of length n and a pattern p of length m.
//
// Work decomposition. A tile is BLOCK * L consecutive candidate starts; one
// workgroup of BLOCK threads owns a tile at a time. The bytes the tile's windows
// need (the starts plus an (m-1)-byte halo, or only the window ends for Hash-q)
// are staged from HBM into LDS with 16-byte coalesced loads. Each lane then owns
// a contiguous segment of L starts and runs one of the paper's bit-parallel or
// skip algorithms over it, reading the text from LDS:
//   * Shift-And (Fig. 3, SA/SO): one 64-bit (or 32-bit) state register per lane,
//     complemented form D = (D << 1) | M[c], with deferred hit detection: bits
//     above m-1 keep the history of the match bit, so hits are examined once per
//     16 (or 4, or 1) bytes instead of every byte.
//   * BNDM and SBNDM (Fig. 3): backward scan of each window with the masks of the
//     reversed pattern, shifting by the longest prefix seen (BNDM) or by the
//     length of the non-factor suffix (SBNDM).
//   * Hash-q (Fig. 1, HASHq): Horspool-style skip on the hash of the q-gram that
//     ends the window; a zero shift triggers byte-exact verification.
// Every lane produces its hits in ascending order. find_all is three launches
// with no waiting between workgroups:
//   count: one pass over the text from HBM; per-tile hit counts, and for a tile
//          with at most STASH_K hits, the hits' offsets in the tile (u16) are
//          kept in a per-tile stash;
//   scan:  exclusive scan of the tile counts (tile output offsets, total) and
//          the ascending list of tiles that have hits;
//   emit:  for each listed tile, positions are written at the tile's offset,
//          from the stash, or -- for tiles with more than STASH_K hits -- by
//          rescanning the tile.
// Positions land sorted and deterministically (count -> scan -> write).
//
// Bounds. Only starts i <= n - m are ever reported, and every window that is
// reported reads bytes < n only. LDS bytes beyond the text are never consulted
// for a reported position. Global loads are 16-byte aligned blocks that contain
// at least one byte of the text, so they never leave the text's pages.
#include <hip/hip_runtime.h>

#include <cstring>

#include "sm_internal.h"
#include "sm_device.h"

namespace sm {
namespace {
using namespace dev;

// ---------------------------------------------------------------------------
// Tiles
// ---------------------------------------------------------------------------
struct ScanArgs {
    const uint8_t *text;
    uint64_t n;
    const Params *prm;
    const uint8_t *pat;
    uint32_t m, q, hbits, tiles_per_wg;
    uint32_t slots;       // find: lanes keep their first hits while counting
    uint32_t bs;          // block filter: starts per sampled block (bf_stride(m))
    uint64_t ntiles;
    uint64_t *total;      // count mode: occurrences are added here
    uint32_t *tile_cnt;   // per-tile counts (count kernel writes, tile scan and emit read)
    uint64_t *super;      // per 64 tiles: (tiles with hits << 40) | hits, added by the count kernel
    uint16_t *stash;      // find mode: STASH_K offsets per tile
    const TileEntry *list;     // emit: tiles with hits, ascending, with their offsets
    const uint64_t *nlist;     // emit: list length
    uint32_t *bits;       // find, bitmap form: hit bitmaps of the dense tiles (T / 32 words per tile)
    int64_t *out;         // emit: hit number k of the pattern goes to out[k - lo]
    uint64_t lo, cap;     // emit: window [lo, lo + cap) of hit numbers
    // Shift-And for m > SA_SUFFIX (the scan finds the pattern's last sfx bytes, sfx =
    // SA_SUFFIX or SA_SHORT as planned; text0 and m_full are the original text and m, for
    // the check of the first m - sfx bytes). Up to SA_STAGE_MAX, text/n/m above are the
    // originals too and the tiles stage whole windows: the scan reads them from sfx_off =
    // m - sfx bytes on. Longer patterns: text/n above are the text shifted by m - sfx, m
    // above is sfx and sfx_off is 0.
    const uint8_t *text0;
    uint32_t m_full, sfx_off;
};

template <int ALGO, int L>
struct Geometry {
    static constexpr int T = BLOCK * L;
    // halo bytes beyond the tile, plus 16 for misalignment and 16 for word reads
    static constexpr int HALO = (ALGO == ALGO_HASHQ) ? (Q_MAX + 32)
                                : (ALGO == ALGO_SHIFT_AND ? (SA_STAGE_MAX + 32) : (BP_MAX_M + 32));
    // whole groups of 8 chunks: the swizzle permutes chunks inside such groups
    static constexpr int CHUNKS = (((T + HALO + 15) / 16 + 1) + 7) & ~7;
    static constexpr int PER = (CHUNKS + BLOCK - 1) / BLOCK;  // chunk loads per thread
};

template <int ALGO, int L>
struct TileShared {
    uint4 text[Geometry<ALGO, L>::CHUNKS];
    uint64_t mask[(ALGO == ALGO_HASHQ) ? 1 : 256];
    uint8_t shift[(ALGO == ALGO_HASHQ) ? (1 << H_MAX) : 1];
    uint32_t w[BLOCK / 64];
};

// Find-mode count pass: counts every hit of the lane and keeps its first four
// tile-relative starts (u16 pairs in two registers), so a tile with few hits
// needs no second scan to fill its stash.
constexpr uint32_t LANE_K = 4;
struct CapEmit {
    uint32_t p0 = 0, p1 = 0, n = 0;
    __device__ __forceinline__ void put(int rel)
    {
        const uint32_t r = (uint32_t)rel & 0xFFFFu;
        if (n == 0) p0 = r;
        else if (n == 1) p0 |= r << 16;
        else if (n == 2) p1 = r;
        else if (n == 3) p1 |= r << 16;
        n++;
    }
    // once more hits than slots are seen, the tile is scanned again anyway: count only
    __device__ __forceinline__ bool saturated() const { return n > LANE_K; }
    __device__ __forceinline__ void add(uint32_t k) { n += k; }
    __device__ __forceinline__ uint16_t get(uint32_t k) const
    {
        const uint32_t w = k < 2 ? p0 : p1;
        return (uint16_t)((k & 1) ? (w >> 16) : (w & 0xFFFFu));
    }
};

// Pattern tables, read from the parameter block into registers (issue), then
// written to LDS (commit): each thread carries one mask entry or 16 Hash-q
// buckets.
template <int ALGO>
__device__ __forceinline__ uint4 tables_issue(const Params *prm, uint32_t hbits)
{
    const uint32_t tid = threadIdx.x;
    uint4 r = {0u, 0u, 0u, 0u};
    if (ALGO == ALGO_HASHQ) {
        if (tid < ((1u << hbits) >> 4)) r = reinterpret_cast<const uint4 *>(prm->shift)[tid];
    } else {
        const uint64_t w = prm->mask[tid];
        r.x = (uint32_t)w;
        r.y = (uint32_t)(w >> 32);
    }
    return r;
}

template <int ALGO, int VAR>
__device__ __forceinline__ void tables_commit(uint4 r, uint64_t *s_mask, uint8_t *s_shift,
                                              uint32_t hbits)
{
    const uint32_t tid = threadIdx.x;
    if (ALGO == ALGO_HASHQ) {
        if (tid < ((1u << hbits) >> 4)) reinterpret_cast<uint4 *>(s_shift)[tid] = r;
    } else if (ALGO == ALGO_SHIFT_AND && (VAR == 0 || VAR == 6)) {  // 32-bit masks
        reinterpret_cast<uint32_t *>(s_mask)[tid] = r.x;
    } else if (ALGO == ALGO_SHIFT_AND && VAR == 4) {  // m <= 8: the masks fit a byte
        reinterpret_cast<uint8_t *>(s_mask)[tid] = (uint8_t)r.x;
    } else {
        s_mask[tid] = ((uint64_t)r.y << 32) | r.x;
    }
}

// Geometry of tile t (t < ntiles): tile start s, staged span [x0, x1), last
// admissible relative start hi_rel, and the span's offset r0 from s.
struct TileGeom {
    uint64_t s, x0, x1;
    int hi_rel, r0;
};

// scanners that read the tile in 16-byte units per lane take the swizzled layout
constexpr bool swz_tile(int algo) { return algo == ALGO_SHIFT_AND || algo == ALGO_BRUTE; }
// scanners whose hits come as masks (bitmap form, first-hit slots)
constexpr bool mask_hits(int algo) { return algo == ALGO_SHIFT_AND || algo == ALGO_BRUTE; }

template <int ALGO, int L>
__device__ __forceinline__ TileGeom tile_geom(const ScanArgs &a, uint64_t t)
{
    constexpr int T = Geometry<ALGO, L>::T;
    TileGeom g;
    const uint64_t last_start = a.n - a.m;  // n >= m guaranteed by the host
    g.s = t * (uint64_t)T;
    const uint64_t lim = last_start - g.s;  // >= 0 since t < ntiles
    g.hi_rel = lim >= (uint64_t)(T - 1) ? T - 1 : (int)lim;
    g.r0 = (ALGO == ALGO_HASHQ) ? (int)(a.m - a.q) : 0;
    g.x0 = g.s + (uint64_t)g.r0;
    // one past the last byte any window reads (FSBNDM: and the byte after it)
    g.x1 = g.s + (uint64_t)g.hi_rel + a.m + (ALGO == ALGO_FSBNDM ? 1u : 0u);
    if (g.x1 > a.n) g.x1 = a.n;
    return g;
}

// Stage tile t synchronously (used by the emit kernel's rescans).
template <int ALGO, int L>
__device__ __forceinline__ void stage_tile(TileShared<ALGO, L> &S, const ScanArgs &a, uint64_t t,
                                           uint64_t &s, int &li0, int &lo, int &hi)
{
    using G = Geometry<ALGO, L>;
    const TileGeom g = tile_geom<ALGO, L>(a, t);
    Staged<G::PER> st;
    stage_issue(st, a.text, g.x0, g.x1);
    stage_commit<swz_tile(ALGO)>(st, S.text);
    s = g.s;
    li0 = st.boff - g.r0;
    lo = threadIdx.x * L;
    hi = (lo + L - 1) < g.hi_rel ? (lo + L - 1) : g.hi_rel;
}

// Pattern words of the brute-force scanner (uniform: scalar registers).
struct BruteWords {
    uint32_t w[BRUTE_MAX_M];
};
template <int ALGO>
__device__ __forceinline__ BruteWords brute_words(const Params *prm)
{
    BruteWords b;
#pragma unroll
    for (int k = 0; k < BRUTE_MAX_M; k++) b.w[k] = ALGO == ALGO_BRUTE ? (uint32_t)prm->mask[k] : 0u;
    return b;
}

template <int ALGO, int L, int VAR, bool WRITE, class E>
__device__ __forceinline__ uint32_t run_lane(TileShared<ALGO, L> &S, const ScanArgs &a, int m,
                                             int sh1, int period, int period_lb, uint64_t s,
                                             int li0, int lo, int hi, E &o, const BruteWords &bw,
                                             uint4 ppre = uint4{0u, 0u, 0u, 0u}, bool full = false)
{
    // suffix forms (m > SA_SUFFIX): variant 5 scans the pattern's last SA_SUFFIX bytes on a
    // 64-bit state, variant 6 its last SA_SHORT bytes on a 32-bit one (32-bit masks)
    constexpr bool SUFFIX_FORM = ALGO == ALGO_SHIFT_AND && (VAR == 5 || VAR == 6);
    constexpr int SFX = VAR == 6 ? SA_SHORT : SA_SUFFIX;
    using SW = std::conditional_t<VAR == 6, uint32_t, uint64_t>;
    static_assert(SFX - 1 + 16 <= 8 * (int)sizeof(SW), "hits checked every 16 bytes");
    if constexpr (SUFFIX_FORM && (takes_masks<E>::value || is_no_emit<E>::value)) {
        // candidates (the last SFX bytes match) as a bitmap first, settled after the scan
        // by the whole wave (every lane takes part)
        const uint32_t per = period > 0 && period <= SFX ? (uint32_t)period : 0u;
        constexpr int NW = L > 64 ? L / 64 : 1;
        BitAcc<NW> cand;
        const int sli0 = li0 + (int)a.sfx_off;  // LDS index of the suffix of start 0
        lane_shift_and<SW, 16, false, L>(S.text, reinterpret_cast<const SW *>(S.mask), SFX, sli0, lo, hi, cand,
                                         full);
        const SuffixCtx sc{a.text0, a.pat, S.text, sli0, s, a.m_full, (uint32_t)SFX, per, ppre};
        const uint32_t c = suffix_resolve<L>(cand, sc, lo);
        if constexpr (takes_masks<E>::value) {
#pragma unroll
            for (int k = 0; k < NW; k++) o.w[k] |= cand.w[k];
        }
        return c;
    }
    if (ALGO != ALGO_HASHQ && lo > hi) return 0u;  // Hash-q lanes take part in wave checks
    if constexpr (ALGO == ALGO_SHIFT_AND) {
        if constexpr (SUFFIX_FORM) {  // m > SA_SUFFIX: the last SFX bytes, then the rest verified
            const uint32_t per = period > 0 && period <= SFX ? (uint32_t)period : 0u;
            {  // hits one by one: checked as they come
                SuffixVerify<E, SFX> sv{o, a.text0, a.pat, a.m_full, per, s, lo};
                lane_shift_and<SW, 16, true, L>(S.text, reinterpret_cast<const SW *>(S.mask), SFX,
                                                li0 + (int)a.sfx_off, lo, hi, sv, full);
                return sv.n;
            }
        }
        if (VAR == 4)
            return lane_shift_and<uint32_t, 16, WRITE, L>(S.text, reinterpret_cast<const uint8_t *>(S.mask), m,
                                                          li0, lo, hi, o, full);
        if (VAR == 0)
            return lane_shift_and<uint32_t, 16, WRITE, L>(S.text, reinterpret_cast<const uint32_t *>(S.mask),
                                                          m, li0, lo, hi, o, full);
        if (VAR == 1) return lane_shift_and<uint64_t, 16, WRITE, L>(S.text, S.mask, m, li0, lo, hi, o, full);
        if (VAR == 2) return lane_shift_and<uint64_t, 4, WRITE, L>(S.text, S.mask, m, li0, lo, hi, o, full);
        return lane_shift_and<uint64_t, 1, WRITE, L>(S.text, S.mask, m, li0, lo, hi, o, full);
    } else if constexpr (ALGO == ALGO_BNDM) {  // VAR selects the q-gram width 1, 2, 4
        constexpr int Q = VAR == 0 ? 1 : (VAR == 1 ? 2 : 4);
        return lane_bndm<Q, WRITE>(reinterpret_cast<const uint8_t *>(S.text), S.mask, m, li0, lo, hi, o);
    } else if constexpr (ALGO == ALGO_FSBNDM) {
        // the last relative start whose byte after the window lies in the text
        const int64_t fh = (int64_t)a.n - (int64_t)m - 1 - (int64_t)s;
        return lane_fsbndm<WRITE>(reinterpret_cast<const uint8_t *>(S.text), S.mask, m, period, li0, lo, hi,
                                  fh < (int64_t)hi ? (int)fh : hi, o);
    } else if constexpr (ALGO == ALGO_BRUTE) {
        return lane_brute<WRITE>(S.text, bw.w, m, li0, lo, hi, o);
    } else if constexpr (ALGO == ALGO_SBNDM) {  // VAR & 3 selects the q-gram width 1, 2, 4, 8
        constexpr int Q = (VAR & 3) == 0 ? 1 : ((VAR & 3) == 1 ? 2 : ((VAR & 3) == 2 ? 4 : 8));
        if constexpr (VAR >= 4) {
            // factor form (m_full > 64): the scan runs over the text shifted by m_full - 64
            // with the masks of the pattern's last 64 bytes and shifts by their period
            // after a full read; each start found is an occurrence when the pattern's
            // first m_full - 64 bytes match too
            SuffixVerify<E, BP_MAX_M> sv{o, a.text0, a.pat, a.m_full, 0u, s, lo};
            lane_sbndm<Q, true>(reinterpret_cast<const uint8_t *>(S.text), S.mask, m, period, li0, lo, hi, sv);
            return sv.n;
        }
        return lane_sbndm<Q, WRITE>(reinterpret_cast<const uint8_t *>(S.text), S.mask, m, period, li0,
                                    lo, hi, o);
    } else {
        return lane_hashq<VAR, WRITE>(reinterpret_cast<const uint32_t *>(S.text), S.shift, m,
                                      (int)a.q, (int)a.hbits, sh1, period, period_lb, li0, lo, hi,
                                      a.text, s, a.pat, o);
    }
}

// Super-chunk totals: the count pass adds each workgroup's tiles into the total of
// their 64-tile super-chunk (one device-scope atomic per workgroup and super-chunk,
// none for tiles without hits), so the tile scan reads 1/64 of the counts before
// its chunk. Thread 0 keeps the pending total of the current super-chunk.
__device__ __forceinline__ void super_flush(const ScanArgs &a, uint64_t i, uint64_t v)
{
    if (v) atomicAdd(reinterpret_cast<unsigned long long *>(a.super + i), (unsigned long long)v);
}
__device__ __forceinline__ void super_add(const ScanArgs &a, uint64_t t, uint32_t tot, uint64_t &i,
                                          uint64_t &v)
{
    const uint64_t k = t >> SUPER_SHIFT;
    if (k != i) {
        super_flush(a, i, v);
        i = k;
        v = 0;
    }
    if (tot) v += (1ull << SUPER_NZ_SHIFT) | tot;
}

// What the count kernel keeps besides the per-tile counts (find mode: each
// tile with 1..STASH_K hits also stashes its hits' offsets).
enum CountMode {
    CM_COUNT = 0,  // counts only
    CM_FIND = 1,   // stash tiles are scanned again into the stash
    CM_CAP = 2,    // Shift-And, L = 16, sparse tiles expected: lanes keep their first LANE_K hits
    CM_BITS = 3,   // Shift-And or brute force, L >= 32: lanes keep hit bitmaps; the bitmaps of tiles with
                   // more than STASH_K hits go to the emit pass, the others fill the stash
};

// Count kernel: per-tile counts go to tile_cnt (the tile-count scan then sums
// them: one atomic per workgroup on a single address would serialize).
// A workgroup owns tiles_per_wg consecutive tiles. PREFETCH: the next tile's
// loads are in flight while the current tile is scanned (costs registers);
// otherwise each tile is loaded after the previous one is done. Each mode is a
// kernel of its own: a mode's registers do not weigh on the others.
template <int ALGO, int L, int VAR, int MODE, bool PREFETCH>
__device__ __forceinline__ void count_body(const ScanArgs &a)
{
    using G = Geometry<ALGO, L>;
    static_assert(MODE == CM_COUNT || MODE == CM_FIND || mask_hits(ALGO), "hit masks come from Shift-And or brute force");
    static_assert(MODE != CM_CAP || ALGO == ALGO_SHIFT_AND, "first-hit slots: Shift-And");
    static_assert(MODE != CM_BITS || L >= 32, "bitmaps take lanes of >= 32 starts");
    constexpr bool FIND = MODE != CM_COUNT;
    __shared__ TileShared<ALGO, L> S;
    const int m = (int)a.m;

    const uint64_t wg = xcd_remap(blockIdx.x, gridDim.x);
    const uint64_t t_begin = wg * a.tiles_per_wg;
    uint64_t t_end = t_begin + a.tiles_per_wg;
    if (t_end > a.ntiles) t_end = a.ntiles;

    // tile loads first, then the tables: one round trip for both
    Staged<G::PER> st;
    TileGeom g = tile_geom<ALGO, L>(a, t_begin);
    stage_issue(st, a.text, g.x0, g.x1);
    const uint4 tb = tables_issue<ALGO>(a.prm, a.hbits);
    const int sh1 = (int)a.prm->sh1;
    const int period = (int)a.prm->period;
    const int period_lb = (int)a.prm->period_lb;
    const BruteWords bw = brute_words<ALGO>(a.prm);
    tables_commit<ALGO, VAR>(tb, S.mask, S.shift, a.hbits);
    uint64_t sup_i = ~0ull, sup_v = 0;  // this workgroup's pending super-chunk total (thread 0)
    // suffix form: the pattern's first 1024 bytes, 16 per lane, for the candidates' checks
    uint4 ppre = {0u, 0u, 0u, 0u};
    if constexpr (ALGO == ALGO_SHIFT_AND && (VAR == 5 || VAR == 6)) {
        const uint32_t lane = threadIdx.x & 63;
        const uint32_t sfx = VAR == 6 ? (uint32_t)SA_SHORT : (uint32_t)SA_SUFFIX;
        if (16 * lane < a.m_full - sfx) ppre = reinterpret_cast<const uint4 *>(a.pat)[lane];
    }

    for (uint64_t t = t_begin; t < t_end; t++) {
        if (!PREFETCH && t != t_begin) {
            g = tile_geom<ALGO, L>(a, t);
            stage_issue(st, a.text, g.x0, g.x1);
        }
        __syncthreads();  // previous tile's LDS readers are done
        stage_commit<swz_tile(ALGO)>(st, S.text);
        const TileGeom cur = g;
        const int li0 = st.boff - cur.r0;
        __syncthreads();
        if (PREFETCH && t + 1 < t_end) {  // the next tile's loads overlap this tile's scan
            g = tile_geom<ALGO, L>(a, t + 1);
            stage_issue(st, a.text, g.x0, g.x1);
        }
        const int lo = threadIdx.x * L;
        const int hi = (lo + L - 1) < cur.hi_rel ? (lo + L - 1) : cur.hi_rel;
        const bool full = cur.hi_rel >= G::T - 1;  // every lane has L starts (uniform)
        constexpr int NW = L > 64 ? L / 64 : 1;
        uint32_t c;
        [[maybe_unused]] CapEmit ce;
        [[maybe_unused]] BitAcc<NW> ba;
        if constexpr (MODE == CM_BITS) {
            c = run_lane<ALGO, L, VAR, false>(S, a, m, sh1, period, period_lb, cur.s, li0, lo, hi, ba, bw, ppre,
                                              full);
        } else if constexpr (MODE == CM_CAP) {
            run_lane<ALGO, L, VAR, true>(S, a, m, sh1, period, period_lb, cur.s, li0, lo, hi, ce, bw, ppre, full);
            c = ce.n;
        } else {
            NoEmit ne;
            c = run_lane<ALGO, L, VAR, false>(S, a, m, sh1, period, period_lb, cur.s, li0, lo, hi, ne, bw, ppre,
                                              full);
        }
        uint32_t tot;
        const uint32_t before = block_excl_scan(c, S.w, tot);
        if (threadIdx.x == 0) {
            a.tile_cnt[t] = tot;
            super_add(a, t, tot, sup_i, sup_v);
        }
        if constexpr (MODE == CM_BITS) {
            if (tot > STASH_K) {  // uniform: the tile's bitmap for the emit pass
                uint32_t *dst = a.bits + t * (uint64_t)(G::T / 32) + threadIdx.x * (L / 32);
                if (L == 32) {
                    *dst = (uint32_t)ba.w[0];
                } else {
#pragma unroll
                    for (int k = 0; k < NW; k++)
                        reinterpret_cast<uint64_t *>(dst)[k] = ba.w[k];
                }
            } else if (tot) {  // uniform: stash from the bitmap
                uint16_t *dst = a.stash + t * STASH_K;
                uint32_t k = before;
#pragma unroll
                for (int i = 0; i < NW; i++) {
                    uint64_t x = ba.w[i];
                    while (x) {
                        dst[k++] = (uint16_t)(lo + 64 * i + __builtin_ctzll(x));
                        x &= x - 1;
                    }
                }
            }
        } else if constexpr (FIND) {
            if (tot && tot <= STASH_K) {  // uniform
                uint16_t *dst = a.stash + t * STASH_K;
                if (MODE == CM_CAP && !__syncthreads_or(c > LANE_K)) {
                    for (uint32_t k = 0; k < c; k++) dst[before + k] = ce.get(k);
                } else {  // scan again into the stash
                    StashEmit se;
                    se.dst = dst;
                    se.idx = before;
                    run_lane<ALGO, L, VAR, true>(S, a, m, sh1, period, period_lb, cur.s, li0, lo, hi, se, bw);
                }
            }
        }
    }
    if (threadIdx.x == 0) super_flush(a, sup_i, sup_v);
}

template <int ALGO, int L, int VAR, int MODE, bool PREFETCH>
__global__ __launch_bounds__(BLOCK) void count_kernel(ScanArgs a)
{
    count_body<ALGO, L, VAR, MODE, PREFETCH>(a);
}

// Shift-And with byte or 32-bit masks (m <= 17) at 64 starts per lane, one tile per
// workgroup: its LDS lets eight workgroups share a CU, and held to 64 VGPRs (without
// spilling) eight waves per SIMD fit too -- more tiles' loads in flight. Measured on
// MI355X at n = 2^30, sigma = 2: m = 8 count pass 214 -> 202 us, m = 4 226 -> 219 us.
template <int ALGO, int L, int VAR, int MODE>
constexpr bool eight_waves()
{
    return ALGO == ALGO_SHIFT_AND && L == 64 && (VAR == 4 || VAR == 0) && MODE != CM_CAP;
}
template <int ALGO, int L, int VAR, int MODE>
__global__ __launch_bounds__(BLOCK, 8) void count_kernel_w8(ScanArgs a)
{
    count_body<ALGO, L, VAR, MODE, false>(a);
}

template <int ALGO, int L, int VAR, int MODE>
void launch_count_kernel(const ScanArgs &a, uint32_t grid, hipStream_t st)
{
    if (a.tiles_per_wg > 1)
        hipLaunchKernelGGL((count_kernel<ALGO, L, VAR, MODE, true>), dim3(grid), dim3(BLOCK), 0, st, a);
    else if constexpr (eight_waves<ALGO, L, VAR, MODE>())
        hipLaunchKernelGGL((count_kernel_w8<ALGO, L, VAR, MODE>), dim3(grid), dim3(BLOCK), 0, st, a);
    else
        hipLaunchKernelGGL((count_kernel<ALGO, L, VAR, MODE, false>), dim3(grid), dim3(BLOCK), 0, st, a);
}

// ---------------------------------------------------------------------------
// Emit pass helpers. Waves work independently on list entries: wave g of G
// takes entries g, g + G, g + 2G, ..., 64 at a time, one per lane, so their
// list, count and offset loads are in flight together.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lane_u32(uint32_t v, int k)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, k);
}
__device__ __forceinline__ uint64_t lane_u64(uint64_t v, int k)
{
    return ((uint64_t)lane_u32((uint32_t)(v >> 32), k) << 32) | lane_u32((uint32_t)v, k);
}

// One batch of a wave's list entries: entry base + lane * G.
struct EmitBatch {
    uint32_t t = 0, cnt = 0;  // tile, its hits
    uint64_t off = 0;         // its first hit number
    uint64_t stash = 0;       // lanes whose tile overlaps the window and uses its stash
    uint64_t dense = 0;       // lanes whose tile overlaps the window and has more hits
};

__device__ __forceinline__ EmitBatch emit_batch(const ScanArgs &a, uint64_t base, uint64_t G, uint64_t nl)
{
    EmitBatch b;
    const uint64_t e = base + (uint64_t)(threadIdx.x & 63) * G;
    if (e < nl) {
        const TileEntry x = a.list[e];
        b.t = x.t;
        b.cnt = x.cnt;
        b.off = x.off;
    }
    const bool in_win = b.cnt && b.off < a.lo + a.cap && b.off + b.cnt > a.lo;
    b.stash = __ballot(in_win && b.cnt <= STASH_K);
    b.dense = __ballot(in_win && b.cnt > STASH_K);
    return b;
}

// The batch's stash tiles (tile-relative starts) to their offsets: four tiles
// at a time, 16 lanes each, every load of the four issued before any store. A
// lane reads 16-byte pieces (eight entries) at entries 8 sub and 8 sub + 128.
__device__ __forceinline__ void emit_stash_batch(const ScanArgs &a, const EmitBatch &b, uint64_t T)
{
    static_assert(STASH_K == 256, "two 128-entry halves per tile");
    uint64_t sm_ = b.stash;
    const uint32_t lane = threadIdx.x & 63, q = lane >> 4, sub = lane & 15;
    while (sm_) {  // uniform
        // this lane group's tile: the q-th of the next four
        uint32_t ck = 0;
        uint64_t tk = 0, ok = 0;
#pragma unroll
        for (uint32_t g = 0; g < 4; g++) {
            if (!sm_) break;
            const int k = __builtin_ctzll(sm_);
            sm_ &= sm_ - 1;
            const uint32_t c = lane_u32(b.cnt, k);
            const uint64_t t = lane_u32(b.t, k), o = lane_u64(b.off, k);
            if (q == g) {
                ck = c;
                tk = t;
                ok = o;
            }
        }
        const uint4 *src = reinterpret_cast<const uint4 *>(a.stash + tk * STASH_K) + sub;
        uint4 v[2] = {{0u, 0u, 0u, 0u}, {0u, 0u, 0u, 0u}};
#pragma unroll
        for (int h = 0; h < 2; h++)
            if (8 * sub + 128 * h < ck) v[h] = src[16 * h];
        const uint64_t s = tk * T;
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const uint32_t w[4] = {v[h].x, v[h].y, v[h].z, v[h].w};
#pragma unroll
            for (int e = 0; e < 8; e++) {
                const uint32_t i = 8 * sub + 128 * h + e;
                const uint64_t r = ok + i - a.lo;
                if (i < ck && r < a.cap) a.out[r] = (int64_t)(s + ((w[e >> 1] >> (16 * (e & 1))) & 0xFFFFu));
            }
        }
    }
}

// Emit kernel: positions of the listed tiles, at their offsets, bounded by cap.
// Tiles with at most STASH_K hits copy their stash. Denser tiles are rescanned
// from LDS in sub-tiles of EMIT_SUB starts (16 per lane): one scan keeps each
// lane's hits in its own LDS slots, and a workgroup scan of the lanes' counts
// gives each lane its output offset. Lanes write their hits there themselves in
// sparse sub-tiles; dense ones are compacted in LDS and written coalesced.
template <int ALGO, int L, int VAR>
__global__ __launch_bounds__(BLOCK) void emit_kernel(ScanArgs a)
{
    constexpr int SUB_LANE = EMIT_SUB / BLOCK;
    __shared__ TileShared<ALGO, L> S;
    // SUB_LANE per lane: all of a lane's hits in a sub-tile
    __shared__ uint16_t s_list[EMIT_SUB];
    const int m = (int)a.m;
    const uint64_t nl = *a.nlist;
    if ((uint64_t)blockIdx.x >= nl) return;
    const int sh1 = (int)a.prm->sh1;
    const int period = (int)a.prm->period;
    const int period_lb = (int)a.prm->period_lb;
    const BruteWords bw = brute_words<ALGO>(a.prm);
    // 1. tiles with at most STASH_K hits: copy their stash (waves on their own)
    {
        const uint64_t G = (uint64_t)gridDim.x * (BLOCK / 64);
        const uint64_t g = (uint64_t)blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6);
        for (uint64_t base = g; base < nl; base += 64 * G)
            emit_stash_batch(a, emit_batch(a, base, G, nl), (uint64_t)Geometry<ALGO, L>::T);
    }
    // 2. denser tiles, rescanned from LDS: the workgroup's entries blockIdx.x +
    // k gridDim.x are examined BLOCK at a time, one per thread, and the dense
    // ones listed in LDS in order
    __shared__ uint32_t s_dt[BLOCK];
    __shared__ uint64_t s_do[BLOCK];
    using G = Geometry<ALGO, L>;
    bool tables = false;
    for (uint64_t base = blockIdx.x; base < nl; base += (uint64_t)BLOCK * gridDim.x) {  // uniform
        const uint64_t e0 = base + (uint64_t)threadIdx.x * gridDim.x;
        TileEntry x{0u, 0u, 0ull};
        if (e0 < nl) x = a.list[e0];
        const uint32_t d = (x.cnt > STASH_K && x.off < a.lo + a.cap && x.off + x.cnt > a.lo) ? 1u : 0u;
        uint32_t nd;
        const uint32_t at = block_excl_scan(d, S.w, nd);  // ends with a barrier
        if (nd == 0) continue;  // uniform
        if (d) {
            s_dt[at] = x.t;
            s_do[at] = x.off;
        }
        if (!tables) {  // read by the scans after the next barrier
            const uint4 tb = tables_issue<ALGO>(a.prm, a.hbits);
            tables_commit<ALGO, VAR>(tb, S.mask, S.shift, a.hbits);
            tables = true;
        }
        __syncthreads();
        for (uint32_t kd = 0; kd < nd; kd++) {
            const uint64_t t = s_dt[kd];
            const uint64_t off = s_do[kd];
            const TileGeom cur = tile_geom<ALGO, L>(a, t);
            Staged<G::PER> st;
            stage_issue(st, a.text, cur.x0, cur.x1);
            __syncthreads();  // the previous tile's LDS readers are done
            stage_commit<swz_tile(ALGO)>(st, S.text);
            const int li0 = st.boff - cur.r0;
            __syncthreads();
            const uint64_t s2 = cur.s;
            const int hi_rel = cur.hi_rel;
            uint64_t run = off;
            for (int sb = 0; sb <= hi_rel && run < a.lo + a.cap; sb += EMIT_SUB) {  // uniform
                const int lo = sb + SUB_LANE * (int)threadIdx.x;
                const int hi = (lo + SUB_LANE - 1) < hi_rel ? (lo + SUB_LANE - 1) : hi_rel;
                // one scan: each lane keeps its hits (at most one per start) in its slots
                ListEmit se;
                se.dst = s_list + SUB_LANE * threadIdx.x;
                se.idx = 0;
                run_lane<ALGO, L, VAR, true>(S, a, m, sh1, period, period_lb, s2, li0, lo, hi, se, bw);
                const uint32_t c = se.idx;
                uint32_t ctot;
                const uint32_t before = block_excl_scan(c, S.w, ctot);  // ends with a barrier
                if (ctot == 0) continue;  // uniform
                if (run + ctot <= a.lo) {  // sub-tile entirely before the window (uniform)
                    run += ctot;
                    continue;
                }
                if (ctot <= (uint32_t)(EMIT_SUB / 8)) {  // uniform
                    // sparse: each lane writes its hits at its offset (a wave's stores of one
                    // slot index land on neighbouring lines and are merged in L2)
                    for (uint32_t k = 0; k < c; k++) {
                        const uint64_t r = run + before + k - a.lo;
                        if (r < a.cap) a.out[r] = (int64_t)(s2 + s_list[SUB_LANE * threadIdx.x + k]);
                    }
                } else {
                    // dense: the lanes' hits compacted in place, then written coalesced
                    uint16_t v[SUB_LANE];
#pragma unroll
                    for (int k = 0; k < SUB_LANE; k++) v[k] = (uint32_t)k < c ? s_list[SUB_LANE * threadIdx.x + k] : 0;
                    __syncthreads();
#pragma unroll
                    for (int k = 0; k < SUB_LANE; k++)
                        if ((uint32_t)k < c) s_list[before + k] = v[k];
                    __syncthreads();
                    for (uint32_t k = threadIdx.x; k < ctot; k += BLOCK) {
                        const uint64_t r = run + k - a.lo;
                        if (r < a.cap) a.out[r] = (int64_t)(s2 + s_list[k]);
                    }
                    __syncthreads();
                }
                run += ctot;
            }
        }
        __syncthreads();  // s_dt / s_do are read before the next batch writes them
    }
}

// ---------------------------------------------------------------------------
// Block filter kernels. A tile is 256 sampled blocks, one per lane: lane l of
// tile t tests block b = 256 t + l at x = b S + S - 1 - phi for the starts
// [b S - phi, b S + S - phi) (from 0 on), where S is a multiple of 16 and phi in
// [0, 15] puts every sampled block on an aligned 16-byte chunk of memory. Only the
// sampled blocks are read from the text (plus the bytes of candidates).
// ---------------------------------------------------------------------------
struct BlockLane {
    uint64_t x, ilo, ihi;  // the block, and the starts it owns (ilo > ihi: none)
};

__device__ __forceinline__ BlockLane block_lane(const ScanArgs &a, uint64_t t)
{
    BlockLane L;
    const uint64_t S = a.bs, b = t * BLOCK + threadIdx.x;
    const uint64_t phi = ((uint64_t)(uintptr_t)a.text + 15) & 15;  // text + x is 16-byte aligned
    L.x = b * S + S - 1 - phi;  // >= 0: S >= 16
    L.ilo = b * S >= phi ? b * S - phi : 0;
    const uint64_t last = a.n - a.m;  // n >= m
    L.ihi = L.x < last ? L.x : last;
    return L;
}

// the sampled block: one aligned chunk
__device__ __forceinline__ uint4 block_load(const ScanArgs &a, const BlockLane &L)
{
    return L.ilo <= L.ihi ? *reinterpret_cast<const uint4 *>(a.text + L.x) : uint4{0u, 0u, 0u, 0u};
}

// Count pass (count and find modes alike: the emit pass tests the tiles with hits
// again). PREFETCH: the next tile's blocks are loaded while this tile's are tested.
template <bool PREFETCH>
__global__ __launch_bounds__(BLOCK) void block_count_kernel(ScanArgs a)
{
    __shared__ uint32_t s_w[BLOCK / 64];
    const uint64_t wg = xcd_remap(blockIdx.x, gridDim.x);
    const uint64_t t_begin = wg * a.tiles_per_wg;
    uint64_t t_end = t_begin + a.tiles_per_wg;
    if (t_end > a.ntiles) t_end = a.ntiles;
    const uint32_t period = a.prm->period, period_lb = a.prm->period_lb;
    uint64_t sup_i = ~0ull, sup_v = 0;
    BlockLane L = block_lane(a, t_begin);
    uint4 blk = block_load(a, L);
    for (uint64_t t = t_begin; t < t_end; t++) {
        if (!PREFETCH && t != t_begin) {
            L = block_lane(a, t);
            blk = block_load(a, L);
        }
        const BlockLane cur = L;
        const uint4 cb = blk;
        if (PREFETCH && t + 1 < t_end) {
            L = block_lane(a, t + 1);
            blk = block_load(a, L);
        }
        NoEmit ne;
        const uint32_t c = lane_block<false>(a.text, a.pat, a.m, a.prm, period, period_lb, cur.x,
                                             cur.ilo, cur.ihi, cb, cur.ilo <= cur.ihi, 0, ne);
        uint32_t tot;
        block_excl_scan(c, s_w, tot);
        if (threadIdx.x == 0) {
            a.tile_cnt[t] = tot;
            super_add(a, t, tot, sup_i, sup_v);
        }
    }
    if (threadIdx.x == 0) super_flush(a, sup_i, sup_v);
}

// Emit pass: every listed tile is tested again, once to count each lane's hits
// (their workgroup scan places the lanes) and once to write them.
__global__ __launch_bounds__(BLOCK) void block_emit_kernel(ScanArgs a)
{
    __shared__ uint32_t s_w[BLOCK / 64];
    const uint64_t nl = *a.nlist;
    const uint32_t period = a.prm->period, period_lb = a.prm->period_lb;
    const uint64_t T = (uint64_t)BLOCK * a.bs;
    for (uint64_t e = blockIdx.x; e < nl; e += gridDim.x) {  // uniform
        const TileEntry te = a.list[e];
        if (te.off >= a.lo + a.cap || te.off + te.cnt <= a.lo) continue;  // outside the window
        const BlockLane L = block_lane(a, te.t);
        const bool any = L.ilo <= L.ihi;
        const uint4 blk = block_load(a, L);
        NoEmit ne;
        const uint32_t c = lane_block<false>(a.text, a.pat, a.m, a.prm, period, period_lb, L.x, L.ilo,
                                             L.ihi, blk, any, 0, ne);
        uint32_t tot;
        const uint32_t before = block_excl_scan(c, s_w, tot);
        PosEmit pe;
        pe.out = a.out;
        pe.idx = te.off + before;
        pe.lo = a.lo;
        pe.span = a.cap;
        pe.base = te.t * T;
        lane_block<true>(a.text, a.pat, a.m, a.prm, period, period_lb, L.x, L.ilo, L.ihi, blk, c != 0,
                         te.t * T, pe);
    }
}

// LDS writes of one lane are seen by the other lanes of its wave after this
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// inclusive scan over the 64 lanes of a wave: DPP row shifts build the scan of
// each row of 16 lanes, then the row broadcasts add the rows before it
__device__ __forceinline__ uint32_t wave_scan_dpp(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, true);   // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, true);   // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, true);   // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, true);   // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return v;
}

// Emit kernel of the bitmap form (dense Shift-And tiles, L >= 32): the count
// pass left each dense tile's hits as a bitmap of its T starts (64-bit words in
// start order) and each sparse tile's in its stash. Waves work independently:
// wave g of G takes list entries g, g + G, g + 2G, ..., 64 at a time (one per
// lane, so their list, count and offset loads are in flight together). A stash
// tile is copied by the whole wave, the next one's loads issued before this
// one's stores. A dense tile is expanded 64 words (4096 starts) per round: a
// wave scan of the words' bit counts places each lane's starts in the wave's
// LDS list, which is copied to the output coalesced whenever the next round
// might not fit, and at the tile's end; the next dense tile's words are loaded
// meanwhile. The text is not read again.
template <int L>
__global__ __launch_bounds__(BLOCK) void emit_bits_kernel(ScanArgs a)
{
    constexpr int T = BLOCK * L;
    constexpr int R = T / 64 / 64;  // rounds of 64 words per tile
    constexpr int LIST = 64 * 64;   // a round's starts at most
    static_assert(T <= 65536 && R >= 1, "tile-relative starts are kept as u16");
    __shared__ uint16_t s_list[BLOCK / 64][LIST];
    const uint64_t nl = *a.nlist;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint64_t G = (uint64_t)gridDim.x * (BLOCK / 64);
    const uint64_t g = (uint64_t)blockIdx.x * (BLOCK / 64) + (uint64_t)wv;
    uint16_t *lst = s_list[wv];
    const uint64_t *bits = reinterpret_cast<const uint64_t *>(a.bits);
    for (uint64_t base = g; base < nl; base += 64 * G) {  // uniform over the wave
        const EmitBatch bt = emit_batch(a, base, G, nl);
        emit_stash_batch(a, bt, (uint64_t)T);
        uint64_t dm = bt.dense;
        // denser tiles: expand their bitmaps
        if (dm) {
            int k = __builtin_ctzll(dm);
            dm &= dm - 1;
            uint64_t tk = lane_u32(bt.t, k), ok = lane_u64(bt.off, k);
            uint64_t x[R];
#pragma unroll
            for (int r = 0; r < R; r++) x[r] = bits[tk * (uint64_t)(T / 64) + r * 64 + lane];
            for (;;) {
                const bool more = dm != 0;
                uint64_t tk2 = 0, ok2 = 0;
                uint64_t x2[R];
                if (more) {  // the next dense tile's words are loaded during this one
                    const int k2 = __builtin_ctzll(dm);
                    dm &= dm - 1;
                    tk2 = lane_u32(bt.t, k2);
                    ok2 = lane_u64(bt.off, k2);
#pragma unroll
                    for (int r = 0; r < R; r++) x2[r] = bits[tk2 * (uint64_t)(T / 64) + r * 64 + lane];
                }
                const uint64_t s = tk * (uint64_t)T;
                uint64_t run = ok;   // hit number of the list's first entry
                uint32_t fill = 0;   // entries in the list
#pragma unroll
                for (int r = 0; r < R; r++) {
                    const uint32_t pc = (uint32_t)__builtin_popcountll(x[r]);
                    const uint32_t incl = wave_scan_dpp(pc);
                    const uint32_t rt = lane_u32(incl, 63);  // this round's starts
                    if (fill + rt > (uint32_t)LIST) {  // uniform: flush first
                        wave_lds_sync();
                        for (uint32_t i = lane; i < fill; i += 64) {
                            const uint64_t o = run + i - a.lo;
                            if (o < a.cap) a.out[o] = (int64_t)(s + lst[i]);
                        }
                        run += fill;
                        fill = 0;
                        wave_lds_sync();  // read before it is written again
                    }
                    uint32_t kk = fill + incl - pc;
                    const int b0 = (r * 64 + lane) * 64;
                    uint64_t y = x[r];
                    while (y) {
                        lst[kk++] = (uint16_t)(b0 + __builtin_ctzll(y));
                        y &= y - 1;
                    }
                    fill += rt;
                }
                wave_lds_sync();
                for (uint32_t i = lane; i < fill; i += 64) {
                    const uint64_t o = run + i - a.lo;
                    if (o < a.cap) a.out[o] = (int64_t)(s + lst[i]);
                }
                wave_lds_sync();
                if (!more) break;
                tk = tk2;
                ok = ok2;
#pragma unroll
                for (int r = 0; r < R; r++) x[r] = x2[r];
            }
        }
    }
}

// Tile-count scan, SCAN_CHUNK tiles per workgroup of 1024 threads and no waiting
// between workgroups: workgroup w first sums the super-chunk totals before its
// chunk itself (one per 64 tiles, eight loads in flight per thread), then scans
// its chunk, SCAN_CHUNK / 1024 consecutive counts per thread.
// Writes the ascending list of tiles with hits (with counts and offsets); the last
// workgroup writes the total and the list length. With list == null only the
// total is produced (count mode).
__device__ __forceinline__ uint4 load_cnt4(const uint32_t *cnt, uint64_t i, uint64_t nt)
{
    if (i + 3 < nt) return *reinterpret_cast<const uint4 *>(cnt + i);
    uint4 r = {0u, 0u, 0u, 0u};
    if (i < nt) r.x = cnt[i];
    if (i + 1 < nt) r.y = cnt[i + 1];
    if (i + 2 < nt) r.z = cnt[i + 2];
    return r;
}

// workgroup-wide sums of (a, b) over 1024 threads (16 waves)
__device__ __forceinline__ void block_sum2_1024(uint64_t &a, uint32_t &b, uint64_t *s_a, uint32_t *s_b)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        a += __shfl_xor(a, d, 64);
        b += __shfl_xor(b, d, 64);
    }
    if (lane == 0) {
        s_a[wv] = a;
        s_b[wv] = b;
    }
    __syncthreads();
    a = 0;
    b = 0;
#pragma unroll
    for (int k = 0; k < 16; k++) {
        a += s_a[k];
        b += s_b[k];
    }
    __syncthreads();
}

__global__ __launch_bounds__(1024) void tile_scan_kernel(const uint32_t *cnt, const uint64_t *super,
                                                         uint64_t nt, uint64_t *total, TileEntry *list,
                                                         uint64_t *nlist)
{
    __shared__ uint64_t s_a[16];
    __shared__ uint32_t s_b[16];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const uint64_t c0 = (uint64_t)blockIdx.x * SCAN_CHUNK;
    // this chunk's counts, SCAN_CHUNK / 1024 consecutive ones per thread, loaded first so
    // that they are in flight with the super-chunk totals below
    constexpr int PER = (int)(SCAN_CHUNK / 1024);
    static_assert(PER % 4 == 0, "whole 16-byte loads");
    const uint64_t i = c0 + PER * (uint64_t)tid;
    uint32_t c[PER];
#pragma unroll
    for (int k = 0; k < PER / 4; k++) {
        const uint4 v = load_cnt4(cnt, i + 4 * k, nt);
        c[4 * k] = v.x;
        c[4 * k + 1] = v.y;
        c[4 * k + 2] = v.z;
        c[4 * k + 3] = v.w;
    }
    // 1. occurrences and listed tiles before this chunk, from the super-chunk totals
    static_assert(SCAN_CHUNK % (1ull << SUPER_SHIFT) == 0, "chunks of whole super-chunks");
    uint64_t pre = 0;
    uint32_t pnz = 0;
    const uint64_t s0 = c0 >> SUPER_SHIFT;
    for (uint64_t i0 = 0; i0 < s0; i0 += 8 * 1024) {
        uint64_t v[8];
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const uint64_t i = i0 + (uint64_t)tid + 1024 * k;
            v[k] = i < s0 ? super[i] : 0ull;
        }
#pragma unroll
        for (int k = 0; k < 8; k++) {
            pre += v[k] & ((1ull << SUPER_NZ_SHIFT) - 1);
            pnz += (uint32_t)(v[k] >> SUPER_NZ_SHIFT);
        }
    }
    block_sum2_1024(pre, pnz, s_a, s_b);
    // 2. this chunk's scan
    uint64_t my = 0;
    uint32_t mz = 0;
#pragma unroll
    for (int k = 0; k < PER; k++) {
        my += c[k];
        mz += c[k] != 0;
    }
    uint64_t incl = my;
    uint32_t zincl = mz;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint64_t o = __shfl_up(incl, d, 64);
        const uint32_t p = __shfl_up(zincl, d, 64);
        if (lane >= d) {
            incl += o;
            zincl += p;
        }
    }
    if (lane == 63) {
        s_a[wv] = incl;
        s_b[wv] = zincl;
    }
    __syncthreads();
    uint64_t wb = 0, ctot = 0;
    uint32_t zb = 0, ztot = 0;
#pragma unroll
    for (int k = 0; k < 16; k++) {
        wb += (k < wv) ? s_a[k] : 0;
        zb += (k < wv) ? s_b[k] : 0;
        ctot += s_a[k];
        ztot += s_b[k];
    }
    if (list) {
        uint64_t o = pre + wb + incl - my;
        uint64_t zp = pnz + zb + zincl - mz;
#pragma unroll
        for (int k = 0; k < PER; k++) {
            if (i + k < nt && c[k]) {
                TileEntry x;
                x.t = (uint32_t)(i + k);
                x.cnt = c[k];
                x.off = o;
                list[zp++] = x;
            }
            o += c[k];
        }
    }
    if (tid == 0 && blockIdx.x == gridDim.x - 1) {
        *total = pre + ctot;
        if (nlist) *nlist = pnz + ztot;
    }
}

// ---------------------------------------------------------------------------
// Prep kernel: one workgroup builds the tables for one pattern.
// ---------------------------------------------------------------------------
struct PrepArgs {
    Params *prm;
    uint8_t *pat;      // destination of the pattern in the workspace
    uint64_t *zero;    // set to 0 (the running total), may be null
    uint64_t *super;   // super-chunk totals to zero (nsuper of them)
    uint64_t nsuper;
    uint32_t m, algo, q, hbits;
    uint32_t inline_len;  // pattern bytes carried below (0: already in pat)
    alignas(4) uint8_t inline_pat[PREP_INLINE];
};

__global__ __launch_bounds__(BLOCK) void prep_kernel(PrepArgs a)
{
    __shared__ uint32_t s_tab[1 << H_MAX];
    __shared__ __align__(16) uint8_t s_pat[PREP_INLINE];
    const int tid = threadIdx.x;
    const uint32_t m = a.m;
    Params *P = a.prm;

    if (a.inline_len) {
        // whole words (the argument block is word aligned), every load issued before
        // any store: at most PREP_INLINE / 4 / BLOCK words per thread; the words past
        // the pattern are zeroed, and the copy is zero padded to a multiple of 16
        constexpr int WPT = PREP_INLINE / 4 / BLOCK;
        static_assert(PREP_INLINE % (4 * BLOCK) == 0, "whole words per thread");
        const uint32_t nw = (a.inline_len + 3) / 4;
        const uint32_t *src = reinterpret_cast<const uint32_t *>(a.inline_pat);
        uint32_t w[WPT];
#pragma unroll
        for (int u = 0; u < WPT; u++) {
            const uint32_t k = tid + BLOCK * u;
            w[u] = k < nw ? src[k] : 0u;
            if (k == nw - 1 && (a.inline_len & 3)) w[u] &= (1u << (8 * (a.inline_len & 3))) - 1u;
        }
        uint32_t *s_pat32 = reinterpret_cast<uint32_t *>(s_pat);
        uint32_t *dst32 = reinterpret_cast<uint32_t *>(a.pat);  // 16-byte aligned in the workspace
        const uint32_t padw = ((m + 15) & ~15u) / 4;
#pragma unroll
        for (int u = 0; u < WPT; u++) {
            const uint32_t k = tid + BLOCK * u;
            if (k < nw) s_pat32[k] = w[u];
            if (k < padw) dst32[k] = w[u];
        }
    }
    for (uint64_t k = tid; k < a.nsuper; k += BLOCK) a.super[k] = 0;
    if (tid == 0) {
        P->m = m;
        P->algo = a.algo;
        P->q = a.q;
        P->hbits = a.hbits;
        if (a.zero) *a.zero = 0;
    }
    __syncthreads();
    // pattern bytes: from LDS when inline, else from the workspace copy
    // (two calls: each reads its pattern copy through its own address space, LDS
    // reads rather than generic ones for the inline copy)
    __shared__ uint32_t s_bad[PERIOD_MAX + 1];
    __shared__ __align__(16) uint32_t s_key[BF_BUILD_LDS];
    // SBNDM's factor form (m > 64): masks and period of the pattern's last 64 bytes
    const uint32_t fo = (a.algo == ALGO_SBNDM && m > (uint32_t)BP_MAX_M) ? m - BP_MAX_M : 0u;
    if (a.inline_len) build_tables(s_pat + fo, m - fo, a.algo, a.q, a.hbits, P, s_tab, s_bad, s_key);
    else build_tables(a.pat + fo, m - fo, a.algo, a.q, a.hbits, P, s_tab, s_bad, s_key);
}

__global__ void set_u64_kernel(uint64_t *dst, uint64_t v) { *dst = v; }

// 256-bin byte histogram (alphabet probe).
__global__ __launch_bounds__(BLOCK) void hist_kernel(const uint8_t *text, uint64_t n, uint64_t *hist)
{
    __shared__ uint32_t s_h[256];
    s_h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * BLOCK;
    for (uint64_t i = (uint64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += stride)
        atomicAdd(&s_h[text[i]], 1u);
    __syncthreads();
    if (s_h[threadIdx.x]) atomicAdd((unsigned long long *)&hist[threadIdx.x], (unsigned long long)s_h[threadIdx.x]);
}

// ---------------------------------------------------------------------------
// dispatch helpers
// ---------------------------------------------------------------------------
enum Kind { K_COUNT, K_FIND_COUNT, K_EMIT };

template <int ALGO, int L, int VAR, int KIND>
hipError_t launch_t(const ScanArgs &a, uint32_t grid, hipStream_t st)
{
    if (grid == 0) return hipSuccess;
    if (KIND == K_COUNT) {
        launch_count_kernel<ALGO, L, VAR, CM_COUNT>(a, grid, st);
    } else if (KIND == K_FIND_COUNT) {
        // Shift-And: hit bitmaps, else (16-byte lanes) the lanes' first hits when sparse
        // tiles are expected (the workspace has no bitmap region for m > 64)
        if constexpr (mask_hits(ALGO)) {
            if (L >= 32 && a.bits) {
                constexpr int LB = L >= 32 ? L : 32;
                launch_count_kernel<ALGO, LB, VAR, CM_BITS>(a, grid, st);
                return hipGetLastError();
            }
        }
        if constexpr (ALGO == ALGO_SHIFT_AND) {
            if (a.slots) {
                launch_count_kernel<ALGO, L, VAR, CM_CAP>(a, grid, st);
                return hipGetLastError();
            }
        }
        launch_count_kernel<ALGO, L, VAR, CM_FIND>(a, grid, st);
    } else if (mask_hits(ALGO) && L >= 32 && a.bits)
        hipLaunchKernelGGL((emit_bits_kernel<L >= 32 ? L : 32>), dim3(grid), dim3(BLOCK), 0, st, a);
    else
        hipLaunchKernelGGL((emit_kernel<ALGO, L, VAR>), dim3(grid), dim3(BLOCK), 0, st, a);
    return hipGetLastError();
}

template <int ALGO, int VAR, int KIND>
hipError_t launch_l(const Plan &p, const ScanArgs &a, uint32_t grid, hipStream_t st)
{
    switch (p.lane_bytes) {
    case 16: return launch_t<ALGO, 16, VAR, KIND>(a, grid, st);
    case 32: return launch_t<ALGO, 32, VAR, KIND>(a, grid, st);
    case 64: return launch_t<ALGO, 64, VAR, KIND>(a, grid, st);
    case 128: return launch_t<ALGO, 128, VAR, KIND>(a, grid, st);
    default: return hipErrorInvalidValue;
    }
}

template <int KIND>
hipError_t launch_any(const Plan &p, const ScanArgs &a, uint32_t grid, hipStream_t st)
{
    switch (p.algo) {
    case ALGO_SHIFT_AND: {
        const int m = (int)p.m;
        // variants: 4 = 32-bit state, byte masks (m <= 8); 0 = 32-bit state and masks;
        // 1 = 64-bit state, hits checked every 16 bytes (m <= 49); 5 = m > 49: the last
        // SA_SUFFIX bytes scanned as variant 1 does, the rest verified (faster than
        // checking hits every 4 or every byte, which m = 50..64 would need); 6 = the same
        // with the last SA_SHORT bytes scanned as variant 0 does (the plan's choice)
        static_assert(SA_SUFFIX == 49, "variant 1 covers m <= 49");
        if (m > SA_SUFFIX) {
            if (p.sfx == SA_SHORT) return launch_l<ALGO_SHIFT_AND, 6, KIND>(p, a, grid, st);
            return launch_l<ALGO_SHIFT_AND, 5, KIND>(p, a, grid, st);
        }
        if (m <= 8) return launch_l<ALGO_SHIFT_AND, 4, KIND>(p, a, grid, st);
        if (m <= 17) return launch_l<ALGO_SHIFT_AND, 0, KIND>(p, a, grid, st);
        return launch_l<ALGO_SHIFT_AND, 1, KIND>(p, a, grid, st);
    }
    case ALGO_BNDM:
        if (p.q == 2) return launch_l<ALGO_BNDM, 1, KIND>(p, a, grid, st);
        if (p.q == 4) return launch_l<ALGO_BNDM, 2, KIND>(p, a, grid, st);
        return launch_l<ALGO_BNDM, 0, KIND>(p, a, grid, st);
    case ALGO_FSBNDM: return launch_l<ALGO_FSBNDM, 0, KIND>(p, a, grid, st);
    case ALGO_BRUTE: return launch_l<ALGO_BRUTE, 0, KIND>(p, a, grid, st);
    case ALGO_SBNDM:  // variants 0..3: q = 1, 2, 4, 8; 4..7: the same, factor form (m > 64)
        if (p.m > (uint64_t)BP_MAX_M) {
            if (p.q <= 1) return launch_l<ALGO_SBNDM, 4, KIND>(p, a, grid, st);
            if (p.q == 2) return launch_l<ALGO_SBNDM, 5, KIND>(p, a, grid, st);
            if (p.q == 4) return launch_l<ALGO_SBNDM, 6, KIND>(p, a, grid, st);
            return launch_l<ALGO_SBNDM, 7, KIND>(p, a, grid, st);
        }
        if (p.q <= 1) return launch_l<ALGO_SBNDM, 0, KIND>(p, a, grid, st);
        if (p.q == 2) return launch_l<ALGO_SBNDM, 1, KIND>(p, a, grid, st);
        if (p.q == 4) return launch_l<ALGO_SBNDM, 2, KIND>(p, a, grid, st);
        return launch_l<ALGO_SBNDM, 3, KIND>(p, a, grid, st);
    case ALGO_HASHQ: {
        const int nw = (p.q + 3) / 4;
        if (nw <= 1) return launch_l<ALGO_HASHQ, 1, KIND>(p, a, grid, st);
        if (nw == 2) return launch_l<ALGO_HASHQ, 2, KIND>(p, a, grid, st);
        if (nw == 3) return launch_l<ALGO_HASHQ, 3, KIND>(p, a, grid, st);
        return launch_l<ALGO_HASHQ, 4, KIND>(p, a, grid, st);
    }
    default: return hipErrorInvalidValue;
    }
}

ScanArgs make_args(const Plan &plan, const uint8_t *d_text, uint64_t n, const Params *d_params,
                   const uint8_t *d_pat, uint64_t ntiles)
{
    ScanArgs a;
    memset(&a, 0, sizeof a);
    a.text = d_text;
    a.n = n;
    a.prm = d_params;
    a.pat = d_pat;
    a.m = (uint32_t)plan.m;
    a.q = (uint32_t)plan.q;
    a.hbits = (uint32_t)plan.hbits;
    a.tiles_per_wg = (uint32_t)plan.tiles_per_wg;
    a.slots = (uint32_t)plan.slots;
    a.bs = plan.algo == ALGO_BLOCK ? (uint32_t)plan.lane_bytes : 0u;
    a.ntiles = ntiles;
    if (plan.algo == ALGO_SHIFT_AND && plan.m > (uint64_t)SA_SUFFIX) {  // suffix form (n >= m)
        const uint32_t sfx = plan.sfx == SA_SHORT ? (uint32_t)SA_SHORT : (uint32_t)SA_SUFFIX;
        const uint64_t sh = plan.m - sfx;
        a.text0 = d_text;
        a.m_full = (uint32_t)plan.m;
        if (plan.m <= (uint64_t)SA_STAGE_MAX) {  // whole windows in LDS
            a.sfx_off = (uint32_t)sh;
        } else {
            a.text = d_text + sh;
            a.n = n - sh;
            a.m = sfx;
        }
    }
    if (plan.algo == ALGO_SBNDM && plan.m > (uint64_t)BP_MAX_M) {  // factor form (n >= m)
        const uint64_t sh = plan.m - BP_MAX_M;
        a.text0 = d_text;
        a.m_full = (uint32_t)plan.m;
        a.text = d_text + sh;
        a.n = n - sh;
        a.m = BP_MAX_M;
    }
    return a;
}

uint32_t count_grid(const ScanArgs &a)
{
    const uint64_t nblk = (a.ntiles + a.tiles_per_wg - 1) / a.tiles_per_wg;
    return nblk > 0x7FFFFFFFull ? 0u : (uint32_t)nblk;
}

}  // namespace

hipError_t launch_prep(const Plan &plan, const uint8_t *pat_host, Params *d_params, uint8_t *d_pat,
                       uint64_t *d_zero, uint64_t *d_super, uint64_t nsuper, hipStream_t stream)
{
    PrepArgs a;
    a.prm = d_params;
    a.pat = d_pat;
    a.zero = d_zero;
    a.super = d_super;
    a.nsuper = d_super ? nsuper : 0;
    a.m = (uint32_t)plan.m;
    a.algo = (uint32_t)plan.algo;
    a.q = (uint32_t)plan.q;
    if (plan.algo == ALGO_SHIFT_AND && plan.m > (uint64_t)SA_SUFFIX)  // suffix masks
        a.q = plan.sfx == SA_SHORT ? (uint32_t)SA_SHORT : (uint32_t)SA_SUFFIX;
    a.hbits = (uint32_t)plan.hbits;
    if (plan.m <= PREP_INLINE) {
        a.inline_len = (uint32_t)plan.m;
        for (uint64_t k = 0; k < plan.m; k++) a.inline_pat[k] = pat_host[k];
    } else {
        a.inline_len = 0;
        const uint64_t padded = align_up(plan.m, 16);
        hipError_t e = hipMemcpyAsync(d_pat, pat_host, plan.m, hipMemcpyHostToDevice, stream);
        if (e != hipSuccess) return e;
        if (padded > plan.m) {
            e = hipMemsetAsync(d_pat + plan.m, 0, padded - plan.m, stream);
            if (e != hipSuccess) return e;
        }
    }
    hipLaunchKernelGGL(prep_kernel, dim3(1), dim3(BLOCK), 0, stream, a);
    return hipGetLastError();
}

static hipError_t launch_tile_scan(const FindWs &w, uint64_t *d_total, bool find, hipStream_t stream)
{
    const uint64_t nb = (w.ntiles + SCAN_CHUNK - 1) / SCAN_CHUNK;
    hipLaunchKernelGGL(tile_scan_kernel, dim3((uint32_t)nb), dim3(1024), 0, stream, w.tile_cnt,
                       (const uint64_t *)w.super, w.ntiles, d_total, find ? w.list : nullptr,
                       find ? w.nlist : nullptr);
    return hipGetLastError();
}

static hipError_t launch_block_count(const ScanArgs &a, uint32_t grid, hipStream_t st)
{
    if (a.tiles_per_wg > 1) hipLaunchKernelGGL(block_count_kernel<true>, dim3(grid), dim3(BLOCK), 0, st, a);
    else hipLaunchKernelGGL(block_count_kernel<false>, dim3(grid), dim3(BLOCK), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_count(const Plan &plan, const uint8_t *d_text, uint64_t n, const Params *d_params,
                        const uint8_t *d_pat, const FindWs &w, uint64_t *d_total, hipStream_t stream,
                        hipEvent_t after_count)
{
    if (w.ntiles == 0) return hipSuccess;
    if (w.ntiles > 0xFFFFFFFFull) return hipErrorInvalidValue;
    ScanArgs a = make_args(plan, d_text, n, d_params, d_pat, w.ntiles);
    a.tile_cnt = w.tile_cnt;
    a.super = w.super;
    const uint32_t g = count_grid(a);
    if (!g) return hipErrorInvalidValue;
    hipError_t e = plan.algo == ALGO_BLOCK ? launch_block_count(a, g, stream)
                                           : launch_any<K_COUNT>(plan, a, g, stream);
    if (e != hipSuccess) return e;
    if (after_count && (e = hipEventRecord(after_count, stream)) != hipSuccess) return e;
    return launch_tile_scan(w, d_total, false, stream);
}

hipError_t launch_find(const Plan &plan, const uint8_t *d_text, uint64_t n, const Params *d_params,
                       const uint8_t *d_pat, const FindWs &w, int64_t *d_out, uint64_t first,
                       uint64_t cap, uint64_t *d_total, hipStream_t stream, hipEvent_t after_count)
{
    if (w.ntiles == 0) return hipSuccess;
    if (w.ntiles > 0xFFFFFFFFull) return hipErrorInvalidValue;
    ScanArgs a = make_args(plan, d_text, n, d_params, d_pat, w.ntiles);
    a.tile_cnt = w.tile_cnt;
    a.super = w.super;
    a.stash = w.stash;
    a.list = w.list;
    a.nlist = w.nlist;
    a.out = d_out;
    a.lo = first;
    a.cap = cap;
    // bitmap form for the mask-producing scans with lanes of >= 32 starts (the
    // workspace holds the bitmap region for m <= 64 only)
    if ((plan.algo == ALGO_SHIFT_AND || plan.algo == ALGO_BRUTE) && plan.lane_bytes >= 32) a.bits = w.bits;
    const uint32_t g = count_grid(a);
    if (!g) return hipErrorInvalidValue;
    const bool block = plan.algo == ALGO_BLOCK;
    hipError_t e = block ? launch_block_count(a, g, stream) : launch_any<K_FIND_COUNT>(plan, a, g, stream);
    if (e != hipSuccess) return e;
    if (after_count) {
        e = hipEventRecord(after_count, stream);
        if (e != hipSuccess) return e;
    }
    if ((e = launch_tile_scan(w, d_total, true, stream)) != hipSuccess) return e;
    if (cap == 0) return hipSuccess;
    uint64_t eg = w.ntiles < EMIT_GRID ? w.ntiles : EMIT_GRID;
    if (block) {
        hipLaunchKernelGGL(block_emit_kernel, dim3((uint32_t)eg), dim3(BLOCK), 0, stream, a);
        return hipGetLastError();
    }
    return launch_any<K_EMIT>(plan, a, (uint32_t)eg, stream);
}

hipError_t launch_set_u64(uint64_t *d_dst, uint64_t value, hipStream_t stream)
{
    hipLaunchKernelGGL(set_u64_kernel, dim3(1), dim3(1), 0, stream, d_dst, value);
    return hipGetLastError();
}

hipError_t launch_histogram(const uint8_t *d_text, uint64_t n, uint64_t *d_hist256, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    uint64_t blocks = (n + BLOCK * 64 - 1) / (BLOCK * 64);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(hist_kernel, dim3((uint32_t)blocks), dim3(BLOCK), 0, stream, d_text, n, d_hist256);
    return hipGetLastError();
}

}  // namespace sm
