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
    uint64_t ntiles;
    uint64_t *total;      // count mode: occurrences are added here
    uint32_t *tile_cnt;   // find mode: per-tile counts (count kernel writes, emit reads)
    uint16_t *stash;      // find mode: STASH_K offsets per tile
    const uint64_t *tile_off;  // emit: exclusive prefix of tile_cnt
    const uint32_t *list;      // emit: tiles with hits, ascending
    const uint64_t *nlist;     // emit: list length
    int64_t *out;         // emit: hit number k of the pattern goes to out[k - lo]
    uint64_t lo, cap;     // emit: window [lo, lo + cap) of hit numbers
};

template <int ALGO, int L>
struct Geometry {
    static constexpr int T = BLOCK * L;
    // halo bytes beyond the tile, plus 16 for misalignment and 16 for word reads
    static constexpr int HALO = (ALGO == ALGO_HASHQ) ? (Q_MAX + 32) : (BP_MAX_M + 32);
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
    } else if (ALGO == ALGO_SHIFT_AND && VAR == 0) {
        reinterpret_cast<uint32_t *>(s_mask)[tid] = r.x;
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
    g.x1 = g.s + (uint64_t)g.hi_rel + a.m;  // one past the last byte any window reads
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
    stage_commit<ALGO == ALGO_SHIFT_AND>(st, S.text);
    s = g.s;
    li0 = st.boff - g.r0;
    lo = threadIdx.x * L;
    hi = (lo + L - 1) < g.hi_rel ? (lo + L - 1) : g.hi_rel;
}

template <int ALGO, int L, int VAR, bool WRITE, class E>
__device__ __forceinline__ uint32_t run_lane(TileShared<ALGO, L> &S, const ScanArgs &a, int m,
                                             int sh1, int period, int period_lb, uint64_t s,
                                             int li0, int lo, int hi, E &o)
{
    if (ALGO != ALGO_HASHQ && lo > hi) return 0u;  // Hash-q lanes take part in wave checks
    if (ALGO == ALGO_SHIFT_AND) {
        if (VAR == 0)
            return lane_shift_and<uint32_t, 16, WRITE>(S.text, reinterpret_cast<const uint32_t *>(S.mask),
                                                       m, li0, lo, hi, o);
        if (VAR == 1) return lane_shift_and<uint64_t, 16, WRITE>(S.text, S.mask, m, li0, lo, hi, o);
        if (VAR == 2) return lane_shift_and<uint64_t, 4, WRITE>(S.text, S.mask, m, li0, lo, hi, o);
        return lane_shift_and<uint64_t, 1, WRITE>(S.text, S.mask, m, li0, lo, hi, o);
    } else if (ALGO == ALGO_BNDM) {
        return lane_bndm<WRITE>(reinterpret_cast<const uint8_t *>(S.text), S.mask, m, li0, lo, hi, o);
    } else if (ALGO == ALGO_SBNDM) {  // VAR selects the q-gram width 1, 2, 4, 8
        constexpr int Q = VAR == 0 ? 1 : (VAR == 1 ? 2 : (VAR == 2 ? 4 : 8));
        return lane_sbndm<Q, WRITE>(reinterpret_cast<const uint8_t *>(S.text), S.mask, m, period, li0,
                                    lo, hi, o);
    } else {
        return lane_hashq<VAR, WRITE>(reinterpret_cast<const uint32_t *>(S.text), S.shift, m,
                                      (int)a.q, (int)a.hbits, sh1, period, period_lb, li0, lo, hi,
                                      a.text, s, a.pat, o);
    }
}

// Count kernel: per-tile counts go to tile_cnt (the tile-count scan then sums
// them: one atomic per workgroup on a single address would serialize). FIND:
// tiles with 1..STASH_K hits also stash their hits' offsets.
// A workgroup owns tiles_per_wg consecutive tiles. PREFETCH: the next tile's
// loads are in flight while the current tile is scanned (costs registers);
// otherwise each tile is loaded after the previous one is done.
template <int ALGO, int L, int VAR, bool FIND, bool PREFETCH>
__global__ __launch_bounds__(BLOCK) void count_kernel(ScanArgs a)
{
    using G = Geometry<ALGO, L>;
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
    tables_commit<ALGO, VAR>(tb, S.mask, S.shift, a.hbits);

    for (uint64_t t = t_begin; t < t_end; t++) {
        if (!PREFETCH && t != t_begin) {
            g = tile_geom<ALGO, L>(a, t);
            stage_issue(st, a.text, g.x0, g.x1);
        }
        __syncthreads();  // previous tile's LDS readers are done
        stage_commit<ALGO == ALGO_SHIFT_AND>(st, S.text);
        const TileGeom cur = g;
        const int li0 = st.boff - cur.r0;
        __syncthreads();
        if (PREFETCH && t + 1 < t_end) {  // the next tile's loads overlap this tile's scan
            g = tile_geom<ALGO, L>(a, t + 1);
            stage_issue(st, a.text, g.x0, g.x1);
        }
        const int lo = threadIdx.x * L;
        const int hi = (lo + L - 1) < cur.hi_rel ? (lo + L - 1) : cur.hi_rel;
        // Shift-And (hits come as bit masks) counts while keeping the lane's first
        // hits; the skip algorithms count (their hits are rare) and scan again
        constexpr bool CAP_OK = FIND && ALGO == ALGO_SHIFT_AND;
        const bool cap = CAP_OK && a.slots;  // uniform
        uint32_t c;
        CapEmit ce;
        if (cap) {
            run_lane<ALGO, L, VAR, true>(S, a, m, sh1, period, period_lb, cur.s, li0, lo, hi, ce);
            c = ce.n;
        } else {
            NoEmit ne;
            c = run_lane<ALGO, L, VAR, false>(S, a, m, sh1, period, period_lb, cur.s, li0, lo, hi, ne);
        }
        uint32_t tot;
        const uint32_t before = block_excl_scan(c, S.w, tot);
        if (threadIdx.x == 0) a.tile_cnt[t] = tot;
        if (FIND && tot && tot <= STASH_K) {  // uniform
            uint16_t *dst = a.stash + t * STASH_K;
            if (cap && !__syncthreads_or(c > LANE_K)) {
                for (uint32_t k = 0; k < c; k++) dst[before + k] = ce.get(k);
            } else {  // scan again into the stash
                StashEmit se;
                se.dst = dst;
                se.idx = before;
                run_lane<ALGO, L, VAR, true>(S, a, m, sh1, period, period_lb, cur.s, li0, lo, hi, se);
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
    // 1. tiles with at most STASH_K hits: copy their stash
    for (uint64_t e = blockIdx.x; e < nl; e += gridDim.x) {
        const uint64_t t = a.list[e];
        const uint32_t tot = a.tile_cnt[t];
        const uint64_t off = a.tile_off[t];
        if (tot > STASH_K || off >= a.lo + a.cap || off + tot <= a.lo) continue;  // uniform
        const uint64_t s = t * (uint64_t)Geometry<ALGO, L>::T;
        const uint16_t *src = a.stash + t * STASH_K;
        for (uint32_t k = threadIdx.x; k < tot; k += BLOCK) {
            const uint64_t r = off + k - a.lo;
            if (r < a.cap) a.out[r] = (int64_t)(s + src[k]);
        }
    }
    // 2. denser tiles: rescan from LDS
    auto next_dense = [&](uint64_t e) -> uint64_t {  // uniform over the workgroup
        for (; e < nl; e += gridDim.x) {
            const uint64_t t = a.list[e];
            const uint32_t tot = a.tile_cnt[t];
            const uint64_t off = a.tile_off[t];
            if (tot > STASH_K && off < a.lo + a.cap && off + tot > a.lo) return e;
        }
        return nl;
    };
    uint64_t e = next_dense(blockIdx.x);
    if (e >= nl) return;
    {
        const uint4 tb = tables_issue<ALGO>(a.prm, a.hbits);
        tables_commit<ALGO, VAR>(tb, S.mask, S.shift, a.hbits);
    }
    using G = Geometry<ALGO, L>;
    for (; e < nl; e = next_dense(e + gridDim.x)) {
        const uint64_t t = a.list[e];
        const uint64_t off = a.tile_off[t];
        const TileGeom cur = tile_geom<ALGO, L>(a, t);
        Staged<G::PER> st;
        stage_issue(st, a.text, cur.x0, cur.x1);
        __syncthreads();  // the previous tile's LDS readers are done
        stage_commit<ALGO == ALGO_SHIFT_AND>(st, S.text);
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
            run_lane<ALGO, L, VAR, true>(S, a, m, sh1, period, period_lb, s2, li0, lo, hi, se);
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
}

// Tile-count scan, SCAN_CHUNK tiles per workgroup of 1024 threads and no waiting
// between workgroups: workgroup w first sums all counts before its chunk itself
// (coalesced 16-byte loads, eight in flight per thread), then scans its chunk.
// Writes exclusive offsets and the ascending list of tiles with hits; the last
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

__global__ __launch_bounds__(1024) void tile_scan_kernel(const uint32_t *cnt, uint64_t nt,
                                                         uint64_t *off, uint64_t *total,
                                                         uint32_t *list, uint64_t *nlist)
{
    __shared__ uint64_t s_a[16];
    __shared__ uint32_t s_b[16];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const uint64_t c0 = (uint64_t)blockIdx.x * SCAN_CHUNK;
    // 1. occurrences and listed tiles before this chunk
    uint64_t pre = 0;
    uint32_t pnz = 0;
    for (uint64_t i0 = 0; i0 < c0; i0 += 8 * 4 * 1024) {
        uint4 v[8];
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const uint64_t i = i0 + 4 * (uint64_t)(tid + 1024 * k);
            v[k] = i < c0 ? load_cnt4(cnt, i, c0) : uint4{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int k = 0; k < 8; k++) {
            pre += (uint64_t)v[k].x + v[k].y + v[k].z + v[k].w;
            pnz += (v[k].x != 0) + (v[k].y != 0) + (v[k].z != 0) + (v[k].w != 0);
        }
    }
    block_sum2_1024(pre, pnz, s_a, s_b);
    // 2. this chunk: SCAN_CHUNK / 1024 = 4 consecutive counts per thread
    const uint64_t i = c0 + 4 * (uint64_t)tid;
    const uint4 v = load_cnt4(cnt, i, nt);
    const uint32_t c[4] = {v.x, v.y, v.z, v.w};
    const uint64_t my = (uint64_t)c[0] + c[1] + c[2] + c[3];
    const uint32_t mz = (c[0] != 0) + (c[1] != 0) + (c[2] != 0) + (c[3] != 0);
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
        for (int k = 0; k < 4; k++) {
            if (i + k < nt) {
                off[i + k] = o;
                if (c[k]) list[zp++] = (uint32_t)(i + k);
                o += c[k];
            }
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
    uint32_t m, algo, q, hbits;
    uint32_t inline_len;  // pattern bytes carried below (0: already in pat)
    uint8_t inline_pat[PREP_INLINE];
};

__global__ __launch_bounds__(BLOCK) void prep_kernel(PrepArgs a)
{
    __shared__ uint32_t s_tab[1 << H_MAX];
    __shared__ uint8_t s_pat[PREP_INLINE];
    const int tid = threadIdx.x;
    const uint32_t m = a.m;
    Params *P = a.prm;

    if (a.inline_len) {
        for (uint32_t k = tid; k < a.inline_len; k += BLOCK) {
            a.pat[k] = a.inline_pat[k];
            s_pat[k] = a.inline_pat[k];
        }
        // zero padding up to a multiple of 16
        const uint32_t padded = (m + 15) & ~15u;
        for (uint32_t k = m + tid; k < padded; k += BLOCK) a.pat[k] = 0;
    }
    if (tid == 0) {
        P->m = m;
        P->algo = a.algo;
        P->q = a.q;
        P->hbits = a.hbits;
        if (a.zero) *a.zero = 0;
    }
    __syncthreads();
    // pattern bytes: from LDS when inline, else from the workspace copy
    const uint8_t *pp = a.inline_len ? s_pat : a.pat;

    __shared__ uint32_t s_bad[PERIOD_MAX + 1];
    build_tables(pp, m, a.algo, a.q, a.hbits, P, s_tab, s_bad);
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
    const bool pf = a.tiles_per_wg > 1;
    if (KIND == K_COUNT) {
        if (pf) hipLaunchKernelGGL((count_kernel<ALGO, L, VAR, false, true>), dim3(grid), dim3(BLOCK), 0, st, a);
        else hipLaunchKernelGGL((count_kernel<ALGO, L, VAR, false, false>), dim3(grid), dim3(BLOCK), 0, st, a);
    } else if (KIND == K_FIND_COUNT) {
        if (pf) hipLaunchKernelGGL((count_kernel<ALGO, L, VAR, true, true>), dim3(grid), dim3(BLOCK), 0, st, a);
        else hipLaunchKernelGGL((count_kernel<ALGO, L, VAR, true, false>), dim3(grid), dim3(BLOCK), 0, st, a);
    } else
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
        if (m <= 17) return launch_l<ALGO_SHIFT_AND, 0, KIND>(p, a, grid, st);
        if (m <= 49) return launch_l<ALGO_SHIFT_AND, 1, KIND>(p, a, grid, st);
        if (m <= 61) return launch_l<ALGO_SHIFT_AND, 2, KIND>(p, a, grid, st);
        return launch_l<ALGO_SHIFT_AND, 3, KIND>(p, a, grid, st);
    }
    case ALGO_BNDM: return launch_l<ALGO_BNDM, 0, KIND>(p, a, grid, st);
    case ALGO_SBNDM:
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
    a.ntiles = ntiles;
    return a;
}

uint32_t count_grid(const ScanArgs &a)
{
    const uint64_t nblk = (a.ntiles + a.tiles_per_wg - 1) / a.tiles_per_wg;
    return nblk > 0x7FFFFFFFull ? 0u : (uint32_t)nblk;
}

}  // namespace

hipError_t launch_prep(const Plan &plan, const uint8_t *pat_host, Params *d_params, uint8_t *d_pat,
                       uint64_t *d_zero, hipStream_t stream)
{
    PrepArgs a;
    a.prm = d_params;
    a.pat = d_pat;
    a.zero = d_zero;
    a.m = (uint32_t)plan.m;
    a.algo = (uint32_t)plan.algo;
    a.q = (uint32_t)plan.q;
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
                       w.ntiles, find ? w.tile_off : nullptr, d_total, find ? w.list : nullptr,
                       find ? w.nlist : nullptr);
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
    const uint32_t g = count_grid(a);
    if (!g) return hipErrorInvalidValue;
    hipError_t e = launch_any<K_COUNT>(plan, a, g, stream);
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
    a.stash = w.stash;
    a.tile_off = w.tile_off;
    a.list = w.list;
    a.nlist = w.nlist;
    a.out = d_out;
    a.lo = first;
    a.cap = cap;
    const uint32_t g = count_grid(a);
    if (!g) return hipErrorInvalidValue;
    hipError_t e = launch_any<K_FIND_COUNT>(plan, a, g, stream);
    if (e != hipSuccess) return e;
    if (after_count) {
        e = hipEventRecord(after_count, stream);
        if (e != hipSuccess) return e;
    }
    if ((e = launch_tile_scan(w, d_total, true, stream)) != hipSuccess) return e;
    if (cap == 0) return hipSuccess;
    uint64_t eg = w.ntiles < EMIT_GRID ? w.ntiles : EMIT_GRID;
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
