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
// Every lane produces its hits in ascending order; lane counts are combined by a
// workgroup scan, and tiles by the tile-count scan, so positions land in the
// output sorted and deterministically (count -> scan -> write).
//
// Bounds. Only starts i <= n - m are ever reported, and every window that is
// reported reads bytes < n only. LDS bytes beyond the text are never consulted
// for a reported position. Global loads are 16-byte aligned blocks that contain
// at least one byte of the text, so they never leave the text's pages.
#include <hip/hip_runtime.h>
#include "sm_internal.h"

namespace sm {
namespace {

__device__ __forceinline__ uint32_t swz(uint32_t u) { return u ^ ((u >> 3) & 7u); }

__device__ __forceinline__ uint32_t alignbyte(uint32_t hi, uint32_t lo, uint32_t s)
{
    return __builtin_amdgcn_alignbyte(hi, lo, s);
}

// Workgroup -> tile-group remap so that consecutive tile groups run on the same
// XCD (workgroups are dealt round-robin over the 8 XCDs); neighbouring tiles share
// their halo bytes through that XCD's L2.
__device__ __forceinline__ uint64_t xcd_remap(uint64_t bid, uint64_t nblk)
{
    const uint64_t X = 8;
    uint64_t x = bid % X, k = bid / X;
    uint64_t per = nblk / X, rem = nblk % X;
    return x < rem ? x * (per + 1) + k : rem * (per + 1) + (x - rem) * per + k;
}

// ---------------------------------------------------------------------------
// q-gram hash: the q bytes, packed little-endian into up to four words (unused
// bytes zero), multiplicatively hashed. Used identically by the prep kernel and
// the scan; any hash is correct because candidates are verified byte-exactly.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t qhash(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3,
                                          uint32_t hbits)
{
    uint32_t h = w0 * 0x9E3779B1u;
    h ^= w1 * 0x85EBCA77u;
    h ^= w2 * 0xC2B2AE3Du;
    h ^= w3 * 0x27D4EB2Fu;
    return h >> (32 - hbits);
}

__device__ __forceinline__ uint32_t byte_mask(int nbytes)  // nbytes in [0, 4]
{
    return nbytes >= 4 ? 0xFFFFFFFFu : ((1u << (8 * nbytes)) - 1u);
}

// ---------------------------------------------------------------------------
// Workgroup reductions (BLOCK = 256 threads = 4 wave64).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

// exclusive scan of v over the workgroup; returns the prefix, sets total
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *s_w, uint32_t &total)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t inc = wave_incl_scan(v);
    if (lane == 63) s_w[wv] = inc;
    __syncthreads();
    uint32_t before = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < BLOCK / 64; k++) {
        uint32_t x = s_w[k];
        before += (k < wv) ? x : 0;
        tot += x;
    }
    __syncthreads();
    total = tot;
    return before + inc - v;
}

// ---------------------------------------------------------------------------
// Tile staging: text positions [x0, x1) (0 <= x0 < x1 <= n) into LDS chunks.
// Returns the byte offset in LDS of position x0 (its offset inside the first
// aligned 16-byte block). SWZ selects the XOR-swizzled chunk layout used by the
// per-lane sequential readers (conflict-free 16-byte LDS reads at any segment
// stride that is a power of two >= 16).
// ---------------------------------------------------------------------------
template <bool SWZ>
__device__ __forceinline__ int stage(uint4 *lds, const uint8_t *text, uint64_t x0, uint64_t x1)
{
    const uintptr_t a0 = (uintptr_t)(text + x0);
    const uintptr_t c0 = a0 & ~(uintptr_t)15;
    const uintptr_t c1 = ((uintptr_t)(text + x1 - 1)) & ~(uintptr_t)15;
    const uint32_t nch = (uint32_t)((c1 - c0) >> 4) + 1;
    const uint4 *src = reinterpret_cast<const uint4 *>(c0);
    for (uint32_t u = threadIdx.x; u < nch; u += BLOCK) {
        uint4 v = src[u];
        lds[SWZ ? swz(u) : u] = v;
    }
    return (int)(a0 & 15);
}

// ---------------------------------------------------------------------------
// Lane scanners. Coordinates are relative to the tile start s. A lane owns
// starts [lo, hi] (hi >= lo). `li0` is the LDS byte index of relative position 0.
// WRITE=false: return the number of hits. WRITE=true: write each hit's global
// position at out[idx++] while idx < cap.
// ---------------------------------------------------------------------------
struct Out {
    int64_t *out;
    uint64_t idx, cap;
    uint64_t base;  // global position of relative position 0
    __device__ __forceinline__ void put(int rel)
    {
        if (idx < cap) out[idx] = (int64_t)(base + (uint64_t)(int64_t)rel);
        idx++;
    }
};

// Shift-And, complemented (Shift-Or) form. W = state word; CHECK = bytes between
// hit checks (requires m - 1 + CHECK <= bits of W).
template <typename W, int CHECK, bool WRITE>
__device__ __forceinline__ uint32_t lane_shift_and(const uint4 *lds, const W *mask, int m, int li0,
                                                  int lo, int hi, Out &o)
{
    const int e_lo = lo + m - 1, e_hi = hi + m - 1;  // relative ends owned by this lane
    const int u0 = (lo + li0) >> 4, u1 = (e_hi + li0) >> 4;
    W D = ~(W)0;
    uint32_t cnt = 0;
    for (int u = u0; u <= u1; u++) {
        const uint4 v = lds[swz((uint32_t)u)];
        const uint32_t wd[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int g = 0; g < 16 / CHECK; g++) {
#pragma unroll
            for (int b = 0; b < CHECK; b++) {
                const int k = g * CHECK + b;
                const uint32_t c = (wd[k >> 2] >> (8 * (k & 3))) & 0xFFu;
                D = (D << 1) | mask[c];
            }
            // relative end of the last byte consumed
            const int e_last = 16 * u + g * CHECK + CHECK - 1 - li0;
            int jlo = e_last - e_hi, jhi = e_last - e_lo;
            jlo = jlo < 0 ? 0 : jlo;
            jhi = jhi > CHECK - 1 ? CHECK - 1 : jhi;
            if (jlo <= jhi) {
                uint32_t hits = (uint32_t)((~D) >> (m - 1)) & ((1u << CHECK) - 1u);
                hits &= ((2u << jhi) - 1u) & ~((1u << jlo) - 1u);
                if (hits) {
                    if (WRITE) {
                        // bit j <-> end e_last - j; ascending positions = descending j
                        while (hits) {
                            const int j = 31 - __builtin_clz(hits);
                            hits &= ~(1u << j);
                            o.put(e_last - j - m + 1);
                        }
                    } else {
                        cnt += __builtin_popcount(hits);
                    }
                }
            }
        }
    }
    return cnt;
}

// BNDM: masks B[c] bit i set iff p[m-1-i] == c.
template <bool WRITE>
__device__ __forceinline__ uint32_t lane_bndm(const uint8_t *lds8, const uint64_t *B, int m,
                                             int li0, int lo, int hi, Out &o)
{
    const uint64_t HB = 1ull << (m - 1);
    const uint64_t ALL = ~0ull >> (64 - m);
    uint32_t cnt = 0;
    int pos = lo;
    while (pos <= hi) {
        int j = m, last = m;
        uint64_t D = ALL;
        const uint8_t *w = lds8 + li0 + pos;
        do {
            j--;
            D &= B[w[j]];
            if (D & HB) {
                if (j > 0) {
                    last = j;
                } else {
                    if (WRITE) o.put(pos); else cnt++;
                    break;
                }
            }
            D <<= 1;
        } while (D != 0 && j > 0);
        pos += last;
    }
    return cnt;
}

// SBNDM: same masks; no prefix tracking; shift m-k+1 when the k-byte suffix is
// not a factor of p; after a hit, shift by the smallest period of p.
template <bool WRITE>
__device__ __forceinline__ uint32_t lane_sbndm(const uint8_t *lds8, const uint64_t *B, int m,
                                              int period, int li0, int lo, int hi, Out &o)
{
    const uint64_t HB = 1ull << (m - 1);
    uint32_t cnt = 0;
    int pos = lo;
    while (pos <= hi) {
        const uint8_t *w = lds8 + li0 + pos;  // window bytes w[0 .. m-1]
        uint64_t D = B[w[m - 1]];
        int k = 1;
        while (D != 0 && k < m) {
            D = (D << 1) & B[w[m - 1 - k]];
            k++;
        }
        if (D & HB) {  // the whole window was read and equals p
            if (WRITE) o.put(pos); else cnt++;
            pos += period;
        } else {
            pos += m - k + 1;
        }
    }
    return cnt;
}

// Byte-exact check of the window starting at global position gpos against p.
// Reads aligned text words that contain window bytes only.
__device__ __noinline__ bool verify_global(const uint8_t *text, uint64_t gpos, const uint8_t *pat,
                                            uint32_t m)
{
    const uintptr_t a = (uintptr_t)(text + gpos);
    const uint32_t *T = reinterpret_cast<const uint32_t *>(a & ~(uintptr_t)3);
    const uint32_t sh = (uint32_t)(a & 3);
    const uint32_t klast = (uint32_t)(((a + m - 1) >> 2) - (a >> 2));
    const uint32_t *P = reinterpret_cast<const uint32_t *>(pat);
    uint32_t prev = T[0];
    for (uint32_t i = 0; i < m; i += 4) {
        const uint32_t kk = (i >> 2) + 1;
        const uint32_t cur = kk <= klast ? T[kk] : 0u;
        const uint32_t w = alignbyte(cur, prev, sh);
        const uint32_t rem = m - i;
        const uint32_t msk = rem >= 4 ? 0xFFFFFFFFu : ((1u << (8 * rem)) - 1u);
        if ((w ^ P[i >> 2]) & msk) return false;
        prev = cur;
    }
    return true;
}

// Hash-q over the lane's windows. The LDS holds text positions from m-q on;
// li0 is the LDS index of relative position 0 (may be negative).
template <int NW, bool WRITE>
__device__ __forceinline__ uint32_t lane_hashq(const uint32_t *lds32, const uint8_t *shift, int m,
                                              int q, int hbits, int sh1, int li0, int lo, int hi,
                                              const uint8_t *text, uint64_t s, const uint8_t *pat,
                                              Out &o)
{
    uint32_t cnt = 0;
    int pos = lo;
    while (pos <= hi) {
        const int gs = li0 + pos + m - q;  // LDS index of the q-gram's first byte
        const int wi = gs >> 2, sb = gs & 3;
        uint32_t d[NW + 1];
#pragma unroll
        for (int k = 0; k <= NW; k++) d[k] = lds32[wi + k];
        uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int k = 0; k < NW; k++) w[k] = alignbyte(d[k + 1], d[k], (uint32_t)sb) & byte_mask(q - 4 * k);
        const uint32_t h = qhash(w[0], w[1], w[2], w[3], (uint32_t)hbits);
        const int sh = shift[h];
        if (sh == 0) {
            if (verify_global(text, s + (uint64_t)pos, pat, (uint32_t)m)) {
                if (WRITE) o.put(pos); else cnt++;
            }
            pos += sh1;
        } else {
            pos += sh;
        }
    }
    return cnt;
}

// ---------------------------------------------------------------------------
// Scan kernel: COUNT (WRITE=false) writes per-tile counts and adds them to the
// total; WRITE=true re-scans tiles with hits and writes their positions.
// ---------------------------------------------------------------------------
struct ScanArgs {
    const uint8_t *text;
    uint64_t n;
    const Params *prm;
    const uint8_t *pat;
    uint32_t m, q, hbits, tiles_per_wg;
    uint64_t ntiles;
    uint32_t *tile_cnt;
    const uint64_t *tile_off;
    uint64_t *total;
    int64_t *out;
    uint64_t cap;
};

template <int ALGO, int L>
struct Geometry {
    static constexpr int T = BLOCK * L;
    // halo bytes beyond the tile, plus 16 for misalignment and 16 for word reads
    static constexpr int HALO = (ALGO == ALGO_HASHQ) ? (Q_MAX + 32) : (BP_MAX_M + 32);
    // whole groups of 8 chunks: the swizzle permutes chunks inside such groups
    static constexpr int CHUNKS = (((T + HALO + 15) / 16 + 1) + 7) & ~7;
};

template <int ALGO, int L, int VAR, bool WRITE>
__global__ __launch_bounds__(BLOCK) void scan_kernel(ScanArgs a)
{
    using G = Geometry<ALGO, L>;
    constexpr int T = G::T;
    __shared__ uint4 s_text[G::CHUNKS];
    __shared__ uint64_t s_mask[(ALGO == ALGO_HASHQ) ? 1 : 256];
    __shared__ uint8_t s_shift[(ALGO == ALGO_HASHQ) ? (1 << H_MAX) : 1];
    __shared__ uint32_t s_w[BLOCK / 64];

    const int tid = threadIdx.x;
    const int m = (int)a.m;

    // tables: once per workgroup
    if (ALGO == ALGO_HASHQ) {
        const uint32_t nb = 1u << a.hbits;
        const uint4 *src = reinterpret_cast<const uint4 *>(a.prm->shift);
        for (uint32_t k = tid; k < nb / 16; k += BLOCK) reinterpret_cast<uint4 *>(s_shift)[k] = src[k];
    } else if (ALGO == ALGO_SHIFT_AND && VAR == 0) {
        reinterpret_cast<uint32_t *>(s_mask)[tid] = (uint32_t)a.prm->mask[tid];
    } else {
        s_mask[tid] = a.prm->mask[tid];
    }
    const int sh1 = (int)a.prm->sh1;
    const int period = (int)a.prm->period;

    const uint64_t nblk = gridDim.x;
    const uint64_t g = xcd_remap(blockIdx.x, nblk);
    const uint64_t t_begin = g * a.tiles_per_wg;
    uint64_t t_end = t_begin + a.tiles_per_wg;
    if (t_end > a.ntiles) t_end = a.ntiles;

    const uint64_t last_start = a.n - a.m;  // n >= m guaranteed by the host

    for (uint64_t t = t_begin; t < t_end; t++) {
        uint64_t out_base = 0;
        if (WRITE) {
            const uint32_t tc = a.tile_cnt[t];
            out_base = a.tile_off[t];
            if (tc == 0 || out_base >= a.cap) continue;  // uniform over the workgroup
        }
        const uint64_t s = t * (uint64_t)T;
        const uint64_t lim = last_start - s;  // >= 0 since t < ntiles
        const int hi_rel = lim >= (uint64_t)(T - 1) ? T - 1 : (int)lim;

        // staged span [x0, x1)
        const uint64_t r0 = (ALGO == ALGO_HASHQ) ? (uint64_t)(m - (int)a.q) : 0;
        const uint64_t x0 = s + r0;
        uint64_t x1 = s + (uint64_t)hi_rel + a.m;  // one past the last byte any window reads
        if (x1 > a.n) x1 = a.n;

        __syncthreads();  // previous tile's LDS readers are done
        const int boff = stage<ALGO == ALGO_SHIFT_AND>(s_text, a.text, x0, x1);
        __syncthreads();

        // LDS byte index of relative position 0
        const int li0 = boff - (int)r0;
        const int lo = tid * L;
        const int hi = (lo + L - 1) < hi_rel ? (lo + L - 1) : hi_rel;

        Out o;
        o.out = a.out;
        o.cap = a.cap;
        o.base = s;
        o.idx = 0;


        uint32_t c = 0;
        if (ALGO == ALGO_SHIFT_AND) {
            if (lo <= hi) {
                if (VAR == 0) {
                    // 32-bit state, check every 16 bytes: m <= 17
                    const uint32_t *msk = reinterpret_cast<const uint32_t *>(s_mask);
                    c = lane_shift_and<uint32_t, 16, false>(s_text, msk, m, li0, lo, hi, o);
                } else if (VAR == 1) {
                    c = lane_shift_and<uint64_t, 16, false>(s_text, s_mask, m, li0, lo, hi, o);
                } else if (VAR == 2) {
                    c = lane_shift_and<uint64_t, 4, false>(s_text, s_mask, m, li0, lo, hi, o);
                } else {
                    c = lane_shift_and<uint64_t, 1, false>(s_text, s_mask, m, li0, lo, hi, o);
                }
            }
        } else if (ALGO == ALGO_BNDM) {
            if (lo <= hi) c = lane_bndm<false>((const uint8_t *)s_text, s_mask, m, li0, lo, hi, o);
        } else if (ALGO == ALGO_SBNDM) {
            if (lo <= hi)
                c = lane_sbndm<false>((const uint8_t *)s_text, s_mask, m, period, li0, lo, hi, o);
        } else {
            if (lo <= hi)
                c = lane_hashq<VAR, false>((const uint32_t *)s_text, s_shift, m, (int)a.q,
                                           (int)a.hbits, sh1, li0, lo, hi, a.text, s, a.pat, o);
        }

        if (!WRITE) {
            uint32_t tot;
            block_excl_scan(c, s_w, tot);
            if (tid == 0) {
                a.tile_cnt[t] = tot;
                if (tot) atomicAdd((unsigned long long *)a.total, (unsigned long long)tot);
            }
        } else {
            uint32_t tot;
            const uint32_t before = block_excl_scan(c, s_w, tot);
            if (c) {
                o.idx = out_base + before;
                if (o.idx < a.cap) {
                    if (ALGO == ALGO_SHIFT_AND) {
                        if (VAR == 0) {
                            const uint32_t *msk = reinterpret_cast<const uint32_t *>(s_mask);
                            lane_shift_and<uint32_t, 16, true>(s_text, msk, m, li0, lo, hi, o);
                        } else if (VAR == 1) {
                            lane_shift_and<uint64_t, 16, true>(s_text, s_mask, m, li0, lo, hi, o);
                        } else if (VAR == 2) {
                            lane_shift_and<uint64_t, 4, true>(s_text, s_mask, m, li0, lo, hi, o);
                        } else {
                            lane_shift_and<uint64_t, 1, true>(s_text, s_mask, m, li0, lo, hi, o);
                        }
                    } else if (ALGO == ALGO_BNDM) {
                        lane_bndm<true>((const uint8_t *)s_text, s_mask, m, li0, lo, hi, o);
                    } else if (ALGO == ALGO_SBNDM) {
                        lane_sbndm<true>((const uint8_t *)s_text, s_mask, m, period, li0, lo, hi, o);
                    } else {
                        lane_hashq<VAR, true>((const uint32_t *)s_text, s_shift, m, (int)a.q,
                                              (int)a.hbits, sh1, li0, lo, hi, a.text, s, a.pat, o);
                    }
                }
            }
        }
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

    if (a.algo == ALGO_SHIFT_AND) {
        // complemented masks: bit j clear iff p[j] == c (j < m); bits >= m clear
        const uint32_t c = tid;
        uint64_t w = 0;
        for (uint32_t j = 0; j < m; j++)
            if (pp[j] != c) w |= 1ull << j;
        P->mask[c] = w;
    } else if (a.algo == ALGO_BNDM || a.algo == ALGO_SBNDM) {
        const uint32_t c = tid;
        uint64_t w = 0;
        for (uint32_t i = 0; i < m; i++)
            if (pp[m - 1 - i] == c) w |= 1ull << i;
        P->mask[c] = w;
        if (tid == 0) {
            // smallest period = m - (longest proper border of p)
            int b = 0;  // border of p[0..k]
            // prefix-function pass, O(m) with m <= 64
            int pi[BP_MAX_M];
            pi[0] = 0;
            for (uint32_t k = 1; k < m; k++) {
                while (b > 0 && pp[k] != pp[b]) b = pi[b - 1];
                if (pp[k] == pp[b]) b++;
                pi[k] = b;
            }
            P->period = m - (uint32_t)pi[m - 1];
        }
    } else if (a.algo == ALGO_HASHQ) {
        const uint32_t q = a.q, hb = a.hbits, nb = 1u << hb;
        const uint32_t dflt = m - q + 1;
        for (uint32_t k = tid; k < nb; k += BLOCK) s_tab[k] = dflt;
        __syncthreads();
        // q-grams ending at j = q-1 .. m-2 (all but the last)
        for (uint32_t j = q - 1 + tid; j + 1 < m; j += BLOCK) {
            uint32_t w[4] = {0, 0, 0, 0};
            for (uint32_t k = 0; k < q; k++) w[k >> 2] |= (uint32_t)pp[j + 1 - q + k] << (8 * (k & 3));
            atomicMin(&s_tab[qhash(w[0], w[1], w[2], w[3], hb)], m - 1 - j);
        }
        __syncthreads();
        uint32_t hl;
        {
            uint32_t w[4] = {0, 0, 0, 0};
            for (uint32_t k = 0; k < q; k++) w[k >> 2] |= (uint32_t)pp[m - q + k] << (8 * (k & 3));
            hl = qhash(w[0], w[1], w[2], w[3], hb);
        }
        if (tid == 0) P->sh1 = s_tab[hl];
        __syncthreads();
        for (uint32_t k = tid; k < nb; k += BLOCK) {
            uint32_t v = (k == hl) ? 0u : s_tab[k];
            P->shift[k] = (uint8_t)(v > 255u ? 255u : v);
        }
    }
}

// ---------------------------------------------------------------------------
// Tile-count scan (single workgroup of 1024 threads) -> exclusive offsets, total.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void tile_scan_kernel(const uint32_t *cnt, uint64_t nt,
                                                         uint64_t *off, uint64_t *total)
{
    __shared__ uint64_t s_part[1024];
    const uint64_t per = (nt + 1023) / 1024;
    const uint64_t b = threadIdx.x * per;
    uint64_t e = b + per;
    if (e > nt) e = nt;
    uint64_t sum = 0;
    for (uint64_t k = b; k < e; k++) sum += cnt[k];
    s_part[threadIdx.x] = sum;
    __syncthreads();
    // Hillis-Steele inclusive scan over 1024 partial sums
    for (int d = 1; d < 1024; d <<= 1) {
        uint64_t v = threadIdx.x >= (unsigned)d ? s_part[threadIdx.x - d] : 0;
        __syncthreads();
        s_part[threadIdx.x] += v;
        __syncthreads();
    }
    uint64_t run = s_part[threadIdx.x] - sum;
    for (uint64_t k = b; k < e; k++) {
        off[k] = run;
        run += cnt[k];
    }
    if (threadIdx.x == 1023) *total = s_part[1023];
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
template <int ALGO, int L, int VAR, bool WRITE>
hipError_t launch_scan_t(const Plan &p, const ScanArgs &a, hipStream_t st)
{
    const uint64_t nblk = (a.ntiles + a.tiles_per_wg - 1) / a.tiles_per_wg;
    if (nblk == 0) return hipSuccess;
    if (nblk > 0x7FFFFFFFull) return hipErrorInvalidValue;
    hipLaunchKernelGGL((scan_kernel<ALGO, L, VAR, WRITE>), dim3((uint32_t)nblk), dim3(BLOCK), 0, st, a);
    return hipGetLastError();
}

template <int ALGO, int VAR, bool WRITE>
hipError_t launch_scan_l(const Plan &p, const ScanArgs &a, hipStream_t st)
{
    switch (p.lane_bytes) {
    case 16: return launch_scan_t<ALGO, 16, VAR, WRITE>(p, a, st);
    case 32: return launch_scan_t<ALGO, 32, VAR, WRITE>(p, a, st);
    case 64: return launch_scan_t<ALGO, 64, VAR, WRITE>(p, a, st);
    case 128: return launch_scan_t<ALGO, 128, VAR, WRITE>(p, a, st);
    default: return hipErrorInvalidValue;
    }
}

template <bool WRITE>
hipError_t launch_scan_any(const Plan &p, const ScanArgs &a, hipStream_t st)
{
    switch (p.algo) {
    case ALGO_SHIFT_AND: {
        const int m = (int)p.m;
        if (m <= 17) return launch_scan_l<ALGO_SHIFT_AND, 0, WRITE>(p, a, st);
        if (m <= 49) return launch_scan_l<ALGO_SHIFT_AND, 1, WRITE>(p, a, st);
        if (m <= 61) return launch_scan_l<ALGO_SHIFT_AND, 2, WRITE>(p, a, st);
        return launch_scan_l<ALGO_SHIFT_AND, 3, WRITE>(p, a, st);
    }
    case ALGO_BNDM: return launch_scan_l<ALGO_BNDM, 0, WRITE>(p, a, st);
    case ALGO_SBNDM: return launch_scan_l<ALGO_SBNDM, 0, WRITE>(p, a, st);
    case ALGO_HASHQ: {
        const int nw = (p.q + 3) / 4;
        if (nw <= 1) return launch_scan_l<ALGO_HASHQ, 1, WRITE>(p, a, st);
        if (nw == 2) return launch_scan_l<ALGO_HASHQ, 2, WRITE>(p, a, st);
        if (nw == 3) return launch_scan_l<ALGO_HASHQ, 3, WRITE>(p, a, st);
        return launch_scan_l<ALGO_HASHQ, 4, WRITE>(p, a, st);
    }
    default: return hipErrorInvalidValue;
    }
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

static ScanArgs make_args(const Plan &plan, const uint8_t *d_text, uint64_t n, const Params *d_params,
                          const uint8_t *d_pat, uint64_t ntiles)
{
    ScanArgs a;
    a.text = d_text;
    a.n = n;
    a.prm = d_params;
    a.pat = d_pat;
    a.m = (uint32_t)plan.m;
    a.q = (uint32_t)plan.q;
    a.hbits = (uint32_t)plan.hbits;
    a.tiles_per_wg = (uint32_t)plan.tiles_per_wg;
    a.ntiles = ntiles;
    a.tile_cnt = nullptr;
    a.tile_off = nullptr;
    a.total = nullptr;
    a.out = nullptr;
    a.cap = 0;
    return a;
}

hipError_t launch_count(const Plan &plan, const uint8_t *d_text, uint64_t n, const Params *d_params,
                        const uint8_t *d_pat, uint32_t *d_tile_cnt, uint64_t *d_total,
                        uint64_t ntiles, hipStream_t stream)
{
    ScanArgs a = make_args(plan, d_text, n, d_params, d_pat, ntiles);
    a.tile_cnt = d_tile_cnt;
    a.total = d_total;
    return launch_scan_any<false>(plan, a, stream);
}

hipError_t launch_scan(const uint32_t *d_tile_cnt, uint64_t ntiles, uint64_t *d_tile_off,
                       uint64_t *d_total, hipStream_t stream)
{
    if (ntiles == 0) return hipSuccess;
    hipLaunchKernelGGL(tile_scan_kernel, dim3(1), dim3(1024), 0, stream, d_tile_cnt, ntiles,
                       d_tile_off, d_total);
    return hipGetLastError();
}

hipError_t launch_write(const Plan &plan, const uint8_t *d_text, uint64_t n, const Params *d_params,
                        const uint8_t *d_pat, const uint32_t *d_tile_cnt,
                        const uint64_t *d_tile_off, int64_t *d_out, uint64_t cap, uint64_t ntiles,
                        hipStream_t stream)
{
    if (cap == 0) return hipSuccess;
    ScanArgs a = make_args(plan, d_text, n, d_params, d_pat, ntiles);
    a.tile_cnt = const_cast<uint32_t *>(d_tile_cnt);
    a.tile_off = d_tile_off;
    a.out = d_out;
    a.cap = cap;
    return launch_scan_any<true>(plan, a, stream);
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
