// Device building blocks shared by the single-pattern and the batched kernels:
// tile staging, the per-lane scanners (Shift-And, BNDM, SBNDM, Hash-q), hit
// emitters, verification and per-pattern table construction.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "sm_internal.h"

namespace sm {
namespace dev {

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

// Block filter hash of 16 bytes (four little-endian words) to BF_H bits. Any
// hash is correct: every candidate is compared byte-exactly.
__device__ __forceinline__ uint32_t bf_hash(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3)
{
    uint32_t h = (w0 * 0x9E3779B1u) ^ (w1 * 0x85EBCA77u) ^ (w2 * 0xC2B2AE3Du) ^ (w3 * 0x27D4EB2Fu);
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    return h >> (32 - BF_H);
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
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Text bytes in flight from HBM to LDS: positions [x0, x1) (0 <= x0 < x1 <= n)
// as aligned 16-byte chunks, PER chunk loads per thread.
template <int PER>
struct Staged {
    u32x4 v[PER];
    uint32_t nch;
    int boff;  // byte offset in LDS of position x0 (inside the first aligned chunk)
};

template <int PER>
__device__ __forceinline__ void stage_issue(Staged<PER> &st, const uint8_t *text, uint64_t x0,
                                            uint64_t x1)
{
    const uintptr_t a0 = (uintptr_t)(text + x0);
    const uintptr_t c0 = a0 & ~(uintptr_t)15;
    const uintptr_t c1 = ((uintptr_t)(text + x1 - 1)) & ~(uintptr_t)15;
    st.nch = (uint32_t)((c1 - c0) >> 4) + 1;
    st.boff = (int)(a0 & 15);
    typedef __attribute__((address_space(1))) const u32x4 global_u32x4;
    global_u32x4 *src = (global_u32x4 *)(c0);  // the text is in global memory
#pragma unroll
    for (int k = 0; k < PER; k++) {
        const uint32_t u = threadIdx.x + BLOCK * k;
        if (u < st.nch) st.v[k] = __builtin_nontemporal_load(src + u);
    }
}

// SWZ selects the XOR-swizzled chunk layout used by the per-lane sequential
// readers (conflict-free 16-byte LDS reads at any power-of-two segment stride).
template <bool SWZ, int PER>
__device__ __forceinline__ void stage_commit(const Staged<PER> &st, uint4 *lds)
{
#pragma unroll
    for (int k = 0; k < PER; k++) {
        const uint32_t u = threadIdx.x + BLOCK * k;
        if (u < st.nch) {
            uint4 w;
            w.x = st.v[k].x;
            w.y = st.v[k].y;
            w.z = st.v[k].z;
            w.w = st.v[k].w;
            lds[SWZ ? swz(u) : u] = w;
        }
    }
}

// ---------------------------------------------------------------------------
// Emitters: where a lane's hits go.
// ---------------------------------------------------------------------------
// Every emitter has put(rel) for one hit (in ascending order); saturated() tells a
// bit-parallel scanner that further hits need only be counted, through add(k).
struct NoEmit {
    __device__ __forceinline__ void put(int) {}
    __device__ __forceinline__ bool saturated() const { return false; }
    __device__ __forceinline__ void add(uint32_t) {}
};

// int64 global positions, bounded by cap
// Positions into an output window: hit number idx goes to out[idx - lo] when
// lo <= idx < lo + span (one unsigned compare covers both ends).
struct PosEmit {
    int64_t *out;
    uint64_t idx, lo, span;
    uint64_t base;  // global position of relative position 0
    __device__ __forceinline__ void put(int rel)
    {
        const uint64_t r = idx - lo;
        if (r < span) out[r] = (int64_t)(base + (uint64_t)(int64_t)rel);
        idx++;
    }
    __device__ __forceinline__ bool saturated() const { return false; }
    __device__ __forceinline__ void add(uint32_t) {}
};

// u16 offsets into an LDS list
struct ListEmit {
    uint16_t *dst;
    uint32_t idx;
    __device__ __forceinline__ void put(int rel) { dst[idx++] = (uint16_t)rel; }
    __device__ __forceinline__ bool saturated() const { return false; }
    __device__ __forceinline__ void add(uint32_t) {}
};

// u16 offsets inside the tile (tile-local stash)
struct StashEmit {
    uint16_t *dst;
    uint32_t idx;
    __device__ __forceinline__ void put(int rel) { dst[idx++] = (uint16_t)rel; }
    __device__ __forceinline__ bool saturated() const { return false; }
    __device__ __forceinline__ void add(uint32_t) {}
};

// Hits as a bitmap of the lane's starts (bit i of w[i / 64] <-> start lo + i),
// kept in registers; the Shift-And scanner hands over whole hit masks.
template <int NW>
struct BitAcc {
    uint64_t w[NW] = {};
    // r: bit i <-> start lo + rel + i; every set bit lies in [0, 64 NW), rel > -32
    __device__ __forceinline__ void put_mask(int rel, uint32_t r)
    {
#pragma unroll
        for (int k = 0; k < NW; k++) {
            const int s = rel - 64 * k;
            if (NW > 1 && (s <= -32 || s >= 64)) continue;
            w[k] |= s >= 0 ? (uint64_t)r << s : (uint64_t)(r >> -s);
        }
    }
};
template <class E>
struct takes_masks {
    static constexpr bool value = false;
};
template <int NW>
struct takes_masks<BitAcc<NW>> {
    static constexpr bool value = true;
};
template <class E>
struct is_no_emit {
    static constexpr bool value = false;
};
template <>
struct is_no_emit<NoEmit> {
    static constexpr bool value = true;
};

// Shift-And, complemented (Shift-Or) form. W = state word; CHECK = bytes between
// hit checks (requires m - 1 + CHECK <= bits of W). MT = mask table entry: W, or
// a byte when m <= 8 (the masks' bits >= m are clear), so that the table index is
// the text byte itself, with no scaling.
//
// The lane owns the nl tile-relative starts lo .. lo + nl - 1 and reads 16-byte units
// ub + k, k = 0..K, where unit ub holds its first start's byte r bytes in; unit k ends
// the windows at relative ends lo - r + 16k + [0, 16). Units whose 16 ends all lie in
// the lane's range [e_lo, e_hi] = [lo + m - 1, lo + nl + m - 2] (k in [kf0, kf1]) take
// every hit; only the units before and after them mask the ends of other lanes' starts
// (SPLIT: with these bounds uniform; otherwise every unit is masked).
template <typename W, int CHECK, bool WRITE, bool SPLIT, class E, typename MT>
__device__ __forceinline__ uint32_t shift_and_units(const uint4 *lds, const MT *mask, int m, int li0, int ub,
                                                   int r, int nl, E &o)
{
    const int K = (r + nl + m - 2) >> 4;
    const int kf0 = (m - 1 + r + 15) >> 4, kf1 = (nl + m - 17 + r) >> 4;
    W D = ~(W)0;
    uint32_t cnt = 0;
    auto unit = [&](int k, auto interior) {
        const int u = ub + k;
        const uint4 v = lds[swz((uint32_t)u)];
        const uint32_t wd[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int g = 0; g < 16 / CHECK; g++) {
            if constexpr (CHECK == 16 && sizeof(W) == 4) {
                // the 16 steps D = (D << 1) | B[c] at once: D << 16 | OR_b B[c_b] << (15 - b),
                // the masks merged pairwise (one shift-or each)
                // Each half's 8 lookups are merged before the next half's are issued, so
                // that at most 8 masks are held at once.
                W x[16];
#pragma unroll
                for (int h = 0; h < 16; h += 8) {
#pragma unroll
                    for (int b = h; b < h + 8; b++) x[b] = (W)mask[(wd[b >> 2] >> (8 * (b & 3))) & 0xFFu];
#pragma unroll
                    for (int w = 1; w < 8; w *= 2) {
#pragma unroll
                        for (int b = h; b < h + 8; b += 2 * w) {
                            x[b] = (x[b] << w) | x[b + w];
                            // kept as one shift-or each: without this the compiler distributes
                            // the shifts (a shift per mask plus three-input ORs, 25 ops, not 15)
                            asm("" : "+v"(x[b]));
                        }
                    }
                    asm volatile("" : "+v"(x[h])::"memory");
                }
                x[0] = (x[0] << 8) | x[8];
                asm("" : "+v"(x[0]));
                D = (D << 16) | x[0];
            } else {
#pragma unroll
                for (int b = 0; b < CHECK; b++) {
                    const int k2 = g * CHECK + b;
                    const uint32_t c = (wd[k2 >> 2] >> (8 * (k2 & 3))) & 0xFFu;
                    D = (D << 1) | (W)mask[c];
                }
            }
            // relative end of the last byte consumed, and its distance past the lane's first
            // and last ends (16 u - li0 = lo + 16 k - r: with r and nl uniform, so are these)
            const int e_last = 16 * u + g * CHECK + CHECK - 1 - li0;
            const int past_lo = 16 * k - r + g * CHECK + CHECK - 1 - (m - 1);  // e_last - e_lo
            const int past_hi = past_lo - (nl - 1);                            // e_last - e_hi
            uint32_t hits = (uint32_t)((~D) >> (m - 1)) & ((1u << CHECK) - 1u);
            if constexpr (!decltype(interior)::value) {
                const int jlo = past_hi < 0 ? 0 : past_hi;
                const int jhi = past_lo > CHECK - 1 ? CHECK - 1 : past_lo;
                hits = jlo <= jhi ? hits & ((2u << jhi) - 1u) & ~((1u << jlo) - 1u) : 0u;
            }
            if (hits) {
                if constexpr (takes_masks<E>::value) {
                    // reversed, bit i <-> end e_last - CHECK + 1 + i, i.e. start
                    // lo + (e_last - CHECK + 1 - e_lo) + i
                    o.put_mask(past_lo - CHECK + 1, __builtin_bitreverse32(hits) >> (32 - CHECK));
                    cnt += __builtin_popcount(hits);
                } else if (WRITE && o.saturated()) {
                    o.add((uint32_t)__builtin_popcount(hits));
                } else if (WRITE) {
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
    };
    using Edge = std::integral_constant<bool, false>;
    using Inner = std::integral_constant<bool, true>;
    int k = 0;
    if constexpr (SPLIT) {
        for (; k < kf0; k++) unit(k, Edge{});
        for (; k <= kf1; k++) unit(k, Inner{});
    }
    for (; k <= K; k++) unit(k, Edge{});
    return cnt;
}

// LN > 0 with full: a lane of LN starts at a multiple of 16 (a whole tile of the count
// pass), so r, K, kf0 and kf1 are the same in every lane and the loops are uniform.
template <typename W, int CHECK, bool WRITE, int LN = 0, class E, typename MT = W>
__device__ __forceinline__ uint32_t lane_shift_and(const uint4 *lds, const MT *mask, int m, int li0,
                                                  int lo, int hi, E &o, bool full = false)
{
    if constexpr (LN > 0) {
        static_assert(LN % 16 == 0, "lanes start at multiples of 16");
        if (full)
            return shift_and_units<W, CHECK, WRITE, true>(lds, mask, m, li0, (lo + li0) >> 4, li0 & 15, LN, o);
    }
    if (lo > hi) return 0u;
    return shift_and_units<W, CHECK, WRITE, false>(lds, mask, m, li0, (lo + li0) >> 4, (lo + li0) & 15, hi - lo + 1,
                                                   o);
}

// BNDM: masks B[c] bit i set iff p[m-1-i] == c. Q > 1 is the q-gram form (BNDMq,
// Fig. 3): the window's last Q bytes are read at once (Q independent mask lookups
// combined by shifts); the suffixes shorter than Q are then not tested as prefixes of
// p, so the shift of a window is at most m - Q + 1. Needs Q <= m.
template <int Q, bool WRITE, class E>
__device__ __forceinline__ uint32_t lane_bndm(const uint8_t *lds8, const uint64_t *B, int m,
                                             int li0, int lo, int hi, E &o)
{
    const uint64_t HB = 1ull << (m - 1);
    const uint64_t ALL = ~0ull >> (64 - m);
    uint32_t cnt = 0;
    int pos = lo;
    while (pos <= hi) {
        const uint8_t *w = lds8 + li0 + pos;
        if (Q > 1) {
            // D after reading w[m - Q .. m - 1]: byte w[m-1-i] enters shifted by Q-1-i
            uint64_t D = B[w[m - Q]];
#pragma unroll
            for (int i = 0; i < Q - 1; i++) D &= B[w[m - 1 - i]] << (Q - 1 - i);
            int j = m - Q, last = m - Q + 1;
            while (D != 0) {
                if (D & HB) {
                    if (j > 0) {
                        last = j;
                    } else {
                        if (WRITE) o.put(pos); else cnt++;
                        break;
                    }
                }
                if (j == 0) break;
                D <<= 1;
                j--;
                D &= B[w[j]];
            }
            pos += last;
            continue;
        }
        int j = m, last = m;
        uint64_t D = ALL;
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

// FSBNDM (Forward SBNDM, Fig. 3): SBNDM for p' = p x, the pattern followed by one
// position x that matches any byte, over windows of m + 1 bytes: the byte after
// the window is read first (a look-ahead, as in Sunday's Quick Search). The masks of
// p' are B'[c] = (B[c] << 1) | 1 (bit 0 is x). An occurrence of p' at pos is one of p;
// a window whose last k bytes are not a factor of p' is left with a shift of
// m + 2 - k. fwd_hi: the last start whose byte after the window lies in the text;
// later starts take x alone. After an occurrence the shift is p's smallest period
// (p and p' have the same periods). Needs m <= 63.
template <bool WRITE, class E>
__device__ __forceinline__ uint32_t lane_fsbndm(const uint8_t *lds8, const uint64_t *B, int m,
                                               int period, int li0, int lo, int hi, int fwd_hi, E &o)
{
    const uint64_t HB = 1ull << m;  // the first byte of p in p'
    uint32_t cnt = 0;
    int pos = lo;
    while (pos <= hi) {
        const uint8_t *w = lds8 + li0 + pos;  // window w[0 .. m-1], look-ahead w[m]
        uint64_t D = pos <= fwd_hi ? ((B[w[m]] << 1) | 1ull) : 1ull;
        int k = 1;
        while (D != 0 && k <= m) {
            D = (D << 1) & ((B[w[m - k]] << 1) | 1ull);
            k++;
        }
        if (D & HB) {  // all m + 1 positions read and matched
            if (WRITE) o.put(pos); else cnt++;
            pos += period;
        } else {
            pos += m + 2 - k;
        }
    }
    return cnt;
}

// SBNDM: same masks; no prefix tracking; shift m-k+1 when the k-byte suffix is
// not a factor of p; after a hit, shift by the smallest period of p. Q > 1 is the
// q-gram form (SBNDMq, Fig. 3): the window's last Q bytes are read at once (Q
// independent mask lookups combined by shifts) and a window whose Q-byte suffix
// is not a factor of p is left with a shift of m-Q+1. Needs Q <= m.
template <int Q, bool WRITE, class E>
__device__ __forceinline__ uint32_t lane_sbndm(const uint8_t *lds8, const uint64_t *B, int m,
                                              int period, int li0, int lo, int hi, E &o)
{
    const uint64_t HB = 1ull << (m - 1);
    uint32_t cnt = 0;
    int pos = lo;
    while (pos <= hi) {
        const uint8_t *w = lds8 + li0 + pos;  // window bytes w[0 .. m-1]
        uint64_t D;
        int k;
        if (Q > 1) {
            // D after Q steps of D = (D << 1) & B[byte]: byte w[m-1-i] enters shifted by Q-1-i
            D = B[w[m - Q]];
#pragma unroll
            for (int i = 0; i < Q - 1; i++) D &= B[w[m - 1 - i]] << (Q - 1 - i);
            if (D == 0) {
                pos += m - Q + 1;
                continue;
            }
            k = Q;
        } else {
            D = B[w[m - 1]];
            k = 1;
        }
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

// 16 bytes starting at byte address p, assembled from aligned words. Only words
// whose first byte is <= last (the last byte that may be read) are loaded; the
// others read as zero.
__device__ __forceinline__ uint4 load16(const uint8_t *p, const uint8_t *last)
{
    const uintptr_t a = (uintptr_t)p;
    const uint32_t *W = reinterpret_cast<const uint32_t *>(a & ~(uintptr_t)3);
    const uint32_t sh = (uint32_t)(a & 3);
    const uintptr_t wl = (uintptr_t)last & ~(uintptr_t)3;  // last loadable word
    uint32_t w[5];
#pragma unroll
    for (int k = 0; k < 5; k++) w[k] = ((uintptr_t)(W + k) <= wl) ? W[k] : 0u;
    uint4 r;
    r.x = alignbyte(w[1], w[0], sh);
    r.y = alignbyte(w[2], w[1], sh);
    r.z = alignbyte(w[3], w[2], sh);
    r.w = alignbyte(w[4], w[3], sh);
    return r;
}

// nonzero iff the first nb (<= 16) bytes of x and y differ
__device__ __forceinline__ uint32_t diff16(uint4 x, uint4 y, uint32_t nb)
{
    uint32_t d = 0;
    d |= (x.x ^ y.x) & byte_mask((int)nb);
    d |= (x.y ^ y.y) & byte_mask((int)nb - 4 < 0 ? 0 : (int)nb - 4);
    d |= (x.z ^ y.z) & byte_mask((int)nb - 8 < 0 ? 0 : (int)nb - 8);
    d |= (x.w ^ y.w) & byte_mask((int)nb - 12 < 0 ? 0 : (int)nb - 12);
    return d;
}

// Compare t[g + off, g + off + len) with p[off, off + len) for len <= 16, where
// g is the window's global start and the window [g, g + m) lies inside the text.
__device__ __forceinline__ bool verify_lane16(const uint8_t *text, uint64_t g, const uint8_t *pat,
                                              uint32_t m, uint32_t off, uint32_t len)
{
    return diff16(load16(text + g + off, text + g + m - 1), load16(pat + off, pat + m + 15), len) == 0;
}

// The same comparison, any len, by a whole wave: lane k takes bytes [16k, 16k + 16) of
// each 1024-byte block. Every lane of the wave must call it with the same
// arguments; the result is the same on all lanes.
__device__ __forceinline__ bool verify_wave(const uint8_t *text, uint64_t g, const uint8_t *pat,
                                            uint32_t m, uint32_t off, uint32_t len)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint8_t *tlast = text + g + m - 1;
    const uint8_t *plast = pat + m + 15;
    uint32_t d = 0;
    for (uint32_t b = 0; b < len; b += 1024) {
        const uint32_t o = b + 16 * lane;
        if (o < len)
            d |= diff16(load16(text + g + off + o, tlast), load16(pat + off + o, plast),
                        len - o < 16 ? len - o : 16);
        if (__ballot(d != 0)) return false;
    }
    return true;
}

// Suffix forms for long patterns: the scan finds the pattern's last SFX bytes
// (Shift-And for m > SA_SUFFIX, SFX = SA_SUFFIX or SA_SHORT; SBNDM for m > 64, its
// factor form); each such start
// g is an occurrence when the first m - SFX bytes match too, read from global
// memory. A start exactly one period (<= SFX) after the lane's previous occurrence
// needs no reading: bytes [0, m - period) repeat that occurrence shifted by the
// period, and the rest lie inside the suffix (the memory idea of Apostolico-Giancarlo
// and Turbo-BM, Fig. 1). Starts come in ascending order; they are passed on to the
// emitter o.
template <class E, int SFX = SA_SUFFIX>
struct SuffixVerify {
    E &o;
    const uint8_t *text0, *pat;
    uint32_t m, period;    // period: the smallest when <= SFX, else 0 (no shortcut)
    uint64_t s;            // tile start (global start of tile-relative start 0)
    int lo;                // the lane's first tile-relative start (bitmap emitters)
    uint64_t last = ~0ull; // this lane's last occurrence
    uint32_t n = 0;
    __device__ __forceinline__ void put(int rel)
    {
        const uint64_t g = s + (uint64_t)rel;
        bool ok = period != 0 && last != ~0ull && g - last == period;
        if (!ok) {  // 64 bytes per round trip: four independent 16-byte loads of each
            ok = true;
            const uint32_t len = m - (uint32_t)SFX;
            const uint8_t *tl = text0 + g + m - 1, *pl = pat + m + 15;
            for (uint32_t off = 0; off < len && ok; off += 64) {
                uint32_t d = 0;
#pragma unroll
                for (uint32_t k = 0; k < 4; k++) {
                    const uint32_t o2 = off + 16 * k;
                    if (o2 < len)
                        d |= diff16(load16(text0 + g + o2, tl), load16(pat + o2, pl), len - o2 < 16 ? len - o2 : 16);
                }
                ok = d == 0;
            }
        }
        if (ok) {
            if constexpr (takes_masks<E>::value) o.put_mask(rel - lo, 1u);
            else o.put(rel);
            last = g;
            n++;
        }
    }
    __device__ __forceinline__ bool saturated() const { return false; }
    __device__ __forceinline__ void add(uint32_t) {}
};

// 16 bytes at byte index idx of an LDS tile in the swizzled chunk layout (the
// chunk holding idx and the next one must be staged).
__device__ __forceinline__ uint4 lds_bytes16(const uint4 *lds, uint32_t idx)
{
    const uint32_t u = idx >> 4, r = idx & 15;
    const uint4 c0 = lds[swz(u)], c1 = lds[swz(u + 1)];
    const uint32_t w[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
    const uint32_t q = r >> 2, sh = r & 3;
    uint32_t v[5];
#pragma unroll
    for (int k = 0; k < 5; k++)
        v[k] = q == 0 ? w[k] : (q == 1 ? w[k + 1] : (q == 2 ? w[k + 2] : w[k + 3]));
    uint4 o;
    o.x = alignbyte(v[1], v[0], sh);
    o.y = alignbyte(v[2], v[1], sh);
    o.z = alignbyte(v[3], v[2], sh);
    o.w = alignbyte(v[4], v[3], sh);
    return o;
}

__device__ __forceinline__ uint4 readlane4(uint4 v, int k)
{
    uint4 r;
    r.x = (uint32_t)__builtin_amdgcn_readlane((int)v.x, k);
    r.y = (uint32_t)__builtin_amdgcn_readlane((int)v.y, k);
    r.z = (uint32_t)__builtin_amdgcn_readlane((int)v.z, k);
    r.w = (uint32_t)__builtin_amdgcn_readlane((int)v.w, k);
    return r;
}

// Where the suffix form reads a candidate's first m - sfx bytes (sfx: the suffix the
// scan matched): the LDS tile holds the (shifted) text from tile-relative position -li0
// on, so a candidate at tile-relative start rel has them in LDS from byte index
// li0 + rel - (m - sfx) when that is >= 0; the pattern's first 1024 bytes sit in
// registers, 16 per lane (lane k: bytes [16 k, 16 k + 16)).
struct SuffixCtx {
    const uint8_t *text0, *pat;  // original text, pattern copy (zero padded)
    const uint4 *lds;            // the staged tile
    int li0;                     // LDS byte index of tile-relative start 0 (shifted text)
    uint64_t s;                  // global start of tile-relative start 0
    uint32_t m, sfx, period;     // period: the smallest when <= sfx, else 0
    uint4 ppre;                  // pattern bytes [16 lane, 16 lane + 16)
};

// Is the candidate at tile-relative start rel an occurrence? Wave-cooperative: all
// lanes call it with the same rel.
__device__ __forceinline__ bool suffix_check_wave(const SuffixCtx &c, int rel)
{
    const uint32_t len = c.m - c.sfx;
    const int b0 = c.li0 + rel - (int)len;  // LDS index of the candidate's first byte
    const uint32_t lane = threadIdx.x & 63;
    if (b0 < 0 || len > 1024) return verify_wave(c.text0, c.s + (uint64_t)rel, c.pat, c.m, 0, len);
    const uint32_t o = 16 * lane;
    uint32_t d = 0;
    if (o < len) d = diff16(lds_bytes16(c.lds, (uint32_t)b0 + o), c.ppre, len - o < 16 ? len - o : 16);
    return __ballot(d != 0) == 0;
}

// The same check by one lane for its own candidate (uniform loop bounds).
__device__ __forceinline__ bool suffix_check_lane(const SuffixCtx &c, int rel, bool active)
{
    const uint32_t len = c.m - c.sfx;
    const int b0 = c.li0 + rel - (int)len;
    bool ok = true;
    if (active && b0 >= 0 && len <= 1024) {
        uint32_t d = 0;
        for (uint32_t o = 0; o < len; o += 16)  // the pattern's 16 bytes from lane o / 16
            d |= diff16(lds_bytes16(c.lds, (uint32_t)b0 + o), readlane4(c.ppre, (int)(o >> 4)),
                        len - o < 16 ? len - o : 16);
        ok = d == 0;
    } else if (active) {
        const uint64_t g = c.s + (uint64_t)rel;
        const uint8_t *tl = c.text0 + g + c.m - 1, *pl = c.pat + c.m + 15;
        for (uint32_t off = 0; off < len && ok; off += 64) {
            uint32_t d = 0;
#pragma unroll
            for (uint32_t q = 0; q < 4; q++) {
                const uint32_t o2 = off + 16 * q;
                if (o2 < len)
                    d |= diff16(load16(c.text0 + g + o2, tl), load16(c.pat + o2, pl), len - o2 < 16 ? len - o2 : 16);
            }
            ok = d == 0;
        }
    }
    return ok;
}

// The suffix form's candidates, settled after the scan: ba holds the lane's starts
// whose last sfx bytes match (bit i <-> tile-relative start lo + i) and keeps
// those that are occurrences. Each lane walks its candidates in ascending order; a
// start exactly one period (<= sfx) after the lane's previous occurrence is
// one without reading (as in SuffixVerify). The others compare their first
// m - sfx bytes with the pattern, from the LDS tile where it holds them:
// when few lanes of the wave have such a candidate at once the whole wave checks
// each of them, 16 bytes per lane; when many do (a text of one symbol: every lane's
// first candidate), each lane checks its own. Wave-cooperative: all 64 lanes call
// it (lanes without starts pass an empty ba). Outside the scan loop, the
// verification's registers do not weigh on the scan.
template <int L, int NW>
__device__ __forceinline__ uint32_t suffix_resolve(BitAcc<NW> &ba, const SuffixCtx &c, int lo)
{
    static_assert(NW <= 2 && L <= 64 * NW, "at most 128 starts per lane");
    constexpr uint64_t FULL0 = L >= 64 ? ~0ull : ((1ull << (L & 63)) - 1ull);  // the lane's bits of word 0
    constexpr uint32_t COOP_MAX = 8;  // lanes checked one after another by the whole wave
    const int lane = (int)(threadIdx.x & 63);
    const uint32_t period = c.period;
    uint64_t x0 = ba.w[0], x1 = NW > 1 ? ba.w[NW > 1 ? 1 : 0] : 0ull;  // candidates left
    uint64_t k0 = 0, k1 = 0;                                        // occurrences
    uint32_t cnt = 0;
    int last = -(1 << 20);  // lane-relative start of the lane's last occurrence
    if (period == 1) {
        // Every start of a lane a candidate (a text of one symbol): the lane's starts are
        // one period apart, so they are all occurrences when its first one is; and when
        // the previous lane is full too, that first start is one period after the previous
        // lane's last. So only the first lane of each run of full lanes is checked.
        const bool full = x0 == FULL0 && (NW == 1 || x1 == ~0ull);
        const uint64_t F = __ballot(full);
        const bool head = full && !(lane > 0 && ((F >> (lane - 1)) & 1ull));
        const uint64_t H = __ballot(head);
        if (F && (uint32_t)__builtin_popcountll(H) <= COOP_MAX) {
            uint64_t p = H, bad = 0;
            while (p) {
                const int kl = __builtin_ctzll(p);
                p &= p - 1;
                if (!suffix_check_wave(c, __shfl(lo, kl, 64))) bad |= 1ull << kl;
            }
            if (!bad) {  // uniform: every full lane holds occurrences only
                if (full) {
                    k0 = x0;
                    k1 = x1;
                    cnt = L;
                    last = L - 1;
                    x0 = x1 = 0;
                }
            }
        }
    }
    for (;;) {
        // 1. accept what the period rule settles; stop at a candidate that needs reading
        int r = -1;
        while (x0 | x1) {
            const bool lo_word = x0 != 0;
            const int b = __builtin_ctzll(lo_word ? x0 : x1);
            if (lo_word) x0 &= x0 - 1;
            else x1 &= x1 - 1;
            const int rr = (lo_word ? 0 : 64) + b;
            if (period != 0 && rr - last == (int)period) {
                if (lo_word) k0 |= 1ull << b;
                else k1 |= 1ull << b;
                last = rr;
                cnt++;
                // a run of consecutive starts one period apart (period 1: a text of one symbol)
                if (period == 1 && b < 63) {
                    if (lo_word && x0 != 0 && x0 == (FULL0 & (~0ull << (b + 1)))) {
                        k0 |= x0;
                        cnt += (uint32_t)__builtin_popcountll(x0);
                        last = 63 - __builtin_clzll(x0 | 1ull);
                        x0 = 0;
                    } else if (!lo_word && x1 == ~0ull << (b + 1)) {
                        k1 |= x1;
                        cnt += (uint32_t)__builtin_popcountll(x1);
                        last = 127;
                        x1 = 0;
                    }
                }
                continue;
            }
            r = rr;
            break;
        }
        const uint64_t pend = __ballot(r >= 0);
        if (!pend) break;
        // 2. check the pending candidates
        bool ok = false;
        if ((uint32_t)__builtin_popcountll(pend) <= COOP_MAX) {
            uint64_t p = pend;
            while (p) {
                const int kl = __builtin_ctzll(p);
                p &= p - 1;
                const bool v = suffix_check_wave(c, __shfl(lo + r, kl, 64));
                if (lane == kl) ok = v;
            }
        } else {
            ok = suffix_check_lane(c, lo + r, r >= 0);
        }
        if (r >= 0 && ok) {
            if (r < 64) k0 |= 1ull << r;
            else k1 |= 1ull << (r - 64);
            last = r;
            cnt++;
        }
    }
    ba.w[0] = k0;
    if (NW > 1) ba.w[NW > 1 ? 1 : 0] = k1;
    return cnt;
}

// Brute force (Fig. 1, BF) over packed bytes, m <= BRUTE_MAX_M. For the four
// starts of a text word, word k of the text shifted by k bytes is compared with
// p[k] replicated in all four bytes (pw[k]); a start matches when its byte is
// zero in the OR of the m differences. The exact zero-byte test sets 0x80 in
// each zero byte; a multiply gathers the four flags. Hits come as masks of the
// 16 starts of an LDS unit, in ascending order, like Shift-And's.
template <bool WRITE, class E>
__device__ __forceinline__ uint32_t lane_brute(const uint4 *lds, const uint32_t *pw, int m, int li0,
                                               int lo, int hi, E &o)
{
    const int u0 = (lo + li0) >> 4, u1 = (hi + li0) >> 4;
    uint4 cur = lds[swz((uint32_t)u0)];
    uint32_t cnt = 0;
    for (int u = u0; u <= u1; u++) {
        const uint4 nx = lds[swz((uint32_t)(u + 1))];
        const uint32_t w[6] = {cur.x, cur.y, cur.z, cur.w, nx.x, nx.y};
        uint32_t z[4];
#pragma unroll
        for (int d = 0; d < 4; d++) {
            uint32_t x = w[d] ^ pw[0];
#pragma unroll
            for (int k = 1; k < BRUTE_MAX_M; k++)
                if (k < m) x |= alignbyte(w[d + (k >> 2) + 1], w[d + (k >> 2)], (uint32_t)(k & 3)) ^ pw[k];
            z[d] = ~(((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x) & 0x80808080u;
        }
        if (z[0] | z[1] | z[2] | z[3]) {
            uint32_t hits = 0;
#pragma unroll
            for (int d = 0; d < 4; d++) hits |= (((z[d] >> 7) * 0x10204080u) >> 28) << (4 * d);
            // bit i <-> relative start base + i; keep the lane's starts [lo, hi]
            const int base = 16 * u - li0;
            int ilo = lo - base, ihi = hi - base;
            ilo = ilo < 0 ? 0 : ilo;
            ihi = ihi > 15 ? 15 : ihi;
            hits &= ((2u << ihi) - 1u) & ~((1u << ilo) - 1u);
            if (hits) {
                if constexpr (takes_masks<E>::value) {
                    o.put_mask(base - lo, hits);
                    cnt += __builtin_popcount(hits);
                } else if (WRITE) {
                    while (hits) {
                        const int b = __builtin_ctz(hits);
                        hits &= hits - 1;
                        o.put(base + b);
                    }
                } else {
                    cnt += __builtin_popcount(hits);
                }
            }
        }
        cur = nx;
    }
    return cnt;
}

// ---------------------------------------------------------------------------
// Block filter (after SSEF, Fig. 1). An occurrence at i contains the 16-byte block
// at x whenever i <= x <= i + m - 16, an interval of m - 15 starts; so blocks
// spaced S <= m - 15 apart meet every occurrence. With S a multiple of 16 they can
// all sit on aligned 16-byte chunks of memory (one load each, never two chunks), at
// x_b = b S + S - 1 - phi for the text's alignment phi; block b is the only one to
// test for the starts it owns, (x_b - S, x_b]: i = x_b - j for an alignment
// j <= x_b - ilo with p[j, j + 16) equal to the block. The text is read at one block
// per S bytes; the pattern's alignments j < m - 15 are bucketed by the block hash.
// ---------------------------------------------------------------------------
// Occurrences among the starts [ilo, ihi] of sampled block x (ilo <= ihi <= x,
// x - ilo < S <= m - 15, x + 16 <= n); blk = the block's 16 bytes. Wave-cooperative:
// all 64 lanes of the wave call it (lanes without starts pass active = false). A lane
// walks its bucket in descending j, i.e. ascending start i = x - j, skips the
// alignments whose start lies before ilo (another block's), and keeps the candidates
// whose p[j, j + 16) equals the block; the wave verifies them 1024 bytes per round
// trip. An occurrence v already found rules out starts closer than the pattern's
// smallest period, and one exactly a period away needs only its last period bytes.
template <bool WRITE, class E>
__device__ __forceinline__ uint32_t lane_block(const uint8_t *text, const uint8_t *pat, uint32_t m,
                                               const Params *prm, uint32_t period, uint32_t period_lb,
                                               uint64_t x, uint64_t ilo, uint64_t ihi, uint4 blk,
                                               bool active, uint64_t base, E &o)
{
    const uint32_t jmax = active ? (uint32_t)(x - ilo) : 0u;  // start x - j >= ilo
    uint32_t k = 0, k1 = 0;
    if (active) {
        const uint32_t h = bf_hash(blk.x, blk.y, blk.z, blk.w);
        k = prm->bf_start[h];
        k1 = prm->bf_start[h + 1];
    }
    active = active && k < k1;
    uint32_t cnt = 0;
    bool have = false;
    uint64_t v = 0;
    while (__ballot(active)) {
        // 1. this lane's next candidate
        bool cand = false;
        uint64_t i = 0;
        while (active && !cand) {
            const uint32_t j = prm->bf_js[k++];
            if (j > jmax) {  // the start is owned by an earlier block
                if (k >= k1) active = false;
                continue;
            }
            i = x - j;
            if (i > ihi) {
                active = false;  // j descending: the remaining starts are larger still
                break;
            }
            const uint4 pb = load16(pat + j, pat + m + 15);
            cand = ((pb.x ^ blk.x) | (pb.y ^ blk.y) | (pb.z ^ blk.z) | (pb.w ^ blk.w)) == 0;
            if (k >= k1) active = false;
        }
        // 2. the period rule, then a check by the lane (<= 16 bytes) or by the wave
        bool hit = false, need_wave = false;
        uint32_t voff = 0, vlen = m;
        if (cand && !(have && i - v < period_lb)) {
            if (have && period && i - v == period) {
                voff = m - period;
                vlen = period;
            }
            if (vlen <= 16) hit = verify_lane16(text, i, pat, m, voff, vlen);
            else need_wave = true;
        }
        uint64_t pend = __ballot(need_wave);
        while (pend) {
            const int kl = __builtin_ctzll(pend);
            pend &= pend - 1;
            const uint64_t ki = ((uint64_t)(uint32_t)__shfl((int)(uint32_t)(i >> 32), kl, 64) << 32) |
                                (uint32_t)__shfl((int)(uint32_t)i, kl, 64);
            const uint32_t koff = (uint32_t)__shfl((int)voff, kl, 64), klen = (uint32_t)__shfl((int)vlen, kl, 64);
            const bool ok = verify_wave(text, ki, pat, m, koff, klen);
            if ((int)(threadIdx.x & 63) == kl) hit = ok;
        }
        if (hit) {
            have = true;
            v = i;
            if (WRITE) o.put((int)(i - base));
            else cnt++;
        }
    }
    return cnt;
}

// Hash-q over the lane's windows. The LDS holds text positions from m-q on;
// li0 is the LDS index of relative position 0 (may be negative).
// Wave-cooperative: all 64 lanes of the wave call it (lanes without starts have
// lo > hi). A lane advances to its next candidate window (zero shift); a
// candidate is settled by the pattern's period when possible (two occurrences are
// at least the smallest period apart, period_lb bounds it from below; at distance
// exactly `period` -- the smallest period when known, else 0 -- from a verified
// occurrence only the last `period` bytes are new), by the lane itself when at most 64
// bytes remain to compare, and otherwise by the whole wave.
template <int NW, bool WRITE, class E>
__device__ __forceinline__ uint32_t lane_hashq(const uint32_t *lds32, const uint8_t *shift, int m,
                                              int q, int hbits, int sh1, int period, int period_lb,
                                              int li0, int lo, int hi, const uint8_t *text,
                                              uint64_t s, const uint8_t *pat, E &o)
{
    uint32_t cnt = 0;
    int pos = lo;
    bool active = lo <= hi;
    bool have_prev = false;  // a verified occurrence of this lane at prev
    int prev = 0;
    for (;;) {
        // 1. next candidate of this lane
        bool cand = false;
        while (active && !cand) {
            const int gs = li0 + pos + m - q;  // LDS index of the q-gram's first byte
            const int wi = gs >> 2, sb = gs & 3;
            uint32_t d[NW + 1];
#pragma unroll
            for (int k = 0; k <= NW; k++) d[k] = lds32[wi + k];
            uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
            for (int k = 0; k < NW; k++)
                w[k] = alignbyte(d[k + 1], d[k], (uint32_t)sb) & byte_mask(q - 4 * k);
            const int sh = shift[qhash(w[0], w[1], w[2], w[3], (uint32_t)hbits)];
            if (sh == 0) {
                cand = true;
            } else {
                pos += sh;
                active = pos <= hi;
            }
        }
        // 2. settle it: period rule, lane check, or mark for the wave
        bool hit = false, need_wave = false;
        uint32_t voff = 0, vlen = (uint32_t)m;
        if (cand) {
            const int dist = pos - prev;
            if (have_prev && dist < period_lb) {
                hit = false;  // closer than the smallest period to an occurrence: impossible
            } else {
                if (have_prev && dist == period && period < m) {
                    voff = (uint32_t)(m - period);
                    vlen = (uint32_t)period;
                }
                if (vlen <= 16) hit = verify_lane16(text, s + (uint64_t)pos, pat, (uint32_t)m, voff, vlen);
                else need_wave = true;
            }
        }
        uint64_t pend = __ballot(need_wave);
        while (pend) {
            const int k = __builtin_ctzll(pend);
            pend &= pend - 1;
            const int kpos = __shfl(pos, k, 64);
            const uint32_t koff = __shfl(voff, k, 64), klen = __shfl(vlen, k, 64);
            const bool ok = verify_wave(text, s + (uint64_t)kpos, pat, (uint32_t)m, koff, klen);
            if ((int)(threadIdx.x & 63) == k) hit = ok;
        }
        // 3. record and move on
        if (cand) {
            if (hit) {
                if (WRITE) o.put(pos); else cnt++;
                have_prev = true;
                prev = pos;
            }
            pos += sh1;
            active = pos <= hi;
        }
        if (!__ballot(active)) break;
    }
    return cnt;
}

// Tables of one pattern (masks, Hash-q shift table and sh1, period bounds) into
// *P, by one whole workgroup of BLOCK threads. pp: the pattern (global or LDS);
// s_tab: LDS scratch of 1 << H_MAX words; s_bad: LDS scratch of PERIOD_MAX + 1.
// LDS the block filter's table build takes (32-bit words)
constexpr int BF_BUILD_LDS = 2 * BF_MAX_M + 64;

// Block filter tables: the hash of every alignment j < S = m - 15 (every block a
// sampled block can meet), counts per
// bucket, their exclusive scan (bf_start); then each j goes to its bucket in any
// order (LDS atomics) and every bucket is sorted in descending j: buckets of at
// most 32 by one thread each (insertion sort), larger ones (periodic or
// repetitive patterns) one after another by the whole workgroup (bitonic sort).
// s_tab: 1 << BF_H words; s: BF_BUILD_LDS words (hashes, then sort scratch | the
// bucketed j | the list of large buckets).
__device__ __forceinline__ void build_block_tables(const uint8_t *pp, uint32_t m, Params *P,
                                                   uint32_t *s_tab, uint32_t *s, uint32_t *s_w)
{
    const uint32_t tid = threadIdx.x;
    const uint32_t S = m - 15, nb = 1u << BF_H;
    uint32_t *s_h = s, *s_js = s + BF_MAX_M, *s_big = s + 2 * BF_MAX_M;
    constexpr uint32_t SMALL = 32, BIG_MAX = 64;  // buckets > 32 (at most 123) are listed 64 at a time
    for (uint32_t k = tid; k < nb; k += BLOCK) s_tab[k] = 0;
    __syncthreads();
    for (uint32_t j = tid; j < S; j += BLOCK) {
        uint32_t w[4] = {0, 0, 0, 0};
#pragma unroll
        for (uint32_t k = 0; k < 16; k++) w[k >> 2] |= (uint32_t)pp[j + k] << (8 * (k & 3));
        const uint32_t h = bf_hash(w[0], w[1], w[2], w[3]);
        s_h[j] = h;
        atomicAdd(&s_tab[h], 1u);
    }
    __syncthreads();
    // exclusive scan of the nb counts, 16 per thread; s_tab becomes the cursors
    constexpr uint32_t PER = (1u << BF_H) / BLOCK;
    uint32_t bstart[PER];
    {
        uint32_t c[PER], sum = 0;
#pragma unroll
        for (uint32_t k = 0; k < PER; k++) {
            c[k] = s_tab[tid * PER + k];
            sum += c[k];
        }
        uint32_t tot;
        uint32_t run = block_excl_scan(sum, s_w, tot);  // ends with a barrier
#pragma unroll
        for (uint32_t k = 0; k < PER; k++) {
            bstart[k] = run;
            P->bf_start[tid * PER + k] = (uint16_t)run;
            s_tab[tid * PER + k] = run;
            run += c[k];
        }
        if (tid == 0) P->bf_start[nb] = (uint16_t)S;
    }
    __syncthreads();
    for (uint32_t j = tid; j < S; j += BLOCK) s_js[atomicAdd(&s_tab[s_h[j]], 1u)] = j;
    __syncthreads();
    // s_tab[h] is now the end of bucket h; small buckets: this thread's 16
#pragma unroll
    for (uint32_t k = 0; k < PER; k++) {
        const uint32_t b0 = bstart[k], b1 = s_tab[tid * PER + k];
        if (b1 - b0 <= SMALL) {
            for (uint32_t x = b0 + 1; x < b1; x++) {  // insertion sort, descending
                const uint32_t v = s_js[x];
                uint32_t y = x;
                while (y > b0 && s_js[y - 1] < v) {
                    s_js[y] = s_js[y - 1];
                    y--;
                }
                s_js[y] = v;
            }
        }
    }
    // large buckets, in passes of at most BIG_MAX listed ones
    for (uint32_t pass_lo = 0;; pass_lo += BIG_MAX) {  // uniform
        __syncthreads();
        // list the large buckets with rank in [pass_lo, pass_lo + BIG_MAX) in bucket order
        uint32_t mine = 0;
#pragma unroll
        for (uint32_t k = 0; k < PER; k++) mine += (s_tab[tid * PER + k] - bstart[k]) > SMALL;
        uint32_t tot;
        uint32_t rank = block_excl_scan(mine, s_w, tot);
#pragma unroll
        for (uint32_t k = 0; k < PER; k++) {
            if ((s_tab[tid * PER + k] - bstart[k]) > SMALL) {
                if (rank >= pass_lo && rank < pass_lo + BIG_MAX) s_big[rank - pass_lo] = tid * PER + k;
                rank++;
            }
        }
        __syncthreads();
        const uint32_t nlist = tot > pass_lo ? (tot - pass_lo < BIG_MAX ? tot - pass_lo : BIG_MAX) : 0;
        for (uint32_t q = 0; q < nlist; q++) {
            __syncthreads();  // the previous bucket's copy back is done with the scratch
            const uint32_t h = s_big[q];
            const uint32_t b0 = h ? s_tab[h - 1] : 0, b1 = s_tab[h], B = b1 - b0;
            uint32_t N = 64;
            while (N < B) N <<= 1;
            // scratch: j + 1, zero padding; bitonic sort descending
            for (uint32_t x = tid; x < N; x += BLOCK) s_h[x] = x < B ? s_js[b0 + x] + 1 : 0;
            for (uint32_t size = 2; size <= N; size <<= 1) {
                for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
                    __syncthreads();
                    for (uint32_t i = tid; i < N / 2; i += BLOCK) {
                        const uint32_t lo = 2 * i - (i & (stride - 1)), hi = lo + stride;
                        const bool down = (lo & size) == 0;
                        const uint32_t a = s_h[lo], b = s_h[hi];
                        if ((a < b) == down) {
                            s_h[lo] = b;
                            s_h[hi] = a;
                        }
                    }
                }
            }
            __syncthreads();
            for (uint32_t x = tid; x < B; x += BLOCK) s_js[b0 + x] = s_h[x] - 1;
        }
        if (tot <= pass_lo + BIG_MAX) break;
    }
    __syncthreads();
    for (uint32_t k = tid; k < S; k += BLOCK) P->bf_js[k] = (uint16_t)s_js[k];
}

__device__ __forceinline__ void build_tables(const uint8_t *pp, uint32_t m, uint32_t algo,
                                             uint32_t q_, uint32_t hbits, Params *P,
                                             uint32_t *s_tab, uint32_t *s_bad, uint32_t *s_key)  // s_key: BF_BUILD_LDS
{
    const int tid = threadIdx.x;
    if (algo == ALGO_SHIFT_AND) {
        // complemented masks: bit j clear iff p[j] == c (j < m); bits >= m clear. With
        // q_ = SA_SUFFIX or SA_SHORT (single-pattern suffix form, m > SA_SUFFIX) the masks
        // are those of the pattern's last q_ bytes.
        const uint32_t c = tid;
        const uint32_t ms = ((q_ == (uint32_t)SA_SUFFIX || q_ == (uint32_t)SA_SHORT) && m > (uint32_t)SA_SUFFIX) ? q_ : m;
        const uint8_t *ps = pp + (m - ms);
        uint64_t w = 0;
        for (uint32_t j = 0; j < ms; j++)
            if (ps[j] != c) w |= 1ull << j;
        P->mask[c] = w;
    } else if (algo == ALGO_BNDM || algo == ALGO_SBNDM || algo == ALGO_FSBNDM) {
        const uint32_t c = tid;
        uint64_t w = 0;
        for (uint32_t i = 0; i < m; i++)
            if (pp[m - 1 - i] == c) w |= 1ull << i;
        P->mask[c] = w;
    } else if (algo == ALGO_HASHQ) {
        const uint32_t q = q_, hb = hbits, nb = 1u << hb;
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
    } else if (algo == ALGO_BRUTE) {  // each pattern byte in the four bytes of a word
        if (tid < (uint32_t)BRUTE_MAX_M) P->mask[tid] = tid < m ? (uint32_t)pp[tid] * 0x01010101u : 0u;
    } else if (algo == ALGO_BLOCK && s_key) {
        build_block_tables(pp, m, P, s_tab, s_key, s_bad);
    }

    // Smallest period of p among 1..PERIOD_MAX: d is a period iff p[i] == p[i+d]
    // for all i < m - d. Four threads test each d. period = that d, or m when p
    // has no proper period <= m-1 (only decided for m <= PERIOD_MAX + 1), else 0
    // (unknown); period_lb is a lower bound on the smallest period.
    if (tid <= PERIOD_MAX) s_bad[tid] = 0;
    __syncthreads();
    {
        const uint32_t d = 1 + (tid >> 2), part = tid & 3;
        if (d <= PERIOD_MAX && d < m) {
            const uint32_t len = m - d;
            const uint32_t per = (len + 3) / 4;
            const uint32_t b = part * per, e = b + per < len ? b + per : len;
            for (uint32_t i = b; i < e; i++)
                if (pp[i] != pp[i + d]) {
                    s_bad[d] = 1;
                    break;
                }
        }
    }
    __syncthreads();
    if (tid < 64) {  // wave 0: lane d - 1 tests period d; the smallest is the first set bit
        static_assert(PERIOD_MAX == 64, "one lane per candidate period");
        const uint32_t d = tid + 1;
        const uint64_t ok = __ballot(d < m && !s_bad[d]);
        uint32_t per = ok ? (uint32_t)__builtin_ctzll(ok) + 1u : 0u;
        if (per == 0 && m <= PERIOD_MAX + 1) per = m;
        if (tid == 0) {
            P->period = per;
            P->period_lb = per ? per : PERIOD_MAX + 1;
        }
    }
}

}  // namespace dev
}  // namespace sm
