/*
 * Seeded synthetic input generators for the exact string matching workloads.
 *
 * This module only produces inputs (texts and random draws). It contains none
 * of the matching arithmetic, and both the CPU oracle and the GPU library are
 * fed from it.
 *
 * Random numbers come from a counter-based SplitMix64 stream (Steele, Lea and
 * Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014):
 *
 *     key      = mix64(seed * GAMMA ^ stream)
 *     value(i) = mix64(key + (i + 1) * GAMMA)            (all mod 2^64)
 *
 * with mix64 the SplitMix64 finaliser. Because value(i) depends only on
 * (seed, stream, i), any slice of a stream can be generated independently and
 * in parallel, and the numpy twin in __init__.py reproduces it bit for bit.
 *
 * Texts of the paper's experiments are i.i.d. uniform over sigma symbols
 * ("Rand sigma" buffers); the natural-language corpora are replaced by order-0
 * Zipf texts whose CDF is supplied by the caller (computed once in Python so
 * that both implementations use the identical table).
 */
#include <stdint.h>
#include <stddef.h>

#define DG_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t dg_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline uint64_t dg_key(uint64_t seed, uint64_t stream)
{
    return dg_mix64(seed * DG_GAMMA ^ stream);
}

/* raw 64-bit draws value(start) .. value(start + count - 1) */
void dg_u64(uint64_t *out, uint64_t count, uint64_t seed, uint64_t stream, uint64_t start)
{
    const uint64_t key = dg_key(seed, stream);
#pragma omp parallel for schedule(static) if (count > (1u << 20))
    for (int64_t i = 0; i < (int64_t)count; i++)
        out[i] = dg_mix64(key + ((uint64_t)i + start + 1) * DG_GAMMA);
}

/* byte(i) = (value(i) >> 32) mod sigma, sigma in [1, 256] */
void dg_uniform(uint8_t *out, uint64_t count, uint32_t sigma, uint64_t seed, uint64_t stream,
                uint64_t start)
{
    const uint64_t key = dg_key(seed, stream);
#pragma omp parallel for schedule(static) if (count > (1u << 20))
    for (int64_t i = 0; i < (int64_t)count; i++) {
        uint64_t x = dg_mix64(key + ((uint64_t)i + start + 1) * DG_GAMMA);
        out[i] = (uint8_t)((x >> 32) % sigma);
    }
}

/*
 * Order-0 inverse-CDF sampling: u = (value(i) >> 11) * 2^-53 in [0, 1);
 * byte = smallest k with u < cdf[k]  (cdf[K-1] must be >= 1.0).
 */
void dg_zipf(uint8_t *out, uint64_t count, const double *cdf, uint32_t K, uint64_t seed,
             uint64_t stream, uint64_t start)
{
    const uint64_t key = dg_key(seed, stream);
#pragma omp parallel for schedule(static) if (count > (1u << 18))
    for (int64_t i = 0; i < (int64_t)count; i++) {
        uint64_t x = dg_mix64(key + ((uint64_t)i + start + 1) * DG_GAMMA);
        double u = (double)(x >> 11) * (1.0 / 9007199254740992.0);
        uint32_t lo = 0, hi = K - 1;
        while (lo < hi) {
            uint32_t mid = (lo + hi) >> 1;
            if (u < cdf[mid]) hi = mid; else lo = mid + 1;
        }
        out[i] = (uint8_t)lo;
    }
}

/* fill with byte a, and byte b at every index i with i % period == period - 1 */
void dg_periodic(uint8_t *out, uint64_t count, uint8_t a, uint8_t b, uint64_t period, uint64_t start)
{
#pragma omp parallel for schedule(static) if (count > (1u << 20))
    for (int64_t i = 0; i < (int64_t)count; i++) {
        uint64_t g = (uint64_t)i + start;
        out[i] = (period && g % period == period - 1) ? b : a;
    }
}
