/* The oracle's naive search against its KMP on random texts, built with address
 * and undefined-behaviour sanitizers: any out-of-bounds access or UB in either
 * ends the run with a report; any disagreement prints FAIL. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

uint64_t oracle_naive(const uint8_t *t, uint64_t n, const uint8_t *p, uint64_t m, uint64_t lo,
                      uint64_t hi, int64_t *out, uint64_t cap);
uint64_t oracle_kmp(const uint8_t *t, uint64_t n, const uint8_t *p, uint64_t m, int64_t *out,
                    uint64_t cap, int64_t *fail);

static uint64_t s = 88172645463325252ull;
static uint64_t rnd(void)
{
    s ^= s << 13;
    s ^= s >> 7;
    s ^= s << 17;
    return s;
}

int main(void)
{
    for (int it = 0; it < 20000; it++) {
        const uint64_t n = rnd() % 300, m = 1 + rnd() % 12, sigma = 1 + rnd() % 4;
        uint8_t *t = malloc(n ? n : 1), *p = malloc(m);
        for (uint64_t i = 0; i < n; i++) t[i] = (uint8_t)(rnd() % sigma);
        for (uint64_t i = 0; i < m; i++) p[i] = (uint8_t)(rnd() % sigma);
        if (n >= m && rnd() % 2) memcpy(p, t + rnd() % (n - m + 1), m);  /* planted */
        const uint64_t cap = rnd() % 2 ? n + 1 : rnd() % 4;
        int64_t *a = malloc(sizeof(int64_t) * (cap ? cap : 1)), *b = malloc(sizeof(int64_t) * (cap ? cap : 1));
        int64_t *fl = malloc(sizeof(int64_t) * (m + 1));
        const uint64_t ca = oracle_naive(t, n, p, m, 0, n, a, cap);
        const uint64_t cb = oracle_kmp(t, n, p, m, b, cap, fl);
        const uint64_t k = ca < cap ? ca : cap;
        if (ca != cb || memcmp(a, b, k * sizeof(int64_t)) != 0) {
            printf("FAIL n=%llu m=%llu\n", (unsigned long long)n, (unsigned long long)m);
            return 1;
        }
        free(t), free(p), free(a), free(b), free(fl);
    }
    printf("ok\n");
    return 0;
}
