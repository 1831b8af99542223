/*
 * CPU oracle for exact string matching -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may load
 * this file's library. The GPU library never calls it and shares no code with
 * it.
 *
 * What is computed (paper, Section 1, problem statement): given a text t of
 * length n and a pattern p of length m over an alphabet, report ALL
 * occurrences of p in t. Read here as 0-based byte offsets, overlapping
 * occurrences included, in ascending order:
 *
 *     occ(t, p) = { i : 0 <= i <= n - m  and  t[i + k] = p[k] for 0 <= k < m }
 *
 * oracle_naive is that definition written out: the Brute-Force algorithm of
 * the paper's Fig. 1 (first row), which tests every window left to right.
 * oracle_kmp is an independent cross-check with the Knuth-Morris-Pratt
 * algorithm of the same figure (failure function over pattern borders).
 *
 * Parity pins (no worked example exists in the paper): KMP agreement, a regex
 * library's overlapping search, exhaustive binary texts with a closed-form
 * total, closed forms for periodic texts, planted occurrences, edge cases.
 */
#include <stdint.h>
#include <stddef.h>

/*
 * Naive search restricted to candidate starts lo <= i < hi.
 * Writes the first `cap` positions (ascending) to out and returns the total
 * number of occurrences in the range. m == 0 is not a valid pattern: returns 0.
 */
uint64_t oracle_naive(const uint8_t *t, uint64_t n, const uint8_t *p, uint64_t m, uint64_t lo,
                      uint64_t hi, int64_t *out, uint64_t cap)
{
    if (m == 0 || m > n)
        return 0;
    uint64_t end = n - m + 1; /* one past the largest admissible start */
#if ORACLE_MUTANT == 1
    end = n - m; /* planted: drops the last admissible start */
#endif
    if (hi > end)
        hi = end;
    uint64_t cnt = 0;
    for (uint64_t i = lo; i < hi; i++) {
        uint64_t k = 0;
#if ORACLE_MUTANT == 2
        while (k + 1 < m && t[i + k] == p[k]) /* planted: ignores the last byte */
            k++;
        if (k + 1 == m)
            k = m;
#elif ORACLE_MUTANT == 3
        while (k < m && t[i + k] == p[m - 1 - k]) /* planted: pattern read reversed */
            k++;
#else
        while (k < m && t[i + k] == p[k])
            k++;
#endif
        if (k == m) {
            if (cnt < cap)
                out[cnt] = (int64_t)i;
            cnt++;
#if ORACLE_MUTANT == 4
            i += m - 1; /* planted: non-overlapping occurrences only */
#endif
        }
    }
#if ORACLE_MUTANT == 5
    if (cnt > 0 && cnt <= cap)
        out[cnt - 1] += 1; /* planted: off-by-one on the last reported position */
#endif
    return cnt;
}

/*
 * Knuth-Morris-Pratt. fail must hold m + 1 entries (caller-owned workspace).
 * fail[k] = length of the longest proper border of p[0..k-1]; the refinement
 * of KMP (strong borders) is not needed for correctness and is not used.
 */
uint64_t oracle_kmp(const uint8_t *t, uint64_t n, const uint8_t *p, uint64_t m, int64_t *out,
                    uint64_t cap, int64_t *fail)
{
    if (m == 0 || m > n)
        return 0;
    fail[0] = -1;
    int64_t b = -1;
    for (uint64_t k = 0; k < m; k++) {
        while (b >= 0 && p[b] != p[k])
            b = fail[b];
        b++;
        fail[k + 1] = b;
    }
    uint64_t cnt = 0;
    int64_t q = 0; /* length of the current match */
    for (uint64_t j = 0; j < n; j++) {
        while (q >= 0 && (q == (int64_t)m || p[q] != t[j]))
            q = fail[q];
        q++;
        if (q == (int64_t)m) {
            if (cnt < cap)
                out[cnt] = (int64_t)(j + 1 - m);
            cnt++;
        }
    }
    return cnt;
}
