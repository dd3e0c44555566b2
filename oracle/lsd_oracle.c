/*
 * Plain CPU oracle for the LSD radix sort -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this file's library.  The product path (the HIP library) shares no
 * code, header, table or helper with it.
 *
 * What it computes (paper, Section 2.6 "Radix sort"): a key is split into
 * d digits of r bits; the sequence is sorted digit by digit from the least
 * to the most significant digit, each time with a *stable* counting sort,
 * which is what keeps equal digits in the order the previous digit left
 * them.  The end result is the unique stable ascending sort by unsigned key:
 * output position i holds the pair with the i-th smallest (key, input index).
 *
 * The counting sort of one digit is written as its three textbook steps,
 * in order, with no blocking or fusion:
 *   1. count:  cnt[b] = number of elements whose digit is b
 *   2. scan:   start[b] = sum of cnt[c] for c < b  (exclusive prefix sum)
 *   3. place:  walk the input in ascending index order and put element i at
 *              start[digit_i]++  (ascending order is the stability)
 *
 * Keys are handled as 64-bit words with a stated key width K (32 or 64);
 * values, when present, are carried along unchanged.  r may be any width in
 * [1, 16]; the number of passes is ceil(K / r), the last digit being the
 * K - (d-1)*r remaining bits.
 *
 * Every entry point returns 0 on success and -1 on a bad argument.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* digit p of key: bits [p*r, p*r + r) */
static uint64_t digit_of(uint64_t key, int p, int r)
{
    int shift = p * r;
    if (shift >= 64)
        return 0;
    return (key >> shift) & ((UINT64_C(1) << r) - 1);
}

static int num_passes(int key_bits, int r)
{
    return (key_bits + r - 1) / r;
}

/* Step 1 of the counting sort: cnt[b] for every digit value b. */
static void count_digits(const uint64_t *key, uint64_t n, int p, int r, uint64_t *cnt)
{
    uint64_t nb = UINT64_C(1) << r;
    for (uint64_t b = 0; b < nb; ++b)
        cnt[b] = 0;
    for (uint64_t i = 0; i < n; ++i)
        cnt[digit_of(key[i], p, r)] += 1;
}

/* Step 2: start[b] = cnt[0] + ... + cnt[b-1]. */
static void exclusive_scan(const uint64_t *cnt, uint64_t nb, uint64_t *start)
{
    uint64_t run = 0;
    for (uint64_t b = 0; b < nb; ++b) {
        start[b] = run;
        run += cnt[b];
    }
}

/* One stable counting-sort pass on digit p: (ka, va) -> (kb, vb). */
static void counting_pass(const uint64_t *ka, const uint64_t *va, uint64_t *kb, uint64_t *vb,
                          uint64_t n, int p, int r, uint64_t *cnt, uint64_t *start)
{
    uint64_t nb = UINT64_C(1) << r;
    count_digits(ka, n, p, r, cnt);
    exclusive_scan(cnt, nb, start);
    for (uint64_t i = 0; i < n; ++i) { /* ascending i: stability */
        uint64_t b = digit_of(ka[i], p, r);
        uint64_t dst = start[b]++;
        kb[dst] = ka[i];
        if (va)
            vb[dst] = va[i];
    }
}

/*
 * LSD radix sort of n 64-bit words holding K-bit keys, values optional.
 * passes_to_run < 0 runs all ceil(K/r) passes; otherwise only the first
 * passes_to_run, which exposes the state after each pass.
 */
static int lsd_sort_words(uint64_t *key, uint64_t *val, uint64_t n, int key_bits, int r,
                          int passes_to_run)
{
    if (r < 1 || r > 16 || (key_bits != 32 && key_bits != 64))
        return -1;
    int d = num_passes(key_bits, r);
    if (passes_to_run < 0 || passes_to_run > d)
        passes_to_run = d;
    if (n < 1 || passes_to_run == 0)
        return 0;
    uint64_t nb = UINT64_C(1) << r;
    uint64_t *kb = malloc(n * sizeof(uint64_t));
    uint64_t *vb = val ? malloc(n * sizeof(uint64_t)) : NULL;
    uint64_t *cnt = malloc(nb * sizeof(uint64_t));
    uint64_t *start = malloc(nb * sizeof(uint64_t));
    if (!kb || (val && !vb) || !cnt || !start) {
        free(kb); free(vb); free(cnt); free(start);
        return -1;
    }
    uint64_t *ka = key, *va = val;
    uint64_t *kt = kb, *vt = vb;
    for (int p = 0; p < passes_to_run; ++p) {
        counting_pass(ka, va, kt, vt, n, p, r, cnt, start);
        uint64_t *s;
        s = ka; ka = kt; kt = s;
        s = va; va = vt; vt = s;
    }
    if (ka != key) { /* result sits in the scratch buffer: move it home */
        memcpy(key, ka, n * sizeof(uint64_t));
        if (val)
            memcpy(val, va, n * sizeof(uint64_t));
    }
    free(kb);
    free(vb);
    free(cnt);
    free(start);
    return 0;
}

/* ---- exported entry points ------------------------------------------- */

/* Sort u32 keys (and u32 values if vals != NULL) in place; r-bit digits;
 * passes_to_run < 0 means all passes. */
int oracle_sort_u32(uint32_t *keys, uint32_t *vals, uint64_t n, int r, int passes_to_run)
{
    if (n > 0 && !keys)
        return -1;
    if (n == 0)
        return (r >= 1 && r <= 16) ? 0 : -1;
    uint64_t *k = malloc(n * sizeof(uint64_t));
    uint64_t *v = vals ? malloc(n * sizeof(uint64_t)) : NULL;
    if (!k || (vals && !v)) {
        free(k); free(v);
        return -1;
    }
    for (uint64_t i = 0; i < n; ++i) {
        k[i] = keys[i];
        if (vals)
            v[i] = vals[i];
    }
    int rc = lsd_sort_words(k, v, n, 32, r, passes_to_run);
    if (rc == 0) {
        for (uint64_t i = 0; i < n; ++i) {
            keys[i] = (uint32_t)k[i];
            if (vals)
                vals[i] = (uint32_t)v[i];
        }
    }
    free(k);
    free(v);
    return rc;
}

/* Sort u64 keys (and u64 values if vals != NULL) in place. */
int oracle_sort_u64(uint64_t *keys, uint64_t *vals, uint64_t n, int r, int passes_to_run)
{
    if (n > 0 && !keys)
        return -1;
    return lsd_sort_words(keys, vals, n, 64, r, passes_to_run);
}

/* Per-digit histograms of all d = ceil(K/r) digit positions of the *input*
 * keys: hist[p * 2^r + b] = #{i : digit_p(key_i) = b}.  keys are read as
 * 32-bit words when key_bits == 32, 64-bit words when key_bits == 64. */
int oracle_digit_histograms(const void *keys, uint64_t n, int key_bits, int r, uint64_t *hist)
{
    if (r < 1 || r > 16 || (key_bits != 32 && key_bits != 64) || (n > 0 && !keys) || !hist)
        return -1;
    int d = num_passes(key_bits, r);
    uint64_t nb = UINT64_C(1) << r;
    uint64_t *w = malloc((n ? n : 1) * sizeof(uint64_t));
    if (!w)
        return -1;
    for (uint64_t i = 0; i < n; ++i)
        w[i] = key_bits == 32 ? ((const uint32_t *)keys)[i] : ((const uint64_t *)keys)[i];
    for (int p = 0; p < d; ++p)
        count_digits(w, n, p, r, hist + (uint64_t)p * nb);
    free(w);
    return 0;
}

/* Segmented sort: segment s is [off[s], off[s+1]) and is sorted on its own;
 * offsets must be non-decreasing with off[num_segments] <= total. */
int oracle_segmented_sort(int key_bits, void *keys, void *vals, const uint64_t *off,
                          uint64_t num_segments, int r)
{
    if (key_bits != 32 && key_bits != 64)
        return -1;
    for (uint64_t s = 0; s < num_segments; ++s) {
        if (off[s + 1] < off[s])
            return -1;
        uint64_t a = off[s], len = off[s + 1] - off[s];
        int rc;
        if (key_bits == 32)
            rc = oracle_sort_u32((uint32_t *)keys + a, vals ? (uint32_t *)vals + a : NULL, len, r, -1);
        else
            rc = oracle_sort_u64((uint64_t *)keys + a, vals ? (uint64_t *)vals + a : NULL, len, r, -1);
        if (rc)
            return rc;
    }
    return 0;
}
