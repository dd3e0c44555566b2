/*
 * Plain CPU oracle for the stable merge sort -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this file's library.  The product path (the HIP library) shares no
 * code, header, table or helper with it.
 *
 * What it computes (paper, Section 2.4 "Merge sort"): divide and conquer.
 * The sequence is cut into subsequences, each is sorted, and sorted
 * subsequences are merged into longer ones until one remains.  A stable merge
 * makes the whole sort stable, so the result is the unique stable ascending
 * sort by unsigned key: output position i holds the pair with the i-th
 * smallest (key, input index).
 *
 * Written as those steps, bottom up, with no blocking or fusion:
 *   1. cut the input into runs of `tile` consecutive elements (the last one
 *      may be shorter) and sort each run with a stable insertion sort (an
 *      element moves left only past strictly greater keys);
 *   2. level 1, 2, ...: merge runs 2j and 2j+1 of the current length into one
 *      run of twice the length (a run without a partner is kept as it is).
 *      The merge walks both runs from the front and takes the left run's
 *      element whenever its key is less than or equal to the right run's:
 *      equal keys keep their input order.
 *
 * Keys are handled as 64-bit words with a stated key width (32 or 64);
 * values, when present, are carried along unchanged.  Every entry point
 * returns 0 on success and -1 on a bad argument or allocation failure.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Step 1: stable insertion sort of key[lo, hi) (values follow). */
static void insertion_sort(uint64_t *key, uint64_t *val, uint64_t lo, uint64_t hi)
{
    for (uint64_t i = lo + 1; i < hi; ++i) {
        uint64_t k = key[i];
        uint64_t v = val ? val[i] : 0;
        uint64_t j = i;
        while (j > lo && key[j - 1] > k) { /* strictly greater: stability */
            key[j] = key[j - 1];
            if (val)
                val[j] = val[j - 1];
            --j;
        }
        key[j] = k;
        if (val)
            val[j] = v;
    }
}

/* Step 2: merge a[lo, mid) and a[mid, hi) into b[lo, hi). */
static void merge_runs(const uint64_t *ka, const uint64_t *va, uint64_t *kb, uint64_t *vb,
                       uint64_t lo, uint64_t mid, uint64_t hi)
{
    uint64_t i = lo, j = mid, o = lo;
    while (i < mid && j < hi) {
        if (ka[i] <= ka[j]) { /* ties go to the left run: stability */
            kb[o] = ka[i];
            if (va)
                vb[o] = va[i];
            ++i;
        } else {
            kb[o] = ka[j];
            if (va)
                vb[o] = va[j];
            ++j;
        }
        ++o;
    }
    while (i < mid) {
        kb[o] = ka[i];
        if (va)
            vb[o] = va[i];
        ++i;
        ++o;
    }
    while (j < hi) {
        kb[o] = ka[j];
        if (va)
            vb[o] = va[j];
        ++j;
        ++o;
    }
}

/* The sort on 64-bit words.  levels < 0 runs every merge level; otherwise
 * the state after that many levels is left in key/val. */
static int merge_sort_words(uint64_t *key, uint64_t *val, uint64_t n, uint64_t tile, int levels)
{
    if (tile == 0)
        return -1;
    for (uint64_t lo = 0; lo < n; lo += tile)
        insertion_sort(key, val, lo, lo + tile < n ? lo + tile : n);
    if (n <= tile)
        return 0;
    uint64_t *kt = (uint64_t *)malloc(n * sizeof(uint64_t));
    uint64_t *vt = val ? (uint64_t *)malloc(n * sizeof(uint64_t)) : NULL;
    if (!kt || (val && !vt)) {
        free(kt);
        free(vt);
        return -1;
    }
    uint64_t *ka = key, *va = val, *kb = kt, *vb = vt;
    int level = 0;
    for (uint64_t width = tile; width < n && (levels < 0 || level < levels); width *= 2) {
        for (uint64_t lo = 0; lo < n; lo += 2 * width) {
            uint64_t mid = lo + width < n ? lo + width : n;
            uint64_t hi = lo + 2 * width < n ? lo + 2 * width : n;
            merge_runs(ka, va, kb, vb, lo, mid, hi);
        }
        uint64_t *t = ka;
        ka = kb;
        kb = t;
        t = va;
        va = vb;
        vb = t;
        ++level;
    }
    if (ka != key) {
        memcpy(key, ka, n * sizeof(uint64_t));
        if (val)
            memcpy(val, va, n * sizeof(uint64_t));
    }
    free(kt);
    free(vt);
    return 0;
}

/* keys/vals: key_bits/8-byte unsigned words (vals may be NULL), sorted in
 * place.  tile >= 1 is the run length of step 1; levels < 0 runs all merge
 * levels. */
int oracle_merge_sort(int key_bits, void *keys, void *vals, uint64_t n, uint64_t tile, int levels)
{
    if ((key_bits != 32 && key_bits != 64) || (n && !keys) || tile == 0)
        return -1;
    if (n == 0)
        return 0;
    uint64_t *k = (uint64_t *)malloc(n * sizeof(uint64_t));
    uint64_t *v = vals ? (uint64_t *)malloc(n * sizeof(uint64_t)) : NULL;
    if (!k || (vals && !v)) {
        free(k);
        free(v);
        return -1;
    }
    for (uint64_t i = 0; i < n; ++i) {
        k[i] = key_bits == 32 ? ((uint32_t *)keys)[i] : ((uint64_t *)keys)[i];
        if (vals)
            v[i] = key_bits == 32 ? ((uint32_t *)vals)[i] : ((uint64_t *)vals)[i];
    }
    int rc = merge_sort_words(k, v, n, tile, levels);
    if (rc == 0) {
        for (uint64_t i = 0; i < n; ++i) {
            if (key_bits == 32) {
                ((uint32_t *)keys)[i] = (uint32_t)k[i];
                if (vals)
                    ((uint32_t *)vals)[i] = (uint32_t)v[i];
            } else {
                ((uint64_t *)keys)[i] = k[i];
                if (vals)
                    ((uint64_t *)vals)[i] = v[i];
            }
        }
    }
    free(k);
    free(v);
    return rc;
}
