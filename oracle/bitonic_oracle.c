/*
 * Plain CPU oracle for the bitonic sorting network -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this file's library.  The product path (the HIP library) shares no
 * code, header, table or helper with it.
 *
 * What it computes (paper, Section 2.1 "Bitonic sort", Batcher's network):
 * a sorting network on N = 2^m slots whose compare-exchange sequence is fixed
 * in advance.  Stage k = 2, 4, ..., N builds sorted runs of length k; within
 * a stage, steps of distance j = k/2, k/4, ..., 1 compare slot i with slot
 * i XOR j (for the lower slot i of each pair) and order the pair ascending
 * when bit k of i is clear, descending when it is set.
 *
 * A network is not stable by itself.  Here every element is the pair
 * (key, input index), compared lexicographically, so all elements differ and
 * the sorted order is the stable sort by key.  Slots past n hold a padding
 * element that compares greater than every real one.
 *
 * oracle_bitonic_network sorts N plain 64-bit words with the network alone
 * (no index), for the 0-1 principle check of the network itself.
 * Every entry point returns 0 on success and -1 on a bad argument or
 * allocation failure.
 */
#include <stdint.h>
#include <stdlib.h>

typedef struct {
    uint64_t key;
    uint64_t idx; /* input index; UINT64_MAX marks padding */
} elem;

static int greater(elem a, elem b)
{
    if (a.key != b.key)
        return a.key > b.key;
    return a.idx > b.idx;
}

/* The network on N slots of any element type, through a comparison. */
static void network_elems(elem *a, uint64_t N)
{
    for (uint64_t k = 2; k <= N; k *= 2) {
        for (uint64_t j = k / 2; j >= 1; j /= 2) {
            for (uint64_t i = 0; i < N; ++i) {
                uint64_t l = i ^ j;
                if (l <= i)
                    continue; /* each pair once, from its lower slot */
                int ascending = (i & k) == 0;
                if (ascending ? greater(a[i], a[l]) : greater(a[l], a[i])) {
                    elem t = a[i];
                    a[i] = a[l];
                    a[l] = t;
                }
            }
        }
    }
}

int oracle_bitonic_network(uint64_t *words, uint64_t N)
{
    if (N == 0 || (N & (N - 1)) || !words)
        return -1;
    elem *a = (elem *)malloc(N * sizeof(elem));
    if (!a)
        return -1;
    for (uint64_t i = 0; i < N; ++i) {
        a[i].key = words[i];
        a[i].idx = 0; /* no tie-break: the bare network */
    }
    network_elems(a, N);
    for (uint64_t i = 0; i < N; ++i)
        words[i] = a[i].key;
    free(a);
    return 0;
}

/* keys/vals: key_bits/8-byte unsigned words (vals may be NULL), n of them,
 * sorted in place by the network on (key, index) over the next power of two. */
int oracle_bitonic_sort(int key_bits, void *keys, void *vals, uint64_t n)
{
    if ((key_bits != 32 && key_bits != 64) || (n && !keys))
        return -1;
    if (n == 0)
        return 0;
    uint64_t N = 1;
    while (N < n)
        N *= 2;
    elem *a = (elem *)malloc(N * sizeof(elem));
    uint64_t *v = vals ? (uint64_t *)malloc(n * sizeof(uint64_t)) : NULL;
    if (!a || (vals && !v)) {
        free(a);
        free(v);
        return -1;
    }
    for (uint64_t i = 0; i < N; ++i) {
        if (i < n) {
            a[i].key = key_bits == 32 ? ((uint32_t *)keys)[i] : ((uint64_t *)keys)[i];
            a[i].idx = i;
        } else {
            a[i].key = UINT64_MAX;
            a[i].idx = UINT64_MAX;
        }
    }
    if (vals)
        for (uint64_t i = 0; i < n; ++i)
            v[i] = key_bits == 32 ? ((uint32_t *)vals)[i] : ((uint64_t *)vals)[i];
    network_elems(a, N);
    for (uint64_t i = 0; i < n; ++i) {
        if (key_bits == 32) {
            ((uint32_t *)keys)[i] = (uint32_t)a[i].key;
            if (vals)
                ((uint32_t *)vals)[i] = (uint32_t)v[a[i].idx];
        } else {
            ((uint64_t *)keys)[i] = a[i].key;
            if (vals)
                ((uint64_t *)vals)[i] = v[a[i].idx];
        }
    }
    free(a);
    free(v);
    return 0;
}
