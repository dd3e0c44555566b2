// LDS-resident radix sort of up to CAP = THREADS x ITEMS elements by one
// workgroup: the same stable counting sort per 8-bit digit as the digit-pass
// kernel (paper, Section 2.6), with every pass between registers and LDS and
// only one read and one write of HBM.  Used for a whole sort when n <= CAP
// (one launch) and for the small and medium segments of a segmented sort.
#pragma once

#include "rs_device.h"

namespace rs {

// Block-sort shapes: kSmall for up to 4096 elements (several workgroups per
// CU), kMedium for up to 16384 (8192 for 64-bit pairs, whose staging would
// not fit otherwise).
template <typename K, bool HAS_V>
struct BlockShape {
    static constexpr int kSmallThreads = 256;
    static constexpr int kMediumThreads = (sizeof(K) == 8 && HAS_V) ? 512 : 1024;
    static constexpr int kItems = 16;
    static constexpr int kSmallCap = kSmallThreads * kItems;
    static constexpr int kMediumCap = kMediumThreads * kItems;
};

// A run of elements to sort on its own.
struct SegRange {
    uint64_t start;       // first element
    uint32_t size;        // elements
    uint32_t tile_start;  // first tile in a batched tile sequence (large segments)
};

struct BlockArgs {
    const void *kin;
    const void *vin;
    void *kout;
    void *vout;
    // segmented use: the workgroups claim entries of list (list_len of them,
    // a device count) through *claim.  Single sort: list == nullptr, one
    // range [0, n).
    const SegRange *list;
    const uint32_t *list_len;
    uint32_t *claim;
    uint64_t n;
    uint32_t kmap;  // key order (kMap*): applied on load, undone on store
    // single sort with a caller's workspace: its error word, cleared here so
    // that a status query after this sort does not report an older one
    uint32_t *err_clear;
};

template <typename K, typename V, bool HAS_V, int THREADS, int ITEMS>
__global__ __launch_bounds__(THREADS) void k_block_sort(BlockArgs a)
{
    constexpr int CAP = THREADS * ITEMS;
    constexpr int W = THREADS / kWave;
    constexpr int D = num_passes<K, kRadixBits>();
    constexpr size_t kStageBytes = (size_t)CAP * (sizeof(K) + (HAS_V ? sizeof(V) : 0));
    static_assert((size_t)W * kRadix * 8 <= kStageBytes, "mask table lives in the staging buffer");

    __shared__ uint32_t s_wcnt[W * kRadix];
    __shared__ uint32_t s_tmp[8];
    __shared__ uint32_t s_item;
    __shared__ __attribute__((aligned(16))) unsigned char s_stage[kStageBytes];
    K *s_k = (K *)s_stage;
    V *s_v = (V *)(s_stage + (size_t)CAP * sizeof(K));
    uint64_t *s_mask = (uint64_t *)s_stage;

    const uint32_t t = threadIdx.x;
    const uint32_t w = t / kWave;
    const uint32_t lane = t % kWave;
    const uint32_t off0 = w * (kWave * ITEMS) + lane;
    uint32_t *wc = s_wcnt + w * kRadix;
    const K *kin = (const K *)a.kin;
    const V *vin = (const V *)a.vin;
    K *kout = (K *)a.kout;
    V *vout = (V *)a.vout;
    if (a.err_clear && blockIdx.x == 0 && t == 0)
        *a.err_clear = 0;

    for (uint32_t iter = 0;; ++iter) {
        if (t == 0)
            s_item = a.list ? atomicAdd(a.claim, 1u) : iter;
        __syncthreads();
        const uint32_t item = s_item;
        uint64_t start;
        uint32_t m;
        if (a.list) {
            if (item >= *a.list_len)
                break;
            start = a.list[item].start;
            m = a.list[item].size;
        } else {
            if (item != 0)
                break;
            start = 0;
            m = (uint32_t)a.n;
        }

        // load: position j*64 + l of the wave's run; padding keys (all ones)
        // stay behind every real key in every pass
        K key[ITEMS];
        V val[HAS_V ? ITEMS : 1];
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t pos = off0 + j * kWave;
            key[j] = pos < m ? kin[start + pos] : KeyTraits<K>::kPad;
            if constexpr (HAS_V)
                val[j] = pos < m ? vin[start + pos] : (V)0;
        }
        // mapped once every load is issued (a map between loads would wait
        // for each in turn); padding keys stay unmapped
        if (a.kmap) {
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) {
                const K mk = map_in(key[j], a.kmap);
                key[j] = off0 + j * kWave < m ? mk : key[j];
            }
        }

        for (int p = 0; p < D; ++p) {
            const int shift = p * kRadixBits;
            for (int i = t; i < W * kRadix; i += THREADS) {
                s_wcnt[i] = 0;
                s_mask[i] = 0;
            }
            __syncthreads();
            uint32_t rank[ITEMS];
            wave_rank<kRadixBits, K, ITEMS>(key, shift, wc, s_mask + w * kRadix, lane, rank);
            __syncthreads();
            // exclusive offsets over (digit, wave): digit-major, so that
            // earlier waves (earlier elements) come first within a digit
            uint32_t cnt = 0;
            if (t < kRadix) {
#pragma unroll
                for (int ww = 0; ww < W; ++ww) {
                    const uint32_t c = s_wcnt[ww * kRadix + t];
                    s_wcnt[ww * kRadix + t] = cnt;
                    cnt += c;
                }
            }
            const uint32_t excl = bins_exclusive_scan<kRadix>(cnt, s_tmp);
            if (t < kRadix) {
#pragma unroll
                for (int ww = 0; ww < W; ++ww)
                    s_wcnt[ww * kRadix + t] += excl;
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) {
                const uint32_t pos = rank[j] + wc[digit_of<kRadixBits>(key[j], shift)];
                s_k[pos] = key[j];
                if constexpr (HAS_V)
                    s_v[pos] = val[j];
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) {
                key[j] = s_k[off0 + j * kWave];
                if constexpr (HAS_V)
                    val[j] = s_v[off0 + j * kWave];
            }
            __syncthreads();
        }

#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t pos = off0 + j * kWave;
            if (pos < m) {
                kout[start + pos] = map_out(key[j], a.kmap);
                if constexpr (HAS_V)
                    vout[start + pos] = val[j];
            }
        }
    }
}

}  // namespace rs
