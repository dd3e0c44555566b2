// Batched segmented sort: many independent stable LSD radix sorts (paper,
// Section 2.6) of uneven sizes in one enqueue, classified on the device:
//   * size 0 or 1           -- nothing to sort (a single element is copied);
//   * size <= small cap     -- one workgroup sorts it in LDS (k_block_sort,
//                              small shape, several workgroups per CU);
//   * size <= medium cap    -- the same with the medium shape;
//   * larger                -- per-segment digit histograms (k_seg_hist), then
//                              one digit-pass launch per digit over the tiles
//                              of all large segments (k_seg_pass), each
//                              segment with its own look-back chain.
// Only device counters decide the work, so the sequence is graph-capturable
// and needs no host round trip.
#pragma once

#include "rs_block.h"
#include "rs_device.h"

namespace rs {

using SegLarge = SegRange;

// Segmented control block (u32 words).
constexpr int kSegSmallLen = 0;
constexpr int kSegMediumLen = 1;
constexpr int kSegLargeLen = 2;
constexpr int kSegTiles = 3;
constexpr int kSegSmallClaim = 4;
constexpr int kSegMediumClaim = 5;
constexpr int kSegHistClaim = 6;
constexpr int kSegError = 7;        // bit 0: a segment of 2^30+ elements; bit 1: tiles overflow
constexpr int kSegPassCounter = 8;  // [8, 16): group counter per pass
constexpr int kSegWords = 64;

struct SegClassifyArgs {
    const uint64_t *offsets;
    uint32_t num_segments;
    uint64_t total;
    uint32_t max_tiles;
    uint32_t *ctrl;
    SegRange *small_list;
    SegRange *medium_list;
    SegLarge *large;
    uint32_t *tile_seg;
    const void *kin;
    const void *vin;
    void *kout;
    void *vout;
    uint32_t small_cap;
    uint32_t medium_cap;
    uint32_t tile;
};

template <typename K, bool HAS_V>
__global__ __launch_bounds__(256) void k_seg_classify(SegClassifyArgs a)
{
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < a.num_segments; s += stride) {
        // clamp to [0, total): a malformed offsets array sorts garbage
        // ranges but never leaves the arrays
        const uint64_t start = std::min<uint64_t>(a.offsets[s], a.total);
        const uint64_t end = std::min<uint64_t>(std::max<uint64_t>(a.offsets[s + 1], start), a.total);
        const uint64_t size = end - start;
        if (size == 0) {
            continue;
        } else if (size == 1) {
            ((K *)a.kout)[start] = ((const K *)a.kin)[start];
            if constexpr (HAS_V)
                ((K *)a.vout)[start] = ((const K *)a.vin)[start];
        } else if (size <= a.small_cap) {
            a.small_list[atomicAdd(&a.ctrl[kSegSmallLen], 1u)] = SegRange{start, (uint32_t)size, 0};
        } else if (size <= a.medium_cap) {
            a.medium_list[atomicAdd(&a.ctrl[kSegMediumLen], 1u)] = SegRange{start, (uint32_t)size, 0};
        } else if (size >= RS_MAX_ELEMENTS) {
            atomicOr(&a.ctrl[kSegError], 1u);
        } else {
            const uint32_t idx = atomicAdd(&a.ctrl[kSegLargeLen], 1u);
            const uint32_t nt = (uint32_t)((size + a.tile - 1) / a.tile);
            const uint32_t ts = atomicAdd(&a.ctrl[kSegTiles], nt);
            // overlapping segments can need more tiles than the workspace
            // holds: such a segment keeps its tiles but sorts nothing
            const bool fits = (uint64_t)ts + nt <= a.max_tiles;
            if (!fits)
                atomicOr(&a.ctrl[kSegError], 2u);
            a.large[idx] = SegLarge{start, fits ? (uint32_t)size : 0u, ts};
            for (uint32_t i = 0; i < nt && ts + i < a.max_tiles; ++i)
                a.tile_seg[ts + i] = idx;
        }
    }
}

// Histograms of all digit positions of each large segment, then their
// exclusive scans: seg_base[seg][p][b] = elements of the segment whose digit
// p is below b.  Persistent workgroups claim segments.
struct SegHistArgs {
    const void *kin;
    const SegLarge *large;
    uint32_t *ctrl;
    uint32_t *seg_base;
};

template <typename K>
__global__ __launch_bounds__(256) void k_seg_hist(SegHistArgs a)
{
    constexpr int D = KeyTraits<K>::kBits / kRadixBits;
    constexpr int W = 256 / kWave;
    __shared__ uint32_t sh[W][D][kRadix];
    __shared__ uint32_t s_tmp[8];
    __shared__ uint32_t s_item;
    const uint32_t t = threadIdx.x;
    const uint32_t w = t / kWave;
    const K *keys = (const K *)a.kin;
    while (true) {
        if (t == 0)
            s_item = atomicAdd(&a.ctrl[kSegHistClaim], 1u);
        for (int i = t; i < W * D * kRadix; i += 256)
            (&sh[0][0][0])[i] = 0;
        __syncthreads();
        const uint32_t item = s_item;
        if (item >= a.ctrl[kSegLargeLen])
            break;
        const SegLarge rec = a.large[item];
        const K *sk = keys + rec.start;
        for (uint32_t i = t; i < rec.size; i += 256) {
            const K key = sk[i];
#pragma unroll
            for (int p = 0; p < D; ++p) {
                const uint32_t dg = KeyTraits<K>::digit(key, p * kRadixBits);
                // a digit held by the whole wave is added once (same-address
                // LDS atomics serialise)
                const uint32_t first = __builtin_amdgcn_readfirstlane(dg);
                const uint64_t active = __ballot(1);  // before any branch narrows it
                if (__ballot(dg != first) == 0) {
                    if (lane_id() == (uint32_t)__builtin_ctzll(active))
                        atomicAdd(&sh[w][p][first], (uint32_t)__popcll(active));
                } else {
                    atomicAdd(&sh[w][p][dg], 1u);
                }
            }
        }
        __syncthreads();
        uint32_t *out = a.seg_base + (uint64_t)item * D * kRadix;
        for (int p = 0; p < D; ++p) {
            uint32_t c = 0;
#pragma unroll
            for (int ww = 0; ww < W; ++ww)
                c += sh[ww][p][t];
            out[p * kRadix + t] = block_exclusive_scan_256<256>(c, s_tmp);
        }
        __syncthreads();
    }
}

}  // namespace rs
