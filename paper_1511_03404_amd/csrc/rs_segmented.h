// Batched segmented sort: many independent stable LSD radix sorts (paper,
// Section 2.6) of uneven sizes in one enqueue, classified on the device:
//   * size 0 or 1           -- nothing to sort (a single element is copied);
//   * size <= tiny cap      -- one wave sorts it in registers with a bitonic
//                              network on (key, position) pairs (Section 2.1,
//                              k_seg_bitonic in rs_bitonic.h; the cap is a
//                              context setting, 0 turns the class off);
//   * size <= small cap     -- one workgroup sorts it in LDS (k_block_sort,
//                              small shape, several workgroups per CU);
//   * size <= medium cap    -- the same with the medium shape;
//   * larger                -- per-segment digit histograms (k_seg_hist), then
//                              one digit-pass launch per digit over the tiles
//                              of all large segments (k_seg_pass, in
//                              rs_kernels.h), each segment with its own
//                              look-back chain.
// Only device counters decide the work, so the sequence is graph-capturable
// and needs no host round trip.
#pragma once

#include "rs.h"
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
constexpr int kSegError = kCtrlError;  // kErrSegTooLarge, kErrSegTiles, kErrWait
constexpr int kSegTinyLen = 8;
constexpr int kSegTinyClaim = 9;
constexpr int kSegPassCounter = 32; // [32, 48): group counter per pass
constexpr int kSegChunks = 16;      // histogram chunks of the large segments
constexpr int kSegChunkClaim = 17;
constexpr int kSegScanClaim = 18;
constexpr int kSegWords = 64;
// Large segments are histogrammed in chunks of this many elements, so that
// one huge segment does not leave a single workgroup reading it alone.
constexpr uint32_t kSegChunk = 1u << 18;

struct SegClassifyArgs {
    const uint64_t *offsets;
    uint32_t num_segments;
    uint64_t total;
    uint32_t max_tiles;
    uint32_t *ctrl;
    SegRange *tiny_list;
    SegRange *small_list;
    SegRange *medium_list;
    SegLarge *large;
    uint32_t *tile_seg;
    uint32_t *chunk_seg;  // large segment of each histogram chunk
    uint32_t max_chunks;
    const void *kin;
    const void *vin;
    void *kout;
    void *vout;
    uint32_t tiny_cap;  // 0: no tiny class
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
        } else if (size <= a.tiny_cap) {
            a.tiny_list[atomicAdd(&a.ctrl[kSegTinyLen], 1u)] = SegRange{start, (uint32_t)size, 0};
        } else if (size <= a.small_cap) {
            a.small_list[atomicAdd(&a.ctrl[kSegSmallLen], 1u)] = SegRange{start, (uint32_t)size, 0};
        } else if (size <= a.medium_cap) {
            a.medium_list[atomicAdd(&a.ctrl[kSegMediumLen], 1u)] = SegRange{start, (uint32_t)size, 0};
        } else if (size >= RS_MAX_ELEMENTS) {
            atomicOr(&a.ctrl[kSegError], kErrSegTooLarge);
        } else {
            const uint32_t idx = atomicAdd(&a.ctrl[kSegLargeLen], 1u);
            const uint32_t nt = (uint32_t)((size + a.tile - 1) / a.tile);
            const uint32_t ts = atomicAdd(&a.ctrl[kSegTiles], nt);
            // overlapping segments can need more tiles than the workspace
            // holds: such a segment keeps its tiles but sorts nothing
            const bool fits = (uint64_t)ts + nt <= a.max_tiles;
            if (!fits)
                atomicOr(&a.ctrl[kSegError], kErrSegTiles);
            a.large[idx] = SegLarge{start, fits ? (uint32_t)size : 0u, ts};
            for (uint32_t i = 0; i < nt && ts + i < a.max_tiles; ++i)
                a.tile_seg[ts + i] = idx;
            const uint32_t nc = (uint32_t)((size + kSegChunk - 1) / kSegChunk);
            const uint32_t cs = atomicAdd(&a.ctrl[kSegChunks], nc);
            for (uint32_t i = 0; i < nc && cs + i < a.max_chunks; ++i)
                a.chunk_seg[cs + i] = idx;
        }
    }
}

}  // namespace rs
