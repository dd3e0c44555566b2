// One digit pass with wide digits (R = 9..11 bits, 512..2048 bins): the same
// stable counting sort per tile as pass_tile in rs_kernels.h (paper,
// Section 2.6), laid out so that 2^R bins fit a gfx950 workgroup's 160 KB
// of LDS beside a full tile of staged pairs.
//
// Wider digits mean fewer passes over the data (three for 32-bit keys at
// 11 bits instead of four at 8), at the price of more bins per tile:
//   * the per-wave digit counters are 16-bit (a wave counts at most
//     64 x ITEMS <= 2048 of a digit; tile positions stay below 2^16) and,
//     with the per-wave lane-mask tables, live inside the staging buffer:
//     they are dead before the first element is staged;
//   * a wave finds the lanes sharing its digit from a lane-mask table
//     indexed by the digit's low 8 bits, refined by one ballot per higher
//     bit (or, for skewed digits and a share of the waves, by R ballots);
//   * the counters are turned into tile positions before staging (one more
//     barrier than pass_tile);
//   * every thread looks back over the two digits it scanned, then stages
//     its elements (with 2^R digits a look-back needs every thread).
#pragma once

#include "rs_device.h"

namespace rs {

// Lane-mask table slots per wave: indexed by the low 8 bits of the digit.
constexpr int kWideSlots = 256;
constexpr int kWideSlotBits = 8;

// Exclusive scan of one value per thread over a workgroup of THREADS
// threads (a multiple of 64, at most 1024).  `tmp` holds THREADS / 64 words.
// Every thread must call it (two barriers inside).  *total receives the sum.
template <int THREADS>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *tmp,
                                                         uint32_t *total)
{
    constexpr int W = THREADS / kWave;
    const uint32_t t = threadIdx.x;
    const uint32_t w = t / kWave;
    const uint32_t inc = wave_inclusive_scan(v);
    if ((t & (kWave - 1)) == kWave - 1)
        tmp[w] = inc;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < W; ++i) {
        const uint32_t x = tmp[i];
        before += (uint32_t)i < w ? x : 0u;
        all += x;
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

// LDS of a wide digit pass.  The staging buffer holds, while ranking, the
// per-wave 16-bit counters [W][2^R] followed by the per-wave lane-mask
// tables [W][256]; then the tile's elements in rank order (pairs as one
// (key, value) word per element).
template <typename K, typename C, bool HAS_V>
struct WideLds {
    static constexpr int W = C::kThreads / kWave;
    static constexpr int NB = C::kBins;
    static constexpr size_t kStageBytes = (size_t)C::kTile * sizeof(K) * (HAS_V ? 2 : 1);
    static constexpr size_t kCountBytes = (size_t)W * NB * sizeof(uint16_t);
    static constexpr size_t kMaskBytes = (size_t)W * kWideSlots * sizeof(uint64_t);
    static constexpr size_t kAreaBytes =
        kStageBytes > kCountBytes + kMaskBytes ? kStageBytes : kCountBytes + kMaskBytes;
    uint32_t gbase[NB];  // digit's start in the output minus its start in the tile
    uint32_t tmp[16];
    uint32_t tile;
    __attribute__((aligned(16))) unsigned char area[kAreaBytes];
};

// Stable ranks of a wave's items among the wave's items of the same digit.
// Items are visited j = 0..ITEMS-1, lanes in order (the input order of the
// wave's elements).  wc: the wave's 2^R 16-bit counters (zeroed by the
// caller); wm: its 256-slot lane-mask table (zeroed, left zeroed), or null
// for the all-ballot form.
template <int R, typename K, int ITEMS>
__device__ __forceinline__ void wave_rank_wide(const K (&key)[ITEMS], int shift, uint16_t *wc,
                                               uint64_t *wm, uint32_t lane,
                                               uint32_t (&rank)[ITEMS])
{
    const uint64_t lane_bit = 1ull << lane;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const uint32_t d = digit_of<R>(key[j], shift);
        uint64_t m;
        if (wm) {
            // lanes with the same low 8 bits, then one ballot per higher bit:
            // the lanes whose bit differs from ours are dropped
            const uint32_t lo = d & (kWideSlots - 1);
            atomicOr(&wm[lo], lane_bit);
            const uint64_t slot = wm[lo];
            uint32_t diff_lo = ~(uint32_t)slot, diff_hi = ~(uint32_t)(slot >> 32);
#pragma unroll
            for (int b = kWideSlotBits; b < R; ++b) {
                const uint32_t s = (uint32_t)__builtin_amdgcn_sbfe((int32_t)d, b, 1);
                const uint64_t bal = __ballot(s != 0);
                diff_lo = __builtin_amdgcn_bitop3_b32(diff_lo, (uint32_t)bal, s, 0xF6);
                diff_hi = __builtin_amdgcn_bitop3_b32(diff_hi, (uint32_t)(bal >> 32), s, 0xF6);
            }
            m = ~(((uint64_t)diff_hi << 32) | diff_lo);
            // the slot's lowest lane clears it (every lane has read it: LDS
            // operations of one wave complete in order)
            if (lanes_below(slot) == 0)
                wm[lo] = 0;
        } else {
            m = peer_mask<R>(d);
        }
        const uint32_t below = lanes_below(m);
        const uint32_t c = wc[d];
        rank[j] = c + below;
        if (below == 0)
            wc[d] = (uint16_t)(c + (uint32_t)__popcll(m));
    }
}

// One tile of a wide digit pass; arguments as pass_tile.  db[] holds this
// thread's digits' starting offsets in the digit-sorted sequence (digits
// DPS*t .. DPS*t + DPS - 1, DPS = 2^R / THREADS, for t < 2^R / DPS).
template <typename K, typename V, bool HAS_V, typename C, typename Hook>
__device__ __forceinline__ void pass_tile_wide(WideLds<K, C, HAS_V> &L, const K *tk, const V *tv,
                                               K *dk, V *dv, uint32_t valid, uint32_t limit,
                                               uint32_t tile, uint32_t first_tile,
                                               uint32_t *status, const uint32_t (&db)[2],
                                               int shift, bool ballot_rank, uint32_t map_load,
                                               uint32_t map_store, const PassArgs &wait,
                                               Hook &&after_lookback)
{
    constexpr int R = C::kRadixBits;
    constexpr uint32_t NB = C::kBins;
    constexpr int THREADS = C::kThreads;
    constexpr int ITEMS = C::kItems;
    constexpr int T = C::kTile;
    constexpr int W = THREADS / kWave;
    constexpr int LBW = C::kLookback;
    // digits per thread (the counters are read two 16-bit words at once)
    constexpr int DPS = NB / THREADS;
    static_assert(DPS == 2, "the wide pass scans two digits per thread");
    static_assert(T <= 65536, "tile positions are 16-bit");
    static_assert(sizeof(V) == sizeof(K), "values have the key's width");
    using Lds = WideLds<K, C, HAS_V>;
    uint16_t *s_cnt = (uint16_t *)L.area;
    uint32_t *s_cnt2 = (uint32_t *)L.area;  // the counters as two 16-bit digits per word
    uint64_t *s_mask = (uint64_t *)(L.area + Lds::kCountBytes);
    KvPair<K> *s_kv = (KvPair<K> *)L.area;
    K *s_k = (K *)L.area;
    const uint32_t t = threadIdx.x;
    const uint32_t w = t / kWave;
    const uint32_t lane = t % kWave;
    const uint32_t off0 = w * (kWave * ITEMS) + lane;
    uint16_t *wc = s_cnt + w * NB;
    uint64_t *wm = s_mask + w * kWideSlots;

    // this wave's counters and table are its own (after the previous tile's
    // closing barrier): it clears them itself
    {
        uint4 *c4 = (uint4 *)wc;
        for (uint32_t i = lane; i < NB * 2 / 16; i += kWave)
            c4[i] = make_uint4(0, 0, 0, 0);
        uint4 *m4 = (uint4 *)wm;
        for (uint32_t i = lane; i < kWideSlots * 8 / 16; i += kWave)
            m4[i] = make_uint4(0, 0, 0, 0);
    }
    K key[ITEMS];
    V val[HAS_V ? ITEMS : 1];
    load_tile<K, V, HAS_V, ITEMS>(tk, tv, valid, off0, key, val, valid == (uint32_t)T, map_load);

    uint32_t rank[ITEMS];
    const bool ballots = ballot_rank || w < (uint32_t)C::kBallotWaves;
    wave_rank_wide<R, K, ITEMS>(key, shift, wc, ballots ? nullptr : wm, lane, rank);
    __syncthreads();

    // scan: thread t takes digits 2t, 2t+1 -- per-wave exclusive offsets,
    // the tile's counts (published as aggregates), the digits' starts in
    // the tile (a workgroup scan), then the per-wave offsets become tile
    // positions.  Offsets stay below the tile size, so two 16-bit fields
    // add as one 32-bit word without carries.
    uint32_t run0 = 0, run1 = 0;
#pragma unroll
    for (int ww = 0; ww < W; ++ww) {
        const uint32_t v = s_cnt2[ww * (NB / 2) + t];
        s_cnt2[ww * (NB / 2) + t] = run0 | (run1 << 16);
        run0 += v & 0xFFFFu;
        run1 += v >> 16;
    }
    {
        const uint32_t f = tile == first_tile ? kFlagInc : kFlagAgg;
        uint32_t *st = status + (uint64_t)tile * NB + 2 * t;
        __hip_atomic_store(st, f | run0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(st + 1, f | run1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    uint32_t tile_total;
    const uint32_t start0 = block_exclusive_scan<THREADS>(run0 + run1, L.tmp, &tile_total);
    const uint32_t start1 = start0 + run0;
    {
        const uint32_t add = start0 | (start1 << 16);
#pragma unroll
        for (int ww = 0; ww < W; ++ww)
            s_cnt2[ww * (NB / 2) + t] += add;
    }
    __syncthreads();
    // position of every item in the tile
#pragma unroll
    for (int j = 0; j < ITEMS; ++j)
        rank[j] += wc[digit_of<R>(key[j], shift)];
    __syncthreads();  // the counters are dead: the staging may overwrite them

    // decoupled look-back of this thread's two digits, each on its own:
    // LBW predecessors per round trip, counts added in order up to the
    // first inclusive word; bounded like pass_tile's.  Then the inclusive
    // words, the digits' bases, and the staging of this thread's elements.
    {
        const int32_t lo = (int32_t)first_tile;
        const uint32_t cnt[2] = {run0, run1};
        uint32_t prefix[2] = {0, 0};
        int32_t k[2] = {(int32_t)tile - 1, (int32_t)tile - 1};
        bool done[2] = {tile == first_tile, tile == first_tile};
        uint32_t spins = 0;
        while (!(done[0] && done[1])) {
            uint32_t st[2][LBW];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int l = 0; l < LBW; ++l)
                    st[i][l] = (!done[i] && k[i] - l >= lo)
                                   ? __hip_atomic_load(
                                         &status[(uint64_t)(k[i] - l) * NB + 2 * t + i],
                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                   : kFlagInc;
            bool progress = false, short_read = false;
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                if (done[i])
                    continue;
                int used = 0;
                bool fin = false;
                if (!(wait.stall & kStallLookback)) {
#pragma unroll
                    for (int l = 0; l < LBW; ++l) {
                        if (!fin && used == l) {
                            const uint32_t f = st[i][l] & kFlagMask;
                            if (f != 0) {
                                prefix[i] += st[i][l] & kCountMask;
                                fin = f == kFlagInc;
                                used = l + 1;
                            }
                        }
                    }
                }
                k[i] -= used;
                done[i] = fin;
                progress = progress || used > 0;
                short_read = short_read || (!fin && used < LBW);
            }
            if (done[0] && done[1])
                break;
            if (!progress && ++spins > wait.spin_limit) {
                atomicOr(wait.err, kErrWait);
                break;
            }
            if (short_read)
                __builtin_amdgcn_s_sleep(1);
        }
        if (tile != first_tile) {
            uint32_t *st = status + (uint64_t)tile * NB + 2 * t;
            __hip_atomic_store(st, kFlagInc | (prefix[0] + cnt[0]), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(st + 1, kFlagInc | (prefix[1] + cnt[1]), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        L.gbase[2 * t] = db[0] + prefix[0] - start0;
        L.gbase[2 * t + 1] = db[1] + prefix[1] - start1;
    }
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        if constexpr (HAS_V)
            s_kv[rank[j]] = KvPair<K>{key[j], (K)val[j]};
        else
            s_k[rank[j]] = key[j];
    }
    __syncthreads();
    after_lookback(t);

    // place: each digit run of the staged tile goes out with consecutive
    // lanes on consecutive addresses.  The thread index is made opaque here
    // so that the compiler recomputes the staging addresses per tile instead
    // of keeping 16 of them live across the tile loop (spilled otherwise).
    uint32_t tp = t;
    asm volatile("" : "+v"(tp));
    uint32_t dst[ITEMS];
    V vk[HAS_V ? ITEMS : 1];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t pos = i * THREADS + tp;
        K kk;
        if constexpr (HAS_V) {
            const KvPair<K> kv = s_kv[pos];
            kk = kv.k;
            vk[i] = (V)kv.v;
        } else {
            kk = s_k[pos];
        }
        dst[i] = L.gbase[digit_of<R>(kk, shift)] + pos;
        if (dst[i] < limit)
            store_at(dk, dst[i], map_out(kk, map_store));
    }
    if constexpr (HAS_V) {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i)
            if (dst[i] < limit)
                store_at(dv, dst[i], vk[i]);
    }
    (void)tile_total;
    __syncthreads();  // LDS is reused by the next tile
}

}  // namespace rs
