// Device building blocks of the gfx950 LSD radix sort.
//
// One digit pass is the stable counting sort of the paper's radix sort
// (Section 2.6): count the digits, exclusive-scan the counts, place every
// element at its digit's running offset in input order.  On the GPU the
// three steps are spread over a tile of T elements per workgroup:
//   * count  -- a wave64 "multisplit": each lane learns the mask of lanes
//               holding the same digit (most waves from a per-wave LDS
//               table of lane masks, the others, and every wave when the
//               digits are skewed, from one ballot per digit bit, so the
//               LDS and the VALU share the work); the lowest such lane adds
//               the group size to a
//               per-wave LDS counter, and the rank inside the group is mbcnt
//               over the mask.  Items are visited in input order
//               (wave-striped: item j of lane l is element j*64 + l of the
//               wave's run), which is what makes the ranking stable;
//   * scan   -- digit_base (global exclusive scan of the digit histogram) +
//               a decoupled look-back over the tiles before this one +
//               the tile-local exclusive scan over digits and waves;
//   * place  -- stage the tile in LDS in rank order, then write each digit
//               run out with consecutive lanes on consecutive addresses.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

namespace rs {

// Digit widths R of 4..8 bits are compiled; a pass has 2^R bins.  kRadix is
// the largest bin count (sizes of LDS tables shared by all widths, the
// 256-thread scans) and kRadixBits the default width.
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kWave = 64;
constexpr int kMaxPasses = 16;  // 64-bit keys at 4-bit digits

// Look-back status word: [31:30] flag, [29:0] digit count.
constexpr uint32_t kFlagAgg = 1u << 30;  // count of this tile only
constexpr uint32_t kFlagInc = 2u << 30;  // count of all tiles up to and including this one
constexpr uint32_t kFlagMask = 3u << 30;
constexpr uint32_t kCountMask = (1u << 30) - 1;

// Control block (u32 words at the start of the workspace).
constexpr int kCtrlTileCounter = 0;  // [0, 16): dynamic tile id per pass
constexpr int kCtrlPlan = 16;        // [16, 32): plan word per pass
constexpr int kCtrlFinal = 48;       // final copy: 0 none, 1 tmp -> out
constexpr int kCtrlWords = 64;

// Error word: the same index in the control block of the plain and of the
// segmented sort, read back by the host after the stream completes.
constexpr int kCtrlError = 56;
constexpr uint32_t kErrSegTooLarge = 1u;  // a segment of 2^30 or more elements was skipped
constexpr uint32_t kErrSegTiles = 2u;     // segments needed more tiles than the workspace holds
constexpr uint32_t kErrWait = 4u;         // a wait on another workgroup gave up (bound reached)

// Waits on other workgroups (tile claims, look-back) poll at most this many
// times without progress, then record kErrWait and go on, so that a lost
// tile ends the kernel with an error instead of a hang.  A poll is one
// device-scope load plus a short sleep (about 1 us under load), so the
// default bound is several seconds: far beyond any wait of a working sort.
constexpr uint32_t kDefaultSpinLimit = 1u << 22;

// Test-only stalls (never set by a working caller): the look-back or the
// tile claim treats every predecessor as not yet published, so each wait
// runs into its bound.
constexpr uint32_t kStallLookback = 1u;
constexpr uint32_t kStallClaim = 2u;

// Plan word of one pass.
constexpr uint32_t kPlanRun = 1u;          // the pass moves data
constexpr uint32_t kPlanCopyIn = 2u;       // no pass runs: copy the keys in -> out here
constexpr int kPlanSrcShift = 2;           // buffer id, 2 bits
constexpr int kPlanDstShift = 4;           // buffer id, 2 bits
constexpr uint32_t kBufIn = 0, kBufOut = 1, kBufTmp = 2;
constexpr uint32_t kPlanBallot = 64u;      // skewed digit: rank with ballots, not the LDS table
constexpr uint32_t kPlanFirst = 128u;      // the first moving pass (reads the input)
constexpr uint32_t kPlanLast = 256u;       // the last moving pass, writing the output
constexpr uint32_t kPlanCopyInV = 512u;    // no pass runs: copy the values in -> out here

template <typename K>
struct KeyTraits;

template <>
struct KeyTraits<uint32_t> {
    static constexpr int kBits = 32;
    static constexpr uint32_t kPad = 0xFFFFFFFFu;
};

template <>
struct KeyTraits<uint64_t> {
    static constexpr int kBits = 64;
    static constexpr uint64_t kPad = ~0ull;
};

// Key orders.  The sort orders unsigned keys; other orders are exact
// bijections of the key bits applied where keys are read from the input and
// undone where they are written to the output:
//   kMapSigned   two's-complement integers: flip the sign bit;
//   kMapFloat    IEEE floats, total order of the bit patterns (-NaN < -inf <
//                ... < -0 < +0 < ... < +inf < +NaN): flip every bit of a
//                negative key, only the sign bit of a positive one;
//   kMapDescending  after the above, complement the key (equal keys keep
//                their input order, so the descending sort is stable too).
constexpr uint32_t kMapSigned = 1u;
constexpr uint32_t kMapFloat = 2u;
constexpr uint32_t kMapDescending = 4u;

// Both maps are branch-free: each is one XOR with a mask built from uniform
// flags and the key's own sign bit, so a tile's loads stay in flight
// together and the unsigned ascending order costs a few ALU operations.
template <typename K>
__device__ __forceinline__ K map_in(K k, uint32_t kmap)
{
    using S = std::make_signed_t<K>;
    constexpr K sign = (K)1 << (KeyTraits<K>::kBits - 1);
    const K x = (kmap & (kMapSigned | kMapFloat)) ? sign : (K)0;
    const K f = (kmap & kMapFloat) ? ~(K)0 : (K)0;
    const K d = (kmap & kMapDescending) ? ~(K)0 : (K)0;
    const K neg = (K)((S)k >> (KeyTraits<K>::kBits - 1));  // all ones if the top bit is set
    return k ^ ((x | (f & neg)) ^ d);
}

template <typename K>
__device__ __forceinline__ K map_out(K k, uint32_t kmap)
{
    using S = std::make_signed_t<K>;
    constexpr K sign = (K)1 << (KeyTraits<K>::kBits - 1);
    const K x = (kmap & (kMapSigned | kMapFloat)) ? sign : (K)0;
    const K f = (kmap & kMapFloat) ? ~(K)0 : (K)0;
    const K d = (kmap & kMapDescending) ? ~(K)0 : (K)0;
    k ^= d;
    // a mapped float with the top bit clear came from a negative key
    const K pos = (K)((S)k >> (KeyTraits<K>::kBits - 1));
    return k ^ (x | (f & ~pos));
}

// Number of R-bit digit positions of a K key (the last one may be narrower).
template <typename K, int R>
constexpr int num_passes()
{
    return (KeyTraits<K>::kBits + R - 1) / R;
}

// The R-bit digit of k that starts at bit `shift` (bits above the key's top
// read as zero, so the last, narrower digit is exact too).
template <int R>
__device__ __forceinline__ uint32_t digit_of(uint32_t k, int shift)
{
    if constexpr (32 % R == 0)
        return __builtin_amdgcn_ubfe(k, (uint32_t)shift, (uint32_t)R);
    else
        return (k >> shift) & ((1u << R) - 1u);
}

template <int R>
__device__ __forceinline__ uint32_t digit_of(uint64_t k, int shift)
{
    if constexpr (32 % R == 0) {
        // the digit lies within one 32-bit half
        const uint32_t w = shift < 32 ? (uint32_t)k : (uint32_t)(k >> 32);
        return __builtin_amdgcn_ubfe(w, (uint32_t)(shift & 31), (uint32_t)R);
    } else {
        return (uint32_t)(k >> shift) & ((1u << R) - 1u);
    }
}

__device__ __forceinline__ uint32_t lane_id()
{
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// Number of set bits of m below this lane.
__device__ __forceinline__ uint32_t lanes_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Mask of the lanes of this (full) wave whose R-bit digit equals ours.
// For every bit b: s = 0 or ~0 (our bit, sign-extended), bal = the wave's
// ballot of that bit; bal ^ s marks the lanes whose bit b differs from ours.
// OR-ing those over the R bits (one 3-input v_bitop3 per half: a | (b ^ c))
// leaves exactly the equal lanes clear.
template <int R>
__device__ __forceinline__ uint64_t peer_mask(uint32_t d)
{
    uint32_t diff_lo = 0, diff_hi = 0;
#pragma unroll
    for (int b = 0; b < R; ++b) {
        const uint32_t s = (uint32_t)__builtin_amdgcn_sbfe((int32_t)d, b, 1);
        const uint64_t bal = __ballot(s != 0);
        diff_lo = __builtin_amdgcn_bitop3_b32(diff_lo, (uint32_t)bal, s, 0xF6);
        diff_hi = __builtin_amdgcn_bitop3_b32(diff_hi, (uint32_t)(bal >> 32), s, 0xF6);
    }
    return ~(((uint64_t)diff_hi << 32) | diff_lo);
}

// Lane i of each 16-lane row takes lane i - n of its row, 0 where that
// lane does not exist (DPP row shift, VALU latency, no LDS round trip).
template <int N>
__device__ __forceinline__ uint32_t row_shr(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x110 + N, 0xf, 0xf, false);
}

// Inclusive scan across the 64 lanes of a wave, with DPP: shifts by 1, 2,
// 4 and 8 lanes make each 16-lane row an inclusive scan; then row 0's last
// lane is added into row 1 and row 2's into row 3 (row_bcast:15), and lane
// 31 (the total of rows 0-1) into rows 2 and 3 (row_bcast:31).
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v)
{
    v += row_shr<1>(v);
    v += row_shr<2>(v);
    v += row_shr<4>(v);
    v += row_shr<8>(v);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);
    return v;
}

// Exclusive scan of one value per thread over the first max(NB, 64) threads
// of the block (NB <= 256: one value per digit bin; threads past NB must pass
// 0).  `tmp` is 4 words of LDS.  Must be called by every thread of the block
// (barriers inside); threads past the scanned ones get 0.
template <int NB>
__device__ __forceinline__ uint32_t bins_exclusive_scan(uint32_t v, uint32_t *tmp)
{
    static_assert(NB <= kRadix, "at most 256 bins");
    constexpr uint32_t kT = NB < kWave ? kWave : NB;
    const uint32_t t = threadIdx.x;
    const uint32_t w = t / kWave;
    uint32_t inc = 0;
    if (t < kT) {
        inc = wave_inclusive_scan(v);
        if ((t & (kWave - 1)) == kWave - 1)
            tmp[w] = inc;
    }
    __syncthreads();
    uint32_t excl = 0;
    if (t < kT) {
        uint32_t before = 0;
        for (uint32_t i = 0; i < w; ++i)
            before += tmp[i];
        excl = before + inc - v;
    }
    __syncthreads();
    return excl;
}

// Stable rank of ITEMS keys per lane among the keys of this wave that share
// their R-bit digit.  Items are visited j = 0..ITEMS-1 and, within an item,
// by lane, which must be the input order of the wave's elements.  wc is the
// wave's 2^R-entry running count per digit (zeroed by the caller); wm a
// 2^R-entry table of 64-bit lane masks (zeroed by the caller, left zeroed).
// For every item each lane ORs its bit into its digit's slot and reads the
// slot back: that is the mask of lanes holding the same digit.  The group's
// lowest lane advances the count and clears the slot.  rank = count before
// the group + lanes of the group below this one.  After the call wc holds
// the wave's total per digit.
template <int R, typename K, int ITEMS>
__device__ __forceinline__ void wave_rank(const K (&key)[ITEMS], int shift, uint32_t *wc,
                                          uint64_t *wm, uint32_t lane, uint32_t (&rank)[ITEMS])
{
    // the lane's bit lives in one 32-bit half of the 64-bit mask: OR only
    // that half (half the LDS bytes of a 64-bit OR, the same mask)
    const uint32_t lane_bit = 1u << (lane & 31);
    uint32_t *wm32 = (uint32_t *)wm + (lane >> 5);
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const uint32_t d = digit_of<R>(key[j], shift);
        atomicOr(&wm32[2 * d], lane_bit);
        const uint64_t m = wm[d];
        const uint32_t c = wc[d];
        const uint32_t below = lanes_below(m);
        rank[j] = c + below;
        if (below == 0) {
            wc[d] = c + (uint32_t)__popcll(m);
            wm[d] = 0;
        }
    }
}

// The same ranks as wave_rank, with the peer mask from R ballots (VALU work)
// instead of the LDS table: every lane reads its digit's running count, the
// group's lowest lane advances it.  wc as in wave_rank.
template <int R, typename K, int ITEMS>
__device__ __forceinline__ void wave_rank_ballot(const K (&key)[ITEMS], int shift, uint32_t *wc,
                                                 uint32_t (&rank)[ITEMS])
{
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const uint32_t d = digit_of<R>(key[j], shift);
        const uint64_t m = peer_mask<R>(d);
        const uint32_t below = lanes_below(m);
        const uint32_t c = wc[d];
        rank[j] = c + below;
        if (below == 0)
            wc[d] = c + (uint32_t)__popcll(m);
    }
}

}  // namespace rs
