// LSD radix sort for gfx950 (MI355X) behind the C-ABI declared in rs.h.
//
// Method (paper, Section 2.6): d = K/8 passes of 8-bit digits, least
// significant first, each a stable counting sort.  The GPU realisation:
//
//   k_init     zero the control block and the digit histograms
//   k_hist     one read of the keys -> histograms of all d digit positions;
//              also clears the look-back words of every pass
//   k_plan     one workgroup: scans each histogram row into digit_base (the
//              counting sort's exclusive prefix sums) and writes a plan:
//              which passes move data (a pass whose histogram has a single
//              non-empty digit is the identity and is skipped) and which
//              buffer each pass reads and writes
//   k_pass     one per digit position: a single sweep over the data that
//              counts, scans (decoupled look-back across tiles) and places
//              each tile; see rs_device.h.
//   k_finalize in-place sorts with an odd number of moving passes only:
//              copy the scratch copy back.
//
// Everything after argument validation is enqueued on the caller's stream
// with no host synchronisation.
#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "rs.h"
#include "rs_block.h"
#include "rs_device.h"
#include "rs_segmented.h"

namespace rs {

// ---------------------------------------------------------------------------
// Tile shapes.

// Tile of one digit pass: kThreads x kItems elements, one tile per
// workgroup.
//   kLookback  predecessor tiles read per look-back round trip
//   kLdsMatch  find the lanes of a wave that share a digit through a per-wave
//              LDS table of 64-bit lane masks (each lane ORs its bit into its
//              digit's slot and reads the slot back) instead of eight ballots
//   kGroup     consecutive tiles claimed as a group (see claim_tile)
// Keys are staged in LDS, written out, then the values go through the same
// buffer; the mask table is only live while ranking and shares it too.  Big
// tiles amortise the per-tile latencies (tile claim, look-back) and make the
// digit runs of the scatter longer; 64-bit pairs need a smaller tile to fit
// the registers of 1024 threads.
template <typename K, bool HAS_V>
struct PassShape {
    static constexpr int kThreads = (sizeof(K) == 8 && HAS_V) ? 512 : 1024;
    static constexpr int kItems = 16;
    static constexpr int kTile = kThreads * kItems;
    static constexpr int kLookback = 8;
    static constexpr bool kLdsMatch = true;
    static constexpr int kGroup = 8;
};

constexpr int kHistThreads = 256;

struct Bufs {
    const void *in_k;
    const void *in_v;
    void *out_k;
    void *out_v;
    void *tmp_k;
    void *tmp_v;
};

template <typename T>
__device__ __forceinline__ T *pick(const Bufs &b, uint32_t id, bool values)
{
    const void *p = values ? (id == kBufIn ? b.in_v : id == kBufOut ? b.out_v : b.tmp_v)
                           : (id == kBufIn ? b.in_k : id == kBufOut ? b.out_k : b.tmp_k);
    return (T *)p;
}

// ---------------------------------------------------------------------------
// k_init: clear the control block and the histograms.

__global__ void k_init(uint32_t *ctrl, uint32_t *hist, int hist_words)
{
    for (int i = threadIdx.x; i < kCtrlWords; i += blockDim.x)
        ctrl[i] = 0;
    for (int i = threadIdx.x; i < hist_words; i += blockDim.x)
        hist[i] = 0;
}

// ---------------------------------------------------------------------------
// k_hist: all-digit histograms in one read of the keys; also clears the
// look-back words of every pass.

struct HistArgs {
    const void *keys;
    uint32_t n;
    uint32_t head;        // leading keys before the first 16-byte boundary
    uint32_t nvec;        // 16-byte vectors after the head
    uint32_t *hist;       // [d][256]
    uint4 *status;        // look-back words of all passes, cleared here
    uint64_t status_vec;  // number of uint4 in status
};

// Count one key's D digits into the wave's LDS sub-histograms.
template <typename K>
__device__ __forceinline__ void count_one(uint32_t (*sh)[kRadix], K key)
{
    constexpr int D = KeyTraits<K>::kBits / kRadixBits;
#pragma unroll
    for (int p = 0; p < D; ++p)
        atomicAdd(&sh[p][KeyTraits<K>::digit(key, p * kRadixBits)], 1u);
}

// Count a batch of NK keys per thread (a full batch: every lane active).
// Key slot i of the wave covers 64 neighbouring vectors of the input, and in
// skewed inputs (zero, sorted, reverse) a digit position is often the same
// over the whole slot; same-address LDS atomics serialise (0.5 lanes/clock
// against ~6 for spread addresses), so such a slot adds 64 once.
template <typename K, int NK>
__device__ __forceinline__ void count_batch(uint32_t (*sh)[kRadix], const K (&key)[NK])
{
    constexpr int D = KeyTraits<K>::kBits / kRadixBits;
#pragma unroll
    for (int p = 0; p < D; ++p) {
#pragma unroll
        for (int i = 0; i < NK; ++i) {
            const uint32_t dg = KeyTraits<K>::digit(key[i], p * kRadixBits);
            const uint32_t first = __builtin_amdgcn_readfirstlane(dg);
            if (__ballot(dg != first) == 0) {
                if (lane_id() == 0)
                    atomicAdd(&sh[p][first], (uint32_t)kWave);
            } else {
                atomicAdd(&sh[p][dg], 1u);
            }
        }
    }
}

template <typename K>
__global__ __launch_bounds__(kHistThreads) void k_hist(HistArgs a)
{
    constexpr int D = KeyTraits<K>::kBits / kRadixBits;
    constexpr int W = kHistThreads / kWave;
    constexpr int KPV = 16 / (int)sizeof(K);  // keys per 16-byte vector
    constexpr int VPT = 16 / KPV;             // vectors per thread per batch
    constexpr int NK = VPT * KPV;             // 16 keys per thread per batch
    constexpr uint32_t BATCH = kHistThreads * VPT;
    __shared__ uint32_t sh[W][D][kRadix];

    const uint32_t t = threadIdx.x;
    const uint32_t w = t / kWave;
    for (int i = t; i < W * D * kRadix; i += kHistThreads)
        (&sh[0][0][0])[i] = 0;

    // clear the look-back words of every pass
    const uint64_t gtid = (uint64_t)blockIdx.x * kHistThreads + t;
    const uint64_t gstride = (uint64_t)gridDim.x * kHistThreads;
    for (uint64_t i = gtid; i < a.status_vec; i += gstride)
        a.status[i] = make_uint4(0, 0, 0, 0);
    __syncthreads();

    const K *keys = (const K *)a.keys;
    const uint4 *vec = (const uint4 *)(keys + a.head);
    const uint64_t full_batches = a.nvec / BATCH;
    for (uint64_t b = blockIdx.x; b < full_batches; b += gridDim.x) {
        // vector v of this thread: b*BATCH + v*THREADS + t (each wave load is 1 KB contiguous)
        uint4 v[VPT];
#pragma unroll
        for (int i = 0; i < VPT; ++i)
            v[i] = vec[b * BATCH + (uint64_t)i * kHistThreads + t];
        K key[NK];
#pragma unroll
        for (int i = 0; i < VPT; ++i) {
            if constexpr (KPV == 4) {
                key[4 * i + 0] = (K)v[i].x;
                key[4 * i + 1] = (K)v[i].y;
                key[4 * i + 2] = (K)v[i].z;
                key[4 * i + 3] = (K)v[i].w;
            } else {
                key[2 * i + 0] = (K)(((uint64_t)v[i].y << 32) | v[i].x);
                key[2 * i + 1] = (K)(((uint64_t)v[i].w << 32) | v[i].z);
            }
        }
        count_batch<K, NK>(sh[w], key);
    }
    // the rest: unaligned head, vectors after the last full batch, ragged
    // tail -- element by element, spread over the whole grid
    const uint64_t rest0 = (uint64_t)a.head + full_batches * BATCH * KPV;
    const uint64_t extra = a.head + (a.n - rest0);
    for (uint64_t i = gtid; i < extra; i += gstride) {
        const uint64_t idx = i < a.head ? i : rest0 + (i - a.head);
        count_one<K>(sh[w], keys[idx]);
    }
    __syncthreads();

    for (int i = t; i < D * kRadix; i += kHistThreads) {
        uint32_t s = 0;
#pragma unroll
        for (int ww = 0; ww < W; ++ww)
            s += (&sh[ww][0][0])[i];
        if (s)
            atomicAdd(&a.hist[i], s);
    }

}

// ---------------------------------------------------------------------------
// k_plan (one workgroup): digit_base = exclusive scan of each histogram row
// (the counting sort's starting offsets), and the plan of every pass.  A
// pass whose digit is the same for all n keys is the identity permutation
// and is skipped; the remaining passes alternate between the output and the
// scratch copy so that the last one lands in the output.

struct PlanArgs {
    const uint32_t *hist;
    uint32_t *digit_base;
    uint32_t *ctrl;
    uint32_t n;
    int in_place;
};

template <int D>
__global__ __launch_bounds__(kRadix) void k_plan(PlanArgs a)
{
    __shared__ uint32_t s_tmp[8];
    __shared__ int s_trivial[D];
    __shared__ int s_skewed[D];
    __shared__ unsigned long long s_sq[kRadix / kWave];
    const uint32_t t = threadIdx.x;
    for (int p = 0; p < D; ++p) {
        const uint32_t c = a.hist[p * kRadix + t];
        const uint32_t ex = block_exclusive_scan_256<kRadix>(c, s_tmp);
        a.digit_base[p * kRadix + t] = ex;
        const int triv = __syncthreads_or(c == a.n);
        // chance that two keys share this digit: sum_b (c_b / n)^2
        unsigned long long sq = (unsigned long long)c * c;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
            sq += __shfl_xor(sq, off);
        if ((t & (kWave - 1)) == 0)
            s_sq[t / kWave] = sq;
        __syncthreads();
        if (t == 0) {
            s_trivial[p] = triv;
            unsigned long long tot = 0;
            for (int i = 0; i < kRadix / kWave; ++i)
                tot += s_sq[i];
            // above 1/100 many lanes of a wave share a slot of the LDS lane-mask
            // table, whose same-address atomics serialise; ballots do not
            s_skewed[p] = tot * 100ull > (unsigned long long)a.n * a.n;
        }
        __syncthreads();
    }
    __syncthreads();
    if (t == 0) {
        int q_total = 0;
        for (int p = 0; p < D; ++p)
            q_total += !s_trivial[p];
        const bool odd_in_place = a.in_place && (q_total & 1);
        int q = 0;
        uint32_t prev = kBufIn;
        for (int p = 0; p < D; ++p) {
            uint32_t plan = 0;
            if (!s_trivial[p]) {
                uint32_t dst;
                if (odd_in_place)
                    dst = (q & 1) ? kBufOut : kBufTmp;
                else
                    dst = ((q_total - 1 - q) & 1) ? kBufTmp : kBufOut;
                plan = kPlanRun | (prev << kPlanSrcShift) | (dst << kPlanDstShift) |
                       (s_skewed[p] ? kPlanBallot : 0u);
                prev = dst;
                ++q;
            }
            a.ctrl[kCtrlPlan + p] = plan;
        }
        if (q_total == 0 && !a.in_place)
            a.ctrl[kCtrlPlan + D - 1] = kPlanCopyIn;
        a.ctrl[kCtrlFinal] = odd_in_place ? 1u : 0u;
    }
}

// ---------------------------------------------------------------------------
// k_pass: one digit pass in a single sweep.

struct PassArgs {
    Bufs b;
    uint32_t n;
    int pass;
    int shift;
    uint32_t *ctrl;
    const uint32_t *digit_base;  // row of this pass
    uint32_t *status;            // [tiles][256] of this pass
    uint32_t *claims;            // per-XCD claim counters and group lists
    uint32_t num_tiles;
    uint32_t num_groups;
};

// Which compute die (XCD) this wave runs on, from the XCC_ID hardware register.
__device__ __forceinline__ uint32_t xcc_id()
{
    return __builtin_amdgcn_s_getreg(20 | (0 << 6) | ((4 - 1) << 11)) & 7u;
}

constexpr uint32_t kNoTile = 0xFFFFFFFFu;

// Claim the next tile for this workgroup (called by one thread).
//
// The digit runs of consecutive tiles meet inside shared cache lines.  When
// the two tiles run on different XCDs, each XCD's L2 writes back a partial
// line, which costs far more than one full line.  So consecutive tiles are
// handed out in groups of GROUP, and the tiles of a group go to workgroups of
// one XCD that start at about the same time:
//   * every XCD keeps its own claim counter; claim k on XCD x takes tile
//     k % GROUP of the XCD's group number k / GROUP;
//   * the claim with k % GROUP == 0 opens that group: it takes the next group
//     from the global counter and publishes the group's id in the XCD's
//     list; the other claims of the same group wait for that id (the opener
//     is running, so the wait is short).
// Groups are opened in global order and the tiles of one XCD's groups
// increase with its claim counter, so the lowest unfinished tile is always
// held or next to be claimed by a running workgroup of its XCD (workgroups
// keep claiming until the groups run out): the look-back waits cannot
// depend on a workgroup that has not started.
//
// claims layout: [0, 8) per-XCD claim counters, then [8 + x*G + j] the id+1
// of group j of XCD x (0 = not yet published, kNoTile = no group left).
template <int GROUP>
__device__ __forceinline__ uint32_t claim_tile(const PassArgs &a, uint32_t xcc)
{
    uint32_t *ctr = &a.ctrl[kCtrlTileCounter + a.pass];
    if constexpr (GROUP == 1) {
        (void)xcc;
        const uint32_t t = atomicAdd(ctr, 1u);
        return t < a.num_tiles ? t : kNoTile;
    } else {
        uint32_t *list = a.claims + 8 + (uint64_t)xcc * a.num_groups;
        while (true) {
            const uint32_t k = atomicAdd(&a.claims[xcc], 1u);
            const uint32_t j = k / GROUP, i = k % GROUP;
            if (j >= a.num_groups)
                return kNoTile;
            uint32_t v;
            if (i == 0) {
                const uint32_t g = atomicAdd(ctr, 1u);
                v = g < a.num_groups ? g + 1 : kNoTile;
                __hip_atomic_store(&list[j], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                while ((v = __hip_atomic_load(&list[j], __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT)) == 0)
                    __builtin_amdgcn_s_sleep(1);
            }
            if (v == kNoTile)
                return kNoTile;
            const uint32_t t = (v - 1) * GROUP + i;
            if (t < a.num_tiles)
                return t;
            // past the end of a short last group: claim again
        }
    }
}

// dst[lo, hi) = src[lo, hi), 16-byte vectors where both arrays allow it.
template <typename T>
__device__ __forceinline__ void copy_range(const T *src, T *dst, uint64_t lo, uint64_t hi,
                                           uint32_t t, uint32_t threads)
{
    constexpr uint64_t E = 16 / sizeof(T);  // elements per vector
    const bool vec = ((((uintptr_t)(src + lo)) | ((uintptr_t)(dst + lo))) & 15) == 0;
    if (vec) {
        const uint64_t nv = (hi - lo) / E;
        const uint4 *s4 = (const uint4 *)(src + lo);
        uint4 *d4 = (uint4 *)(dst + lo);
        for (uint64_t i = t; i < nv; i += threads)
            d4[i] = s4[i];
        for (uint64_t i = lo + nv * E + t; i < hi; i += threads)
            dst[i] = src[i];
    } else {
        for (uint64_t i = lo + t; i < hi; i += threads)
            dst[i] = src[i];
    }
}

template <typename K, typename V, bool HAS_V>
__device__ __forceinline__ void copy_tile(const PassArgs &a, uint64_t lo, uint64_t hi,
                                          uint32_t t, uint32_t threads)
{
    copy_range(pick<const K>(a.b, kBufIn, false), pick<K>(a.b, kBufOut, false), lo, hi, t,
               threads);
    if constexpr (HAS_V)
        copy_range(pick<const V>(a.b, kBufIn, true), pick<V>(a.b, kBufOut, true), lo, hi, t,
                   threads);
}

// p[i] = v.  For 4-byte elements the byte offset fits in 32 bits (n < 2^30),
// which lets the store use a scalar base and a 32-bit vector offset.
template <typename T>
__device__ __forceinline__ void store_at(T *p, uint32_t i, T v)
{
    if constexpr (sizeof(T) == 4)
        *(T *)((char *)p + (i << 2)) = v;
    else
        p[i] = v;
}

template <typename K, typename V, bool HAS_V, int ITEMS>
__device__ __forceinline__ void load_tile(const K *tk, const V *tv, uint32_t valid, uint32_t off0,
                                          K (&key)[ITEMS], V (&val)[HAS_V ? ITEMS : 1], bool full)
{
    if (full) {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j)
            key[j] = tk[off0 + j * kWave];
        if constexpr (HAS_V) {
#pragma unroll
            for (int j = 0; j < ITEMS; ++j)
                val[j] = tv[off0 + j * kWave];
        }
    } else {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j)
            key[j] = off0 + j * kWave < valid ? tk[off0 + j * kWave] : KeyTraits<K>::kPad;
        if constexpr (HAS_V) {
#pragma unroll
            for (int j = 0; j < ITEMS; ++j)
                val[j] = off0 + j * kWave < valid ? tv[off0 + j * kWave] : (V)0;
        }
    }
}

// LDS of one digit pass over tiles of T elements.
template <typename K, typename V, int THREADS, int T>
struct PassLds {
    static constexpr int W = THREADS / kWave;
    static constexpr size_t kStageBytes = (size_t)T * sizeof(K);
    uint32_t wcnt[W * kRadix];  // per wave and digit: count, then base in tile
    uint32_t gbase[kRadix];
    uint32_t tmp[8];
    uint32_t tile;
    __attribute__((aligned(16))) unsigned char stage[kStageBytes];
};

// One tile of a digit pass (the paper's counting sort, Section 2.6, spread
// over workgroups): rank, publish the tile's digit counts, decoupled
// look-back over tiles [first_tile, tile), stage in LDS, write the digit
// runs.  The tile's elements are tk/tv[0, valid); destination index i of the
// digit-sorted sequence is dk/dv[i] for i < limit.  dbase (threads < 256) is
// the digit's starting offset in that sequence.  Ends with a barrier.
template <typename K, typename V, bool HAS_V, int THREADS, int ITEMS, int LBW, bool LDS_MATCH>
__device__ __forceinline__ void pass_tile(PassLds<K, V, THREADS, THREADS * ITEMS> &L,
                                          const K *tk, const V *tv, K *dk, V *dv,
                                          uint32_t valid, uint32_t limit, uint32_t tile,
                                          uint32_t first_tile, uint32_t *status, uint32_t dbase,
                                          int shift, bool ballot_rank)
{
    constexpr int T = THREADS * ITEMS;
    constexpr int W = THREADS / kWave;
    static_assert(sizeof(V) == sizeof(K), "values have the key's width");
    static_assert(!LDS_MATCH || (size_t)W * kRadix * 8 <= (size_t)T * sizeof(K),
                  "the mask table lives in the staging buffer");
    K *s_k = (K *)L.stage;
    V *s_v = (V *)L.stage;
    uint64_t *s_mask = (uint64_t *)L.stage;
    const uint32_t t = threadIdx.x;
    const uint32_t w = t / kWave;
    const uint32_t lane = t % kWave;
    const uint32_t off0 = w * (kWave * ITEMS) + lane;
    uint32_t *wc = L.wcnt + w * kRadix;

    // load: item j of lane l is element j*64 + l of this wave's run
    K key[ITEMS];
    V val[HAS_V ? ITEMS : 1];
    load_tile<K, V, HAS_V, ITEMS>(tk, tv, valid, off0, key, val, valid == (uint32_t)T);

    // count: stable rank of every item among the wave's items of its digit
    uint32_t rank[ITEMS];
    if (LDS_MATCH && !ballot_rank) {
        wave_rank<K, KeyTraits<K>, ITEMS>(key, shift, wc, s_mask + w * kRadix, lane, rank);
    } else {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t d = KeyTraits<K>::digit(key[j], shift);
            const uint64_t m = peer_mask(d);
            const uint32_t below = lanes_below(m);
            const uint32_t leader = (uint32_t)__builtin_ctzll(m);
            uint32_t old = 0;
            if (below == 0)
                old = atomicAdd(&wc[d], (uint32_t)__popcll(m));
            old = shfl_idx(old, leader);
            rank[j] = old + below;
        }
    }
    __syncthreads();

    // scan: wave offsets per digit, tile count, publish the aggregate,
    // tile-local offsets
    uint32_t cnt = 0;
    if (t < kRadix) {
#pragma unroll
        for (int ww = 0; ww < W; ++ww) {
            const uint32_t c = L.wcnt[ww * kRadix + t];
            L.wcnt[ww * kRadix + t] = cnt;
            cnt += c;
        }
        __hip_atomic_store(&status[(uint64_t)tile * kRadix + t],
                           (tile == first_tile ? kFlagInc : kFlagAgg) | cnt, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    const uint32_t excl = block_exclusive_scan_256<THREADS>(cnt, L.tmp);
    if (t < kRadix) {
        // decoupled look-back: read LBW predecessors per round trip, add
        // their counts in order up to the first inclusive one; on a tile
        // that has not published yet, wait and re-read from there
        uint32_t prefix = 0;
        int64_t k = (int64_t)tile - 1;
        const int64_t lo = first_tile;
        while (k >= lo) {
            uint32_t st[LBW];
#pragma unroll
            for (int i = 0; i < LBW; ++i)
                st[i] = (k - i >= lo)
                            ? __hip_atomic_load(&status[(uint64_t)(k - i) * kRadix + t],
                                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                            : kFlagInc;
            int used = 0;
            bool done = false;
#pragma unroll
            for (int i = 0; i < LBW; ++i) {
                if (!done && used == i) {
                    const uint32_t f = st[i] & kFlagMask;
                    if (f != 0) {
                        prefix += st[i] & kCountMask;
                        done = f == kFlagInc;
                        used = i + 1;
                    }
                }
            }
            if (done)
                break;
            k -= used;
            if (used < LBW)
                __builtin_amdgcn_s_sleep(1);
        }
        if (tile != first_tile)
            __hip_atomic_store(&status[(uint64_t)tile * kRadix + t], kFlagInc | (prefix + cnt),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        L.gbase[t] = dbase + prefix - excl;
#pragma unroll
        for (int ww = 0; ww < W; ++ww)
            L.wcnt[ww * kRadix + t] += excl;
    }
    __syncthreads();

    // place: stage the keys in rank order, then write each digit run out
    // with consecutive lanes on consecutive addresses; then the values
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        rank[j] += wc[KeyTraits<K>::digit(key[j], shift)];  // position in the tile
        s_k[rank[j]] = key[j];
    }
    __syncthreads();
    uint32_t dst[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t pos = i * THREADS + t;
        const K k = s_k[pos];
        dst[i] = L.gbase[KeyTraits<K>::digit(k, shift)] + pos;
        if (dst[i] < limit)
            store_at(dk, dst[i], k);
    }
    if constexpr (HAS_V) {
        __syncthreads();
#pragma unroll
        for (int j = 0; j < ITEMS; ++j)
            s_v[rank[j]] = val[j];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < ITEMS; ++i)
            if (dst[i] < limit)
                store_at(dv, dst[i], s_v[i * THREADS + t]);
    }
    __syncthreads();  // LDS is reused by the next tile
}

template <typename K, typename V, bool HAS_V>
__global__ __launch_bounds__((PassShape<K, HAS_V>::kThreads)) void k_pass(PassArgs a)
{
    using S = PassShape<K, HAS_V>;
    constexpr int THREADS = S::kThreads;
    constexpr int T = S::kTile;
    __shared__ PassLds<K, V, THREADS, T> L;

    const uint32_t t = threadIdx.x;
    const uint32_t plan = a.ctrl[kCtrlPlan + a.pass];
    if (!(plan & kPlanRun)) {
        if (plan & kPlanCopyIn) {
            for (uint64_t tl = blockIdx.x; tl < a.num_tiles; tl += gridDim.x) {
                const uint64_t lo = tl * T;
                const uint64_t hi = std::min<uint64_t>(lo + T, a.n);
                copy_tile<K, V, HAS_V>(a, lo, hi, t, THREADS);
            }
        }
        return;
    }
    const uint32_t src = (plan >> kPlanSrcShift) & 3u;
    const uint32_t dstb = (plan >> kPlanDstShift) & 3u;
    const K *sk = pick<const K>(a.b, src, false);
    const V *sv = HAS_V ? pick<const V>(a.b, src, true) : nullptr;
    K *dk = pick<K>(a.b, dstb, false);
    V *dv = HAS_V ? pick<V>(a.b, dstb, true) : nullptr;
    // this digit's starting offset, fetched early (used after the look-back)
    const uint32_t dbase = t < kRadix ? a.digit_base[t] : 0u;
    const uint32_t xcc = t == 0 ? xcc_id() : 0u;
    while (true) {
        if (t == 0)
            L.tile = claim_tile<S::kGroup>(a, xcc);
        for (int i = t; i < PassLds<K, V, THREADS, T>::W * kRadix; i += THREADS) {
            L.wcnt[i] = 0;
            if constexpr (S::kLdsMatch)
                ((uint64_t *)L.stage)[i] = 0;
        }
        __syncthreads();
        const uint32_t tile = L.tile;
        if (tile == kNoTile)
            break;
        const uint64_t tb = (uint64_t)tile * T;
        const uint32_t valid = (uint32_t)std::min<uint64_t>(T, a.n - tb);
        pass_tile<K, V, HAS_V, THREADS, S::kItems, S::kLookback, S::kLdsMatch>(
            L, sk + tb, HAS_V ? sv + tb : nullptr, dk, dv, valid, a.n, tile, 0, a.status, dbase,
            a.shift, (plan & kPlanBallot) != 0);
    }
}

// ---------------------------------------------------------------------------
// k_seg_pass: one digit pass over the tiles of every large segment of a
// segmented sort.  Each segment's tiles are consecutive in the batched tile
// sequence and its look-back chain starts at its first tile.

struct SegPassArgs {
    const void *src_k;
    const void *src_v;
    void *dst_k;
    void *dst_v;
    const SegLarge *large;
    const uint32_t *tile_seg;
    const uint32_t *seg_base;  // [large segment][d][256]
    uint32_t *ctrl;            // segmented control block
    uint32_t *status;          // look-back words of this pass
    uint32_t *claims;          // claim counters of this pass
    uint32_t max_tiles;        // tiles the workspace holds
    int pass;
    int shift;
    int d;
};

template <typename K, typename V, bool HAS_V>
__global__ __launch_bounds__((PassShape<K, HAS_V>::kThreads)) void k_seg_pass(SegPassArgs a)
{
    using S = PassShape<K, HAS_V>;
    constexpr int THREADS = S::kThreads;
    constexpr int T = S::kTile;
    __shared__ PassLds<K, V, THREADS, T> L;
    const uint32_t t = threadIdx.x;
    PassArgs pa{};
    pa.ctrl = a.ctrl + (kSegPassCounter - kCtrlTileCounter);
    pa.pass = a.pass;
    pa.claims = a.claims;
    pa.num_tiles = std::min(a.ctrl[kSegTiles], a.max_tiles);
    pa.num_groups = (pa.num_tiles + S::kGroup - 1) / S::kGroup;
    const uint32_t xcc = t == 0 ? xcc_id() : 0u;
    while (true) {
        if (t == 0)
            L.tile = claim_tile<S::kGroup>(pa, xcc);
        for (int i = t; i < PassLds<K, V, THREADS, T>::W * kRadix; i += THREADS) {
            L.wcnt[i] = 0;
            if constexpr (S::kLdsMatch)
                ((uint64_t *)L.stage)[i] = 0;
        }
        __syncthreads();
        const uint32_t tile = L.tile;
        if (tile == kNoTile)
            break;
        const uint32_t seg = a.tile_seg[tile];
        const SegLarge rec = a.large[seg];
        const uint32_t lt = tile - rec.tile_start;
        const uint32_t first = lt * T;
        const uint32_t valid = rec.size > first ? std::min<uint32_t>(T, rec.size - first) : 0u;
        const uint32_t dbase =
            t < kRadix ? a.seg_base[((uint64_t)seg * a.d + a.pass) * kRadix + t] : 0u;
        const uint64_t off = rec.start + (uint64_t)lt * T;
        pass_tile<K, V, HAS_V, THREADS, S::kItems, S::kLookback, S::kLdsMatch>(
            L, (const K *)a.src_k + off, HAS_V ? (const V *)a.src_v + off : nullptr,
            (K *)a.dst_k + rec.start, HAS_V ? (V *)a.dst_v + rec.start : nullptr, valid, rec.size,
            tile, rec.tile_start, a.status, dbase, a.shift, false);
    }
}

// Grid-stride fill of n uint4 with zero (clears counters without a memset
// node, so a captured graph stays memset-free).
__global__ void k_zero(uint4 *p, uint64_t n)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        p[i] = make_uint4(0, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// k_finalize: in-place sort with an odd number of moving passes.

template <typename K, typename V, bool HAS_V>
__global__ void k_finalize(Bufs b, uint32_t n, const uint32_t *ctrl)
{
    if (ctrl[kCtrlFinal] != 1u)
        return;
    const K *tk = (const K *)b.tmp_k;
    K *ok = (K *)b.out_k;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        ok[i] = tk[i];
        if constexpr (HAS_V)
            ((V *)b.out_v)[i] = ((const V *)b.tmp_v)[i];
    }
}

}  // namespace rs

// ===========================================================================
// Host side: validation, workspace layout, launches.

using namespace rs;

struct ProfRecord {
    const char *name;
    int tag;
    size_t ev;  // index of the first of two events in the pool
};

struct rs_context {
    int device = 0;
    void *own_ws = nullptr;
    size_t own_ws_bytes = 0;
    // per-kernel timing (rs_profile_*)
    bool prof = false;
    int prof_tag = 0;
    std::vector<ProfRecord> recs;
    std::vector<hipEvent_t> events;  // grow-only pool, reused after a reset
    size_t events_used = 0;
    uint32_t cus = 0;  // compute units, queried on first use
};

// Launch through f(), bracketed by two events when profiling is on.
template <typename F>
static void launch(rs_context *ctx, hipStream_t s, const char *name, F &&f)
{
    if (!ctx->prof) {
        f();
        return;
    }
    while (ctx->events.size() < ctx->events_used + 2) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) {
            (void)hipGetLastError();
            f();
            return;
        }
        ctx->events.push_back(e);
    }
    const size_t i = ctx->events_used;
    ctx->events_used += 2;
    (void)hipEventRecord(ctx->events[i], s);
    f();
    (void)hipEventRecord(ctx->events[i + 1], s);
    ctx->recs.push_back({name, ctx->prof_tag, i});
}

static thread_local std::string g_last_error;

static rs_status fail(rs_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

static inline uint64_t align_up(uint64_t x, uint64_t a)
{
    return (x + a - 1) / a * a;
}

struct Layout {
    int d;
    uint32_t tile;
    uint64_t tiles;
    uint64_t off_ctrl, off_hist, off_base, off_status, off_tmp_k, off_tmp_v, total;
    uint64_t status_bytes;  // look-back words and claim counters of all passes
    uint64_t claim_words;
};

static Layout make_layout(int key_bytes, bool has_values, uint64_t n)
{
    Layout L{};
    L.d = key_bytes;  // 8-bit digits: one pass per key byte
    if (key_bytes == 4)
        L.tile = has_values ? PassShape<uint32_t, true>::kTile : PassShape<uint32_t, false>::kTile;
    else
        L.tile = has_values ? PassShape<uint64_t, true>::kTile : PassShape<uint64_t, false>::kTile;
    L.tiles = (n + L.tile - 1) / L.tile;
    uint64_t o = 0;
    L.off_ctrl = o;
    o = align_up(o + kCtrlWords * 4, 256);
    L.off_hist = o;
    o = align_up(o + (uint64_t)L.d * kRadix * 4, 256);
    L.off_base = o;
    o = align_up(o + (uint64_t)L.d * kRadix * 4, 256);
    L.off_status = o;
    L.claim_words = 8 + 8 * L.tiles;  // per-XCD counters + per-XCD group lists
    L.status_bytes = align_up((uint64_t)L.d * (L.tiles * kRadix + L.claim_words) * 4, 16);
    o = align_up(o + L.status_bytes, 256);
    L.off_tmp_k = o;
    o = align_up(o + n * key_bytes, 256);
    L.off_tmp_v = o;
    o = align_up(o + (has_values ? n * key_bytes : 0), 256);
    L.total = o;
    return L;
}

static bool overlaps(const void *a, uint64_t an, const void *b, uint64_t bn)
{
    uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return an && bn && x < y + bn && y < x + an;
}

namespace {

struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess)
            return;
        if (prev != dev && hipSetDevice(dev) != hipSuccess)
            return;
        ok = true;
    }
    ~DeviceGuard()
    {
        if (ok && prev >= 0)
            (void)hipSetDevice(prev);
    }
};

}  // namespace

// Compute units of the context's device (queried once).
static uint32_t ctx_cus(rs_context *ctx)
{
    if (ctx->cus == 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, ctx->device) !=
                hipSuccess ||
            v < 1) {
            (void)hipGetLastError();
            v = 1;
        }
        ctx->cus = (uint32_t)v;
    }
    return ctx->cus;
}

static rs_status get_workspace(rs_context *ctx, void *ws, size_t ws_bytes, uint64_t need,
                               void **out)
{
    if (ws) {
        *out = ws;
        return RS_OK;
    }
    if (ctx->own_ws_bytes < need) {
        if (ctx->own_ws) {
            (void)hipFree(ctx->own_ws);
            ctx->own_ws = nullptr;
            ctx->own_ws_bytes = 0;
        }
        if (hipMalloc(&ctx->own_ws, need) != hipSuccess) {
            (void)hipGetLastError();
            ctx->own_ws = nullptr;
            return fail(RS_ERR_OUT_OF_MEMORY, "could not allocate %llu bytes of scratch",
                        (unsigned long long)need);
        }
        ctx->own_ws_bytes = need;
    }
    (void)ws_bytes;
    *out = ctx->own_ws;
    return RS_OK;
}

static rs_status validate_sort(const rs_context *ctx, int key_bytes, const void *kin,
                               const void *vin, void *kout, void *vout, bool has_values,
                               uint64_t n, const void *ws, size_t ws_bytes, Layout *L)
{
    if (!ctx)
        return fail(RS_ERR_INVALID_ARGUMENT, "ctx is NULL");
    if (n >= RS_MAX_ELEMENTS)
        return fail(RS_ERR_UNSUPPORTED, "n = %llu exceeds the limit of 2^30 - 1 elements",
                    (unsigned long long)n);
    *L = make_layout(key_bytes, has_values, n);
    if (n == 0)
        return RS_OK;
    if (!kin || !kout || (has_values && (!vin || !vout)))
        return fail(RS_ERR_INVALID_ARGUMENT, "NULL data pointer with n > 0");
    const uintptr_t al = (uintptr_t)key_bytes - 1;
    if (((uintptr_t)kin & al) || ((uintptr_t)kout & al) ||
        (has_values && (((uintptr_t)vin & al) || ((uintptr_t)vout & al))))
        return fail(RS_ERR_INVALID_ARGUMENT, "data pointers must be %d-byte aligned", key_bytes);
    const uint64_t bytes = n * (uint64_t)key_bytes;
    if (kin != kout && overlaps(kin, bytes, kout, bytes))
        return fail(RS_ERR_INVALID_ARGUMENT, "keys_in and keys_out partially overlap");
    if (has_values) {
        if (vin != vout && overlaps(vin, bytes, vout, bytes))
            return fail(RS_ERR_INVALID_ARGUMENT, "vals_in and vals_out partially overlap");
        if (overlaps(kin, bytes, vin, bytes) || overlaps(kin, bytes, vout, bytes) ||
            overlaps(kout, bytes, vin, bytes) || overlaps(kout, bytes, vout, bytes))
            return fail(RS_ERR_INVALID_ARGUMENT, "key and value arrays overlap");
    }
    if (ws) {
        if ((uintptr_t)ws & 255)
            return fail(RS_ERR_INVALID_ARGUMENT, "workspace must be 256-byte aligned");
        if (ws_bytes < L->total)
            return fail(RS_ERR_INVALID_ARGUMENT, "workspace of %zu bytes is below the %llu needed",
                        ws_bytes, (unsigned long long)L->total);
        if (overlaps(ws, L->total, kin, bytes) || overlaps(ws, L->total, kout, bytes) ||
            (has_values && (overlaps(ws, L->total, vin, bytes) || overlaps(ws, L->total, vout, bytes))))
            return fail(RS_ERR_INVALID_ARGUMENT, "workspace overlaps a data array");
    }
    return RS_OK;
}

template <typename K, bool HAS_V>
static const char *pass_name()
{
    if (sizeof(K) == 4)
        return HAS_V ? "k_pass_u32_pairs" : "k_pass_u32_keys";
    return HAS_V ? "k_pass_u64_pairs" : "k_pass_u64_keys";
}

template <typename K, bool HAS_V>
static rs_status run_sort(rs_context *ctx, const K *kin, const K *vin, K *kout, K *vout,
                          uint64_t n, void *ws, size_t ws_bytes, void *stream)
{
    Layout L;
    rs_status st = validate_sort(ctx, sizeof(K), kin, vin, kout, vout, HAS_V, n, ws, ws_bytes, &L);
    if (st != RS_OK || n == 0)
        return st;
    DeviceGuard guard(ctx->device);
    if (!guard.ok)
        return fail(RS_ERR_DEVICE, "cannot select HIP device %d", ctx->device);
    hipStream_t s = (hipStream_t)stream;
    using B = BlockShape<K, HAS_V>;
    if (n <= (uint64_t)B::kMediumCap) {
        // the whole array fits one workgroup's LDS: one launch, all passes
        BlockArgs ba{kin, vin, kout, vout, nullptr, nullptr, nullptr, n};
        if (n <= (uint64_t)B::kSmallCap) {
            launch(ctx, s, "k_block_sort_small", [&] {
                hipLaunchKernelGGL((k_block_sort<K, K, HAS_V, B::kSmallThreads, B::kItems>),
                                   dim3(1), dim3(B::kSmallThreads), 0, s, ba);
            });
        } else {
            launch(ctx, s, "k_block_sort_medium", [&] {
                hipLaunchKernelGGL((k_block_sort<K, K, HAS_V, B::kMediumThreads, B::kItems>),
                                   dim3(1), dim3(B::kMediumThreads), 0, s, ba);
            });
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return fail(RS_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
        return RS_OK;
    }
    void *w = nullptr;
    st = get_workspace(ctx, ws, ws_bytes, L.total, &w);
    if (st != RS_OK)
        return st;
    char *wb = (char *)w;
    uint32_t *ctrl = (uint32_t *)(wb + L.off_ctrl);
    uint32_t *hist = (uint32_t *)(wb + L.off_hist);
    uint32_t *base = (uint32_t *)(wb + L.off_base);
    uint32_t *status = (uint32_t *)(wb + L.off_status);
    // in-place if either array is: the first moving pass must not write its own input
    const bool in_place = (const void *)kin == (const void *)kout || (HAS_V && vin == vout);

    Bufs b{kin, vin, kout, vout, wb + L.off_tmp_k, HAS_V ? (void *)(wb + L.off_tmp_v) : nullptr};

    launch(ctx, s, "k_init", [&] {
        hipLaunchKernelGGL(k_init, dim3(1), dim3(256), 0, s, ctrl, hist, L.d * kRadix);
    });

    HistArgs ha{};
    ha.keys = kin;
    ha.n = (uint32_t)n;
    const uint64_t mis = ((uintptr_t)kin & 15) / sizeof(K);
    ha.head = (uint32_t)std::min<uint64_t>(n, mis ? (16 / sizeof(K)) - mis : 0);
    ha.nvec = (uint32_t)((n - ha.head) / (16 / sizeof(K)));
    ha.hist = hist;
    ha.status = (uint4 *)status;
    ha.status_vec = L.status_bytes / 16;
    const uint64_t hist_blocks = std::max<uint64_t>(
        1, std::min<uint64_t>(2048, (n + 16383) / 16384));
    launch(ctx, s, sizeof(K) == 4 ? "k_hist_u32" : "k_hist_u64", [&] {
        hipLaunchKernelGGL(k_hist<K>, dim3((uint32_t)hist_blocks), dim3(kHistThreads), 0, s, ha);
    });

    PlanArgs pl{hist, base, ctrl, (uint32_t)n, in_place};
    launch(ctx, s, "k_plan", [&] {
        hipLaunchKernelGGL(k_plan<KeyTraits<K>::kBits / kRadixBits>, dim3(1), dim3(kRadix), 0, s,
                           pl);
    });

    using S = PassShape<K, HAS_V>;
    // workgroups loop over claimed tiles: launch only what fits on the device
    // at once (more would start at the end just to find no work)
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_pass<K, K, HAS_V>, S::kThreads,
                                                     0) != hipSuccess ||
        per_cu < 1) {
        (void)hipGetLastError();
        per_cu = 1;
    }
    const uint32_t pass_grid =
        (uint32_t)std::min<uint64_t>(L.tiles, (uint64_t)per_cu * ctx_cus(ctx));
    for (int p = 0; p < L.d; ++p) {
        PassArgs pa{};
        pa.b = b;
        pa.n = (uint32_t)n;
        pa.pass = p;
        pa.shift = p * kRadixBits;
        pa.ctrl = ctrl;
        pa.digit_base = base + p * kRadix;
        pa.status = status + (uint64_t)p * L.tiles * kRadix;
        pa.claims = status + (uint64_t)L.d * L.tiles * kRadix + (uint64_t)p * L.claim_words;
        pa.num_tiles = (uint32_t)L.tiles;
        pa.num_groups = (uint32_t)((L.tiles + S::kGroup - 1) / S::kGroup);
        launch(ctx, s, pass_name<K, HAS_V>(), [&] {
            hipLaunchKernelGGL((k_pass<K, K, HAS_V>), dim3(pass_grid), dim3(S::kThreads),
                               0, s, pa);
        });
    }
    if (in_place) {
        const uint32_t blocks = (uint32_t)std::min<uint64_t>(4096, (n + 255) / 256);
        launch(ctx, s, "k_finalize", [&] {
            hipLaunchKernelGGL((k_finalize<K, K, HAS_V>), dim3(blocks), dim3(256), 0, s, b,
                               (uint32_t)n, (const uint32_t *)ctrl);
        });
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(RS_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return RS_OK;
}

// ---------------------------------------------------------------------------
// Segmented sort host side.

static constexpr uint64_t kSegMaxTotal = (uint64_t)1 << 36;

struct SegLayout {
    int d;
    uint64_t max_tiles;
    uint64_t claim_words;
    uint64_t max_chunks;
    uint64_t off_ctrl, off_small, off_medium, off_large, off_base, off_tile_seg, off_status,
        status_bytes, off_tmp_k, off_tmp_v, total;
    uint64_t off_hist, off_chunk_seg;
};

static SegLayout make_seg_layout(int key_bytes, bool has_values, uint64_t total, uint32_t nseg)
{
    SegLayout L{};
    L.d = key_bytes;
    const uint64_t T = key_bytes == 4 ? (has_values ? PassShape<uint32_t, true>::kTile
                                                    : PassShape<uint32_t, false>::kTile)
                                      : (has_values ? PassShape<uint64_t, true>::kTile
                                                    : PassShape<uint64_t, false>::kTile);
    // every large segment adds at most one partial tile
    L.max_tiles = total / T + nseg + 1;
    L.claim_words = 8 + 8 * L.max_tiles;
    uint64_t o = 0;
    L.off_ctrl = o;
    o = align_up(o + kSegWords * 4, 256);
    L.off_small = o;
    o = align_up(o + (uint64_t)nseg * sizeof(SegRange), 256);
    L.off_medium = o;
    o = align_up(o + (uint64_t)nseg * sizeof(SegRange), 256);
    L.off_large = o;
    o = align_up(o + (uint64_t)nseg * sizeof(SegLarge), 256);
    L.off_base = o;
    o = align_up(o + (uint64_t)nseg * L.d * kRadix * 4, 256);
    L.off_tile_seg = o;
    o = align_up(o + L.max_tiles * 4, 256);
    L.max_chunks = total / kSegChunk + nseg + 1;
    L.off_chunk_seg = o;
    o = align_up(o + L.max_chunks * 4, 256);
    // zeroed region: look-back words, claim counters, segment histograms
    L.off_status = o;
    L.status_bytes = align_up((uint64_t)L.d * (L.max_tiles * kRadix + L.claim_words) * 4, 16);
    L.off_hist = L.off_status + L.status_bytes;
    L.status_bytes += align_up((uint64_t)nseg * L.d * kRadix * 4, 16);
    o = align_up(o + L.status_bytes, 256);
    L.off_tmp_k = o;
    o = align_up(o + total * key_bytes, 256);
    L.off_tmp_v = o;
    o = align_up(o + (has_values ? total * key_bytes : 0), 256);
    L.total = o;
    return L;
}

template <typename K, bool HAS_V>
static rs_status run_segmented(rs_context *ctx, const void *kin, const void *vin, void *kout,
                               void *vout, const uint64_t *offsets, uint32_t nseg, uint64_t total,
                               void *ws, size_t ws_bytes, void *stream)
{
    if (!ctx)
        return fail(RS_ERR_INVALID_ARGUMENT, "ctx is NULL");
    if (total >= kSegMaxTotal)
        return fail(RS_ERR_UNSUPPORTED, "total exceeds 2^36 elements");
    if (HAS_V && (!vin || !vout))
        return fail(RS_ERR_INVALID_ARGUMENT, "values need both vals_in and vals_out");
    const SegLayout L = make_seg_layout(sizeof(K), HAS_V, total, nseg);
    if (nseg == 0 || total == 0)
        return RS_OK;
    if (!offsets)
        return fail(RS_ERR_INVALID_ARGUMENT, "offsets is NULL");
    if (!kin || !kout)
        return fail(RS_ERR_INVALID_ARGUMENT, "NULL data pointer with total > 0");
    const uintptr_t al = sizeof(K) - 1;
    if (((uintptr_t)kin & al) || ((uintptr_t)kout & al) || ((uintptr_t)offsets & 7) ||
        (HAS_V && (((uintptr_t)vin & al) || ((uintptr_t)vout & al))))
        return fail(RS_ERR_INVALID_ARGUMENT, "misaligned pointer");
    const uint64_t bytes = total * sizeof(K);
    if (kin != kout && overlaps(kin, bytes, kout, bytes))
        return fail(RS_ERR_INVALID_ARGUMENT, "keys_in and keys_out partially overlap");
    if (HAS_V) {
        if (vin != vout && overlaps(vin, bytes, vout, bytes))
            return fail(RS_ERR_INVALID_ARGUMENT, "vals_in and vals_out partially overlap");
        if (overlaps(kin, bytes, vin, bytes) || overlaps(kin, bytes, vout, bytes) ||
            overlaps(kout, bytes, vin, bytes) || overlaps(kout, bytes, vout, bytes))
            return fail(RS_ERR_INVALID_ARGUMENT, "key and value arrays overlap");
    }
    if (ws) {
        if ((uintptr_t)ws & 255)
            return fail(RS_ERR_INVALID_ARGUMENT, "workspace must be 256-byte aligned");
        if (ws_bytes < L.total)
            return fail(RS_ERR_INVALID_ARGUMENT, "workspace of %zu bytes is below the %llu needed",
                        ws_bytes, (unsigned long long)L.total);
        if (overlaps(ws, L.total, kin, bytes) || overlaps(ws, L.total, kout, bytes) ||
            (HAS_V && (overlaps(ws, L.total, vin, bytes) || overlaps(ws, L.total, vout, bytes))))
            return fail(RS_ERR_INVALID_ARGUMENT, "workspace overlaps a data array");
    }
    DeviceGuard guard(ctx->device);
    if (!guard.ok)
        return fail(RS_ERR_DEVICE, "cannot select HIP device %d", ctx->device);
    void *w = nullptr;
    rs_status st = get_workspace(ctx, ws, ws_bytes, L.total, &w);
    if (st != RS_OK)
        return st;
    hipStream_t s = (hipStream_t)stream;
    char *wb = (char *)w;
    uint32_t *ctrl = (uint32_t *)(wb + L.off_ctrl);
    SegRange *small_list = (SegRange *)(wb + L.off_small);
    SegRange *medium_list = (SegRange *)(wb + L.off_medium);
    SegLarge *large = (SegLarge *)(wb + L.off_large);
    uint32_t *seg_base = (uint32_t *)(wb + L.off_base);
    uint32_t *tile_seg = (uint32_t *)(wb + L.off_tile_seg);
    uint32_t *chunk_seg = (uint32_t *)(wb + L.off_chunk_seg);
    uint32_t *seg_hist = (uint32_t *)(wb + L.off_hist);
    uint32_t *status = (uint32_t *)(wb + L.off_status);
    void *tmp_k = wb + L.off_tmp_k;
    void *tmp_v = HAS_V ? (void *)(wb + L.off_tmp_v) : nullptr;
    using B = BlockShape<K, HAS_V>;
    using S = PassShape<K, HAS_V>;
    const uint32_t cus = ctx_cus(ctx);

    launch(ctx, s, "k_zero", [&] {
        hipLaunchKernelGGL(k_zero, dim3(1), dim3(256), 0, s, (uint4 *)ctrl,
                           (uint64_t)kSegWords * 4 / 16);
    });
    launch(ctx, s, "k_zero", [&] {
        const uint64_t nvec = L.status_bytes / 16;
        const uint32_t g = (uint32_t)std::min<uint64_t>(4096, (nvec + 255) / 256);
        hipLaunchKernelGGL(k_zero, dim3(std::max(1u, g)), dim3(256), 0, s, (uint4 *)status, nvec);
    });
    SegClassifyArgs ca{offsets, nseg, total, (uint32_t)L.max_tiles, ctrl, small_list, medium_list,
                       large, tile_seg, chunk_seg, (uint32_t)L.max_chunks, kin, vin, kout, vout,
                       (uint32_t)B::kSmallCap, (uint32_t)B::kMediumCap, (uint32_t)S::kTile};
    launch(ctx, s, "k_seg_classify", [&] {
        const uint32_t g = std::min<uint32_t>(1024, (nseg + 255) / 256);
        hipLaunchKernelGGL((k_seg_classify<K, HAS_V>), dim3(std::max(1u, g)), dim3(256), 0, s, ca);
    });
    // small and medium segments: persistent workgroups over the device lists
    auto grid_of = [&](const void *kernel, int threads) {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) !=
                hipSuccess ||
            per_cu < 1) {
            (void)hipGetLastError();
            per_cu = 1;
        }
        return (uint32_t)per_cu * cus;
    };
    {
        BlockArgs ba{kin, vin, kout, vout, small_list, ctrl + kSegSmallLen, ctrl + kSegSmallClaim,
                     0};
        auto kern = k_block_sort<K, K, HAS_V, B::kSmallThreads, B::kItems>;
        const uint32_t g = std::min<uint32_t>(grid_of((const void *)kern, B::kSmallThreads), nseg);
        launch(ctx, s, "k_block_sort_small", [&] {
            hipLaunchKernelGGL(kern, dim3(g), dim3(B::kSmallThreads), 0, s, ba);
        });
    }
    {
        BlockArgs ba{kin, vin, kout, vout, medium_list, ctrl + kSegMediumLen,
                     ctrl + kSegMediumClaim, 0};
        auto kern = k_block_sort<K, K, HAS_V, B::kMediumThreads, B::kItems>;
        const uint32_t g = std::min<uint32_t>(grid_of((const void *)kern, B::kMediumThreads), nseg);
        launch(ctx, s, "k_block_sort_medium", [&] {
            hipLaunchKernelGGL(kern, dim3(g), dim3(B::kMediumThreads), 0, s, ba);
        });
    }
    // large segments: per-segment histograms, then the batched digit passes,
    // in -> tmp -> out -> ... (an even number of passes ends in out)
    {
        SegHistArgs ha{kin, large, chunk_seg, (uint32_t)L.max_chunks, ctrl, seg_hist, seg_base};
        auto kern = k_seg_hist<K>;
        const uint32_t g = std::min<uint64_t>(grid_of((const void *)kern, 256), L.max_chunks);
        launch(ctx, s, "k_seg_hist", [&] { hipLaunchKernelGGL(kern, dim3(g), dim3(256), 0, s, ha); });
        auto scan = k_seg_scan<KeyTraits<K>::kBits / kRadixBits>;
        const uint32_t gs = std::min<uint32_t>(grid_of((const void *)scan, 256), nseg);
        launch(ctx, s, "k_seg_scan", [&] { hipLaunchKernelGGL(scan, dim3(gs), dim3(256), 0, s, ha); });
    }
    {
        auto kern = k_seg_pass<K, K, HAS_V>;
        const uint32_t g = grid_of((const void *)kern, S::kThreads);
        for (int p = 0; p < L.d; ++p) {
            SegPassArgs pa{};
            pa.src_k = p == 0 ? kin : ((p & 1) ? tmp_k : kout);
            pa.src_v = p == 0 ? vin : ((p & 1) ? tmp_v : vout);
            pa.dst_k = (p & 1) ? kout : tmp_k;
            pa.dst_v = (p & 1) ? vout : tmp_v;
            pa.large = large;
            pa.tile_seg = tile_seg;
            pa.seg_base = seg_base;
            pa.ctrl = ctrl;
            pa.status = status + (uint64_t)p * L.max_tiles * kRadix;
            pa.claims = status + (uint64_t)L.d * L.max_tiles * kRadix + (uint64_t)p * L.claim_words;
            pa.max_tiles = (uint32_t)L.max_tiles;
            pa.pass = p;
            pa.shift = p * kRadixBits;
            pa.d = L.d;
            launch(ctx, s, sizeof(K) == 4 ? "k_seg_pass_u32" : "k_seg_pass_u64", [&] {
                hipLaunchKernelGGL(kern, dim3(g), dim3(S::kThreads), 0, s, pa);
            });
        }
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(RS_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return RS_OK;
}

// ===========================================================================
// Exported C-ABI.

extern "C" {

rs_status rs_context_create(int device, rs_context **out)
{
    if (!out)
        return fail(RS_ERR_INVALID_ARGUMENT, "out is NULL");
    *out = nullptr;
    if (device < 0)
        return fail(RS_ERR_INVALID_ARGUMENT, "device must be >= 0");
    rs_context *c = new (std::nothrow) rs_context();
    if (c)
        c->device = device;
    if (!c)
        return fail(RS_ERR_OUT_OF_MEMORY, "cannot allocate a context");
    *out = c;
    return RS_OK;
}

void rs_context_destroy(rs_context *ctx)
{
    if (!ctx)
        return;
    if (ctx->own_ws || !ctx->events.empty()) {
        DeviceGuard g(ctx->device);
        if (ctx->own_ws)
            (void)hipFree(ctx->own_ws);
        for (hipEvent_t e : ctx->events)
            (void)hipEventDestroy(e);
    }
    delete ctx;
}

rs_status rs_profile_enable(rs_context *ctx, int enable)
{
    if (!ctx)
        return fail(RS_ERR_INVALID_ARGUMENT, "ctx is NULL");
    ctx->prof = enable != 0;
    return RS_OK;
}

rs_status rs_profile_tag(rs_context *ctx, int tag)
{
    if (!ctx)
        return fail(RS_ERR_INVALID_ARGUMENT, "ctx is NULL");
    ctx->prof_tag = tag;
    return RS_OK;
}

rs_status rs_profile_reset(rs_context *ctx)
{
    if (!ctx)
        return fail(RS_ERR_INVALID_ARGUMENT, "ctx is NULL");
    ctx->recs.clear();
    ctx->events_used = 0;
    return RS_OK;
}

rs_status rs_profile_read(rs_context *ctx, const char **names, int *tags, float *ms, int max,
                          int *count)
{
    if (!ctx || !count || max < 0 || (max > 0 && (!names || !tags || !ms)))
        return fail(RS_ERR_INVALID_ARGUMENT, "bad profile_read arguments");
    *count = (int)ctx->recs.size();
    if (ctx->recs.empty() || max == 0)
        return RS_OK;
    DeviceGuard g(ctx->device);
    if (!g.ok)
        return fail(RS_ERR_DEVICE, "cannot select HIP device %d", ctx->device);
    const int m = std::min<int>(max, (int)ctx->recs.size());
    for (int i = 0; i < m; ++i) {
        const ProfRecord &r = ctx->recs[i];
        if (hipEventSynchronize(ctx->events[r.ev + 1]) != hipSuccess)
            return fail(RS_ERR_DEVICE, "event synchronise failed");
        float t = 0.f;
        if (hipEventElapsedTime(&t, ctx->events[r.ev], ctx->events[r.ev + 1]) != hipSuccess)
            return fail(RS_ERR_DEVICE, "event elapsed time failed");
        names[i] = r.name;
        tags[i] = r.tag;
        ms[i] = t;
    }
    return RS_OK;
}

rs_status rs_workspace_bytes(const rs_context *ctx, rs_key_type key_type, int has_values,
                             uint64_t n, size_t *bytes)
{
    if (!ctx || !bytes)
        return fail(RS_ERR_INVALID_ARGUMENT, "ctx or bytes is NULL");
    if (key_type != RS_KEY_U32 && key_type != RS_KEY_U64)
        return fail(RS_ERR_INVALID_ARGUMENT, "unknown key type %d", (int)key_type);
    if (n >= RS_MAX_ELEMENTS)
        return fail(RS_ERR_UNSUPPORTED, "n exceeds the limit of 2^30 - 1 elements");
    *bytes = (size_t)make_layout(key_type == RS_KEY_U32 ? 4 : 8, has_values != 0, n).total;
    return RS_OK;
}

rs_status rs_sort_keys_u32(rs_context *ctx, const uint32_t *keys_in, uint32_t *keys_out,
                           uint64_t n, void *ws, size_t ws_bytes, void *stream)
{
    return run_sort<uint32_t, false>(ctx, keys_in, nullptr, keys_out, nullptr, n, ws, ws_bytes,
                                     stream);
}

rs_status rs_sort_keys_u64(rs_context *ctx, const uint64_t *keys_in, uint64_t *keys_out,
                           uint64_t n, void *ws, size_t ws_bytes, void *stream)
{
    return run_sort<uint64_t, false>(ctx, keys_in, nullptr, keys_out, nullptr, n, ws, ws_bytes,
                                     stream);
}

rs_status rs_sort_pairs_u32(rs_context *ctx, const uint32_t *keys_in, const uint32_t *vals_in,
                            uint32_t *keys_out, uint32_t *vals_out, uint64_t n, void *ws,
                            size_t ws_bytes, void *stream)
{
    return run_sort<uint32_t, true>(ctx, keys_in, vals_in, keys_out, vals_out, n, ws, ws_bytes,
                                    stream);
}

rs_status rs_sort_pairs_u64(rs_context *ctx, const uint64_t *keys_in, const uint64_t *vals_in,
                            uint64_t *keys_out, uint64_t *vals_out, uint64_t n, void *ws,
                            size_t ws_bytes, void *stream)
{
    return run_sort<uint64_t, true>(ctx, keys_in, vals_in, keys_out, vals_out, n, ws, ws_bytes,
                                    stream);
}

rs_status rs_segmented_workspace_bytes(const rs_context *ctx, rs_key_type key_type,
                                       int has_values, uint64_t total, uint32_t num_segments,
                                       size_t *bytes)
{
    if (!ctx || !bytes)
        return fail(RS_ERR_INVALID_ARGUMENT, "ctx or bytes is NULL");
    if (key_type != RS_KEY_U32 && key_type != RS_KEY_U64)
        return fail(RS_ERR_INVALID_ARGUMENT, "unknown key type %d", (int)key_type);
    if (total >= kSegMaxTotal)
        return fail(RS_ERR_UNSUPPORTED, "total exceeds 2^36 elements");
    *bytes = (size_t)make_seg_layout(key_type == RS_KEY_U32 ? 4 : 8, has_values != 0, total,
                                     num_segments)
                 .total;
    return RS_OK;
}

rs_status rs_segmented_sort(rs_context *ctx, rs_key_type key_type, const void *keys_in,
                            const void *vals_in, void *keys_out, void *vals_out,
                            const uint64_t *offsets, uint32_t num_segments, uint64_t total,
                            void *ws, size_t ws_bytes, void *stream)
{
    if (key_type == RS_KEY_U32) {
        if (vals_in || vals_out)
            return run_segmented<uint32_t, true>(ctx, keys_in, vals_in, keys_out, vals_out, offsets,
                                                 num_segments, total, ws, ws_bytes, stream);
        return run_segmented<uint32_t, false>(ctx, keys_in, vals_in, keys_out, vals_out, offsets,
                                              num_segments, total, ws, ws_bytes, stream);
    }
    if (key_type == RS_KEY_U64) {
        if (vals_in || vals_out)
            return run_segmented<uint64_t, true>(ctx, keys_in, vals_in, keys_out, vals_out, offsets,
                                                 num_segments, total, ws, ws_bytes, stream);
        return run_segmented<uint64_t, false>(ctx, keys_in, vals_in, keys_out, vals_out, offsets,
                                              num_segments, total, ws, ws_bytes, stream);
    }
    return fail(RS_ERR_INVALID_ARGUMENT, "unknown key type %d", (int)key_type);
}

const char *rs_status_string(rs_status status)
{
    switch (status) {
    case RS_OK: return "ok";
    case RS_ERR_INVALID_ARGUMENT: return "invalid argument";
    case RS_ERR_UNSUPPORTED: return "unsupported";
    case RS_ERR_OUT_OF_MEMORY: return "out of memory";
    case RS_ERR_DEVICE: return "device error";
    }
    return "unknown status";
}

const char *rs_last_error(void)
{
    return g_last_error.c_str();
}

}  // extern "C"
