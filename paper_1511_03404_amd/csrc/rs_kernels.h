// Digit-pass kernels of the LSD radix sort, templated on the configuration
// (digit width R, tile shape THREADS x ITEMS).
//
// Method (paper, Section 2.6): d = ceil(K/R) passes of R-bit digits, least
// significant first, each a stable counting sort.  The GPU realisation:
//
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
//   k_seg_hist / k_seg_scan / k_seg_pass
//              the same for the large segments of a segmented sort, every
//              segment with its own histograms and look-back chain.
#pragma once

#include <algorithm>

#include "rs_device.h"
#include "rs_segmented.h"

namespace rs {

// Consecutive tiles claimed as a group (see claim_tile).
constexpr int kClaimGroup = 8;

// One wave in kBallotShare ranks with ballots (see PassCfg::kBallotWaves).
constexpr int kBallotShare = 4;

// Configuration of the digit passes.
//   kLookback  predecessor tiles read per look-back round trip
//   kGroup     consecutive tiles claimed as a group (see claim_tile)
// Keys are staged in LDS, written out, then the values go through the same
// buffer; the per-wave lane-mask table is only live while ranking and shares
// it too.  Big tiles amortise the per-tile latencies (tile claim, look-back)
// and make the digit runs of the scatter longer.
template <int R, int THREADS, int ITEMS>
struct PassCfg {
    static_assert(R >= 4 && R <= 8, "digit widths of 4..8 bits");
    static_assert(THREADS % kWave == 0 && THREADS >= 256 && THREADS <= 1024, "256..1024 threads");
    static constexpr int kRadixBits = R;
    static constexpr int kBins = 1 << R;
    static constexpr int kThreads = THREADS;
    static constexpr int kItems = ITEMS;
    static constexpr int kTile = THREADS * ITEMS;
    static constexpr int kLookback = 8;
    static constexpr int kGroup = kClaimGroup;
    // waves that find their digit peers with ballots (VALU) instead of the
    // LDS lane-mask table: the two methods give the same masks, and splitting
    // the waves between them keeps both the VALU and the LDS busy
    static constexpr int kBallotWaves = THREADS / kWave / kBallotShare;
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
// k_hist: all-digit histograms in one read of the keys; also clears the
// look-back words of every pass.

struct HistArgs {
    const void *keys;
    uint32_t n;
    uint32_t head;        // leading keys before the first 16-byte boundary
    uint32_t nvec;        // 16-byte vectors after the head
    uint32_t *hist;       // [d][2^R]
    uint4 *status;        // look-back words of all passes, cleared here
    uint64_t status_vec;  // number of uint4 in status
};

// Count one key's D digits into the wave's LDS sub-histograms.
template <typename K, int R>
__device__ __forceinline__ void count_one(uint32_t (*sh)[1 << R], K key)
{
    constexpr int D = num_passes<K, R>();
#pragma unroll
    for (int p = 0; p < D; ++p)
        atomicAdd(&sh[p][digit_of<R>(key, p * R)], 1u);
}

// Count a batch of NK keys per thread (a full batch: every lane active).
// Key slot i of the wave covers 64 neighbouring vectors of the input, and in
// skewed inputs (zero, sorted, reverse) a digit position is often the same
// over the whole slot; same-address LDS atomics serialise (0.5 lanes/clock
// against ~6 for spread addresses), so such a slot adds 64 once.
template <typename K, int R, int NK>
__device__ __forceinline__ void count_batch(uint32_t (*sh)[1 << R], const K (&key)[NK])
{
    constexpr int D = num_passes<K, R>();
#pragma unroll
    for (int p = 0; p < D; ++p) {
#pragma unroll
        for (int i = 0; i < NK; ++i) {
            const uint32_t dg = digit_of<R>(key[i], p * R);
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

template <typename K, int R>
__global__ __launch_bounds__(kHistThreads) void k_hist(HistArgs a)
{
    constexpr int D = num_passes<K, R>();
    constexpr int NB = 1 << R;
    constexpr int W = kHistThreads / kWave;
    constexpr int KPV = 16 / (int)sizeof(K);  // keys per 16-byte vector
    constexpr int VPT = 16 / KPV;             // vectors per thread per batch
    constexpr int NK = VPT * KPV;             // 16 keys per thread per batch
    constexpr uint32_t BATCH = kHistThreads * VPT;
    __shared__ uint32_t sh[W][D][NB];

    const uint32_t t = threadIdx.x;
    const uint32_t w = t / kWave;
    for (int i = t; i < W * D * NB; i += kHistThreads)
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
        count_batch<K, R, NK>(sh[w], key);
    }
    // the rest: unaligned head, vectors after the last full batch, ragged
    // tail -- element by element, spread over the whole grid
    const uint64_t rest0 = (uint64_t)a.head + full_batches * BATCH * KPV;
    const uint64_t extra = a.head + (a.n - rest0);
    for (uint64_t i = gtid; i < extra; i += gstride) {
        const uint64_t idx = i < a.head ? i : rest0 + (i - a.head);
        count_one<K, R>(sh[w], keys[idx]);
    }
    __syncthreads();

    for (int i = t; i < D * NB; i += kHistThreads) {
        uint32_t s = 0;
#pragma unroll
        for (int ww = 0; ww < W; ++ww)
            s += (&sh[ww][0][0])[i];
        if (s)
            atomicAdd(&a.hist[i], s);
    }
}

// ---------------------------------------------------------------------------
// k_plan (one workgroup of 256 threads): digit_base = exclusive scan of each
// histogram row (the counting sort's starting offsets), and the plan of
// every pass.  A pass whose digit is the same for all n keys is the identity
// permutation and is skipped; the remaining passes alternate between the
// output and the scratch copy so that the last one lands in the output.

struct PlanArgs {
    const uint32_t *hist;
    uint32_t *digit_base;
    uint32_t *ctrl;
    uint32_t n;
    int in_place;
};

template <typename K, int R>
__global__ __launch_bounds__(kRadix) void k_plan(PlanArgs a)
{
    constexpr int D = num_passes<K, R>();
    constexpr int NB = 1 << R;
    __shared__ uint32_t s_tmp[8];
    __shared__ int s_trivial[D];
    __shared__ int s_skewed[D];
    __shared__ unsigned long long s_sq[kRadix / kWave];
    const uint32_t t = threadIdx.x;
    for (int p = 0; p < D; ++p) {
        const uint32_t c = t < (uint32_t)NB ? a.hist[p * NB + t] : 0u;
        const uint32_t ex = bins_exclusive_scan<NB>(c, s_tmp);
        if (t < (uint32_t)NB)
            a.digit_base[p * NB + t] = ex;
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
    uint32_t *status;            // [tiles][2^R] of this pass
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
// An XCD's opener takes its global id only after the XCD's previous group is
// open, so the tiles of one XCD's groups increase with its claim counter
// (two openers racing between their two atomics could otherwise give the
// later group the lower tiles).  Then a workgroup's claims are increasing
// tiles, an empty claim means no later claim of the XCD gets a tile, and the
// lowest unfinished tile is always held or next to be claimed by a running
// workgroup of its XCD (workgroups keep claiming until the groups run out):
// the look-back waits cannot depend on a workgroup that has not started,
// and claiming ahead cannot leave a higher tile waiting on a lower one that
// nobody will claim.
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
                uint32_t prev = 1;
                if (j > 0) {
                    while ((prev = __hip_atomic_load(&list[j - 1], __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT)) == 0)
                        __builtin_amdgcn_s_sleep(1);
                }
                if (prev == kNoTile) {
                    v = kNoTile;
                } else {
                    const uint32_t g = atomicAdd(ctr, 1u);
                    v = g < a.num_groups ? g + 1 : kNoTile;
                }
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

// Where one tile's elements are and where its digit runs go.
struct TileRef {
    uint64_t src_off;  // first element of the tile in the source arrays
    uint64_t dst_off;  // first element of the sequence its digit runs land in
    uint32_t valid;    // elements in the tile
    uint32_t limit;    // length of that sequence (destination indices are below it)
    uint32_t first;    // first tile of its look-back chain
    uint32_t seg;      // segment of a segmented sort (for its digit offsets)
};

// LDS of one digit pass.  Keys and values have staging buffers of their own;
// the per-wave lane-mask tables of the ranking live in the key buffer, which
// is free until the keys are staged.  Tiles are claimed two iterations ahead
// into two slots (iteration i's tile sits in slot i % 2).
template <typename K, typename C, bool HAS_V>
struct PassLds {
    static constexpr int W = C::kThreads / kWave;
    static constexpr size_t kStageBytes = (size_t)C::kTile * sizeof(K);
    static_assert((size_t)W * C::kBins * 8 <= kStageBytes,
                  "the lane-mask tables live in the staging buffer");
    uint32_t wcnt[W * C::kBins];  // per wave and digit: count, then base in tile
    uint32_t gbase[C::kBins];
    uint32_t tmp[8];
    uint32_t slot_tile[2];
    TileRef slot_ref[2];
    __attribute__((aligned(16))) unsigned char stage[kStageBytes];
    __attribute__((aligned(16))) unsigned char vstage[HAS_V ? kStageBytes : 16];

    // zero the counters and the lane-mask tables before a tile
    __device__ __forceinline__ void clear(uint32_t t)
    {
        for (int i = t; i < W * C::kBins; i += C::kThreads) {
            wcnt[i] = 0;
            ((uint64_t *)stage)[i] = 0;
        }
    }
};

// The thread that claims tiles during the look-back: one of a wave with no
// digit bin (such waves are idle then), else thread 0.
template <typename C>
constexpr uint32_t claim_thread()
{
    return C::kThreads - kWave >= C::kBins ? C::kThreads - kWave : 0;
}

__device__ __forceinline__ uint32_t uniform(uint32_t v)
{
    return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ uint64_t uniform64(uint64_t v)
{
    return ((uint64_t)uniform((uint32_t)(v >> 32)) << 32) | uniform((uint32_t)v);
}

// One digit pass over claimed tiles (the paper's counting sort, Section 2.6,
// spread over workgroups).  Per tile: rank every element among its wave's
// elements of the same digit, publish the tile's digit counts, stage keys
// and values in LDS in digit order (tile-local offsets), then -- while the
// next tile's loads are in flight -- the decoupled look-back over the
// earlier tiles of the chain gives the tile's global offsets, and each digit
// run is written with consecutive lanes on consecutive addresses.
//
// Res maps a tile to its TileRef (resolve) and gives a digit's starting
// offset (dbase); the claim thread resolves a tile when it claims it, two
// iterations before its use, so no iteration waits on that lookup.
template <typename K, typename V, bool HAS_V, typename C, typename Res>
__device__ __forceinline__ void run_pass(PassLds<K, C, HAS_V> &L, const PassArgs &claim,
                                         const Res &res, const K *sk, const V *sv, K *dk, V *dv,
                                         uint32_t *status, int shift, bool ballot_rank)
{
    constexpr int R = C::kRadixBits;
    constexpr uint32_t NB = C::kBins;
    constexpr int THREADS = C::kThreads;
    constexpr int ITEMS = C::kItems;
    constexpr int T = C::kTile;
    constexpr int W = THREADS / kWave;
    constexpr int LBW = C::kLookback;
    static_assert(sizeof(V) == sizeof(K), "values have the key's width");
    K *s_k = (K *)L.stage;
    V *s_v = (V *)L.vstage;
    uint64_t *s_mask = (uint64_t *)L.stage;
    const uint32_t t = threadIdx.x;
    const uint32_t w = t / kWave;
    const uint32_t lane = t % kWave;
    const uint32_t off0 = w * (kWave * ITEMS) + lane;
    uint32_t *wc = L.wcnt + w * NB;

    // the first two tiles
    if (t == 0) {
        const uint32_t x = xcc_id();
#pragma unroll
        for (int sl = 0; sl < 2; ++sl) {
            const uint32_t tl = claim_tile<C::kGroup>(claim, x);
            L.slot_tile[sl] = tl;
            if (tl != kNoTile)
                L.slot_ref[sl] = res.resolve(tl);
        }
    }
    L.clear(t);
    __syncthreads();
    uint32_t tile = uniform(L.slot_tile[0]);
    if (tile == kNoTile)
        return;
    TileRef cur = L.slot_ref[0];
    K key[ITEMS];
    V val[HAS_V ? ITEMS : 1];
    load_tile<K, V, HAS_V, ITEMS>(sk + uniform64(cur.src_off), HAS_V ? sv + uniform64(cur.src_off) : nullptr,
                                  uniform(cur.valid), off0, key, val, uniform(cur.valid) == (uint32_t)T);
    uint32_t dbase = t < NB ? res.dbase(cur, t) : 0u;

    for (uint32_t it = 0;; ++it) {
        // count: stable rank of every item among the wave's items of its digit
        uint32_t rank[ITEMS];
        if (ballot_rank || w < (uint32_t)C::kBallotWaves)
            wave_rank_ballot<R, K, ITEMS>(key, shift, wc, rank);
        else
            wave_rank<R, K, ITEMS>(key, shift, wc, s_mask + w * NB, lane, rank);
        __syncthreads();

        // scan: wave offsets per digit, tile count, publish the aggregate,
        // tile-local offsets
        const uint32_t first = uniform(cur.first);
        uint32_t cnt = 0;
        if (t < NB) {
#pragma unroll
            for (int ww = 0; ww < W; ++ww) {
                const uint32_t c = L.wcnt[ww * NB + t];
                L.wcnt[ww * NB + t] = cnt;
                cnt += c;
            }
            __hip_atomic_store(&status[(uint64_t)tile * NB + t],
                               (tile == first ? kFlagInc : kFlagAgg) | cnt, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        const uint32_t excl = bins_exclusive_scan<NB>(cnt, L.tmp);
        if (t < NB) {
#pragma unroll
            for (int ww = 0; ww < W; ++ww)
                L.wcnt[ww * NB + t] += excl;
        }
        __syncthreads();

        // stage keys and values in digit order (the tile-local offsets do
        // not wait for the look-back)
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t pos = rank[j] + wc[digit_of<R>(key[j], shift)];
            s_k[pos] = key[j];
            if constexpr (HAS_V)
                s_v[pos] = val[j];
        }

        // the next tile (claimed two iterations ago): its loads fly during
        // the look-back and the writes of this tile
        const uint32_t ns = (it + 1) & 1;
        const uint32_t next = uniform(L.slot_tile[ns]);
        TileRef nref{};
        uint32_t ndbase = 0;
        if (next != kNoTile) {
            nref = L.slot_ref[ns];
            const uint64_t so = uniform64(nref.src_off);
            const uint32_t nv = uniform(nref.valid);
            load_tile<K, V, HAS_V, ITEMS>(sk + so, HAS_V ? sv + so : nullptr, nv, off0, key, val,
                                          nv == (uint32_t)T);
            ndbase = t < NB ? res.dbase(nref, t) : 0u;
        }
        // the tile after it, into the slot this iteration's tile came from
        if (t == claim_thread<C>()) {
            const uint32_t tl = claim_tile<C::kGroup>(claim, xcc_id());
            L.slot_tile[it & 1] = tl;
            if (tl != kNoTile)
                L.slot_ref[it & 1] = res.resolve(tl);
        }

        if (t < NB) {
            // decoupled look-back: read LBW predecessors per round trip, add
            // their counts in order up to the first inclusive one; on a tile
            // that has not published yet, wait and re-read from there
            uint32_t prefix = 0;
            int64_t k = (int64_t)tile - 1;
            const int64_t lo = first;
            while (k >= lo) {
                uint32_t st[LBW];
#pragma unroll
                for (int i = 0; i < LBW; ++i)
                    st[i] = (k - i >= lo)
                                ? __hip_atomic_load(&status[(uint64_t)(k - i) * NB + t],
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
            if (tile != first)
                __hip_atomic_store(&status[(uint64_t)tile * NB + t], kFlagInc | (prefix + cnt),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            L.gbase[t] = dbase + prefix - excl;
        }
        __syncthreads();

        // place: each digit run with consecutive lanes on consecutive addresses
        {
            const uint64_t doff = uniform64(cur.dst_off);
            const uint32_t limit = uniform(cur.limit);
            K *dkt = dk + doff;
            V *dvt = HAS_V ? dv + doff : nullptr;
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const uint32_t pos = i * THREADS + t;
                const K k = s_k[pos];
                const uint32_t dst = L.gbase[digit_of<R>(k, shift)] + pos;
                if (dst < limit) {
                    store_at(dkt, dst, k);
                    if constexpr (HAS_V)
                        store_at(dvt, dst, s_v[pos]);
                }
            }
        }
        __syncthreads();  // the staging buffers are reused by the next tile
        if (next == kNoTile)
            break;
        L.clear(t);
        __syncthreads();
        tile = next;
        cur = nref;
        dbase = ndbase;
    }
}

// Tiles of a plain sort: tile i holds elements [i*T, min((i+1)*T, n)).
struct PlainTiles {
    uint32_t n;
    uint32_t tile_elems;
    const uint32_t *digit_base;  // row of this pass
    __device__ TileRef resolve(uint32_t tile) const
    {
        const uint64_t lo = (uint64_t)tile * tile_elems;
        return TileRef{lo, 0, (uint32_t)std::min<uint64_t>(tile_elems, n - lo), n, 0, 0};
    }
    __device__ uint32_t dbase(const TileRef &, uint32_t t) const { return digit_base[t]; }
};

template <typename K, typename V, bool HAS_V, typename C>
__global__ __launch_bounds__(C::kThreads) void k_pass(PassArgs a)
{
    constexpr int THREADS = C::kThreads;
    constexpr int T = C::kTile;
    __shared__ PassLds<K, C, HAS_V> L;

    const uint32_t t = threadIdx.x;
    const uint32_t plan = a.ctrl[kCtrlPlan + a.pass];
    if (!(plan & kPlanRun)) {
        if (plan & kPlanCopyIn) {
            // no pass moves data: copy in -> out
            for (uint64_t tl = blockIdx.x; tl < a.num_tiles; tl += gridDim.x) {
                const uint64_t lo = tl * T;
                const uint64_t hi = std::min<uint64_t>(lo + T, a.n);
                copy_range(pick<const K>(a.b, kBufIn, false), pick<K>(a.b, kBufOut, false), lo,
                           hi, t, THREADS);
                if constexpr (HAS_V)
                    copy_range(pick<const V>(a.b, kBufIn, true), pick<V>(a.b, kBufOut, true), lo,
                               hi, t, THREADS);
            }
        }
        return;
    }
    const uint32_t src = (plan >> kPlanSrcShift) & 3u;
    const uint32_t dstb = (plan >> kPlanDstShift) & 3u;
    const PlainTiles res{a.n, (uint32_t)T, a.digit_base};
    run_pass<K, V, HAS_V, C>(L, a, res, pick<const K>(a.b, src, false),
                             HAS_V ? pick<const V>(a.b, src, true) : nullptr,
                             pick<K>(a.b, dstb, false), HAS_V ? pick<V>(a.b, dstb, true) : nullptr,
                             a.status, a.shift, (plan & kPlanBallot) != 0);
}

// ---------------------------------------------------------------------------
// Segmented sort: digit histograms of the large segments, chunk by chunk.
// Persistent workgroups claim chunks of kSegChunk elements, count all digit
// positions in LDS and add the counts to the segment's histogram (global
// atomics).

struct SegHistArgs {
    const void *kin;
    const SegLarge *large;
    const uint32_t *chunk_seg;
    uint32_t max_chunks;
    uint32_t *ctrl;
    uint32_t *seg_hist;  // [large segment][d][2^R], zeroed
    uint32_t *seg_base;  // [large segment][d][2^R]
};

template <typename K, int R>
__global__ __launch_bounds__(256) void k_seg_hist(SegHistArgs a)
{
    constexpr int D = num_passes<K, R>();
    constexpr int NB = 1 << R;
    constexpr int W = 256 / kWave;
    __shared__ uint32_t sh[W][D][NB];
    __shared__ uint32_t s_item;
    const uint32_t t = threadIdx.x;
    const uint32_t w = t / kWave;
    const K *keys = (const K *)a.kin;
    const uint32_t chunks = min(a.ctrl[kSegChunks], a.max_chunks);
    while (true) {
        if (t == 0)
            s_item = atomicAdd(&a.ctrl[kSegChunkClaim], 1u);
        for (int i = t; i < W * D * NB; i += 256)
            (&sh[0][0][0])[i] = 0;
        __syncthreads();
        const uint32_t item = s_item;
        if (item >= chunks)
            break;
        const uint32_t seg = a.chunk_seg[item];
        const SegLarge rec = a.large[seg];
        // this chunk's index within its segment: chunks of a segment are
        // consecutive, so count back to the segment's first chunk
        uint32_t first = item;
        while (first > 0 && a.chunk_seg[first - 1] == seg)
            --first;
        const uint64_t lo = (uint64_t)(item - first) * kSegChunk;
        const uint32_t len = rec.size > lo ? (uint32_t)min<uint64_t>(kSegChunk, rec.size - lo) : 0u;
        const K *sk = keys + rec.start + lo;
        for (uint32_t i = t; i < len; i += 256) {
            const K key = sk[i];
            const uint64_t active = __ballot(1);  // before any branch narrows it
#pragma unroll
            for (int p = 0; p < D; ++p) {
                const uint32_t dg = digit_of<R>(key, p * R);
                // a digit held by the whole wave is added once (same-address
                // LDS atomics serialise)
                const uint32_t first_dg = __builtin_amdgcn_readfirstlane(dg);
                if (__ballot(dg != first_dg) == 0) {
                    if (lane_id() == (uint32_t)__builtin_ctzll(active))
                        atomicAdd(&sh[w][p][first_dg], (uint32_t)__popcll(active));
                } else {
                    atomicAdd(&sh[w][p][dg], 1u);
                }
            }
        }
        __syncthreads();
        uint32_t *out = a.seg_hist + (uint64_t)seg * D * NB;
        for (int i = t; i < D * NB; i += 256) {
            uint32_t c = 0;
#pragma unroll
            for (int ww = 0; ww < W; ++ww)
                c += (&sh[ww][0][0])[i];
            if (c)
                atomicAdd(&out[i], c);
        }
        __syncthreads();
    }
}

// seg_base[seg][p] = exclusive scan of seg_hist[seg][p], one workgroup per
// large segment (persistent).
template <typename K, int R>
__global__ __launch_bounds__(256) void k_seg_scan(SegHistArgs a)
{
    constexpr int D = num_passes<K, R>();
    constexpr int NB = 1 << R;
    __shared__ uint32_t s_tmp[8];
    __shared__ uint32_t s_item;
    const uint32_t t = threadIdx.x;
    while (true) {
        if (t == 0)
            s_item = atomicAdd(&a.ctrl[kSegScanClaim], 1u);
        __syncthreads();
        const uint32_t item = s_item;
        if (item >= a.ctrl[kSegLargeLen])
            break;
        for (int p = 0; p < D; ++p) {
            const uint64_t i = ((uint64_t)item * D + p) * NB + t;
            const uint32_t c = t < (uint32_t)NB ? a.seg_hist[i] : 0u;
            const uint32_t ex = bins_exclusive_scan<NB>(c, s_tmp);
            if (t < (uint32_t)NB)
                a.seg_base[i] = ex;
        }
        __syncthreads();
    }
}

// k_seg_pass: one digit pass over the tiles of every large segment.  Each
// segment's tiles are consecutive in the batched tile sequence and its
// look-back chain starts at its first tile.

struct SegPassArgs {
    const void *src_k;
    const void *src_v;
    void *dst_k;
    void *dst_v;
    const SegLarge *large;
    const uint32_t *tile_seg;
    const uint32_t *seg_base;  // [large segment][d][2^R]
    uint32_t *ctrl;            // segmented control block
    uint32_t *status;          // look-back words of this pass
    uint32_t *claims;          // claim counters of this pass
    uint32_t max_tiles;        // tiles the workspace holds
    int pass;
    int shift;
    int d;
};

// Tiles of the large segments: tile i is tile i - tile_start of its segment.
struct SegTiles {
    const SegLarge *large;
    const uint32_t *tile_seg;
    const uint32_t *seg_base;  // [large segment][d][2^R]
    uint32_t tile_elems;
    uint32_t pass;
    uint32_t d;
    uint32_t bins;
    __device__ TileRef resolve(uint32_t tile) const
    {
        const uint32_t seg = tile_seg[tile];
        const SegLarge rec = large[seg];
        const uint32_t lt = tile - rec.tile_start;
        const uint32_t lo = lt * tile_elems;
        const uint32_t valid = rec.size > lo ? std::min<uint32_t>(tile_elems, rec.size - lo) : 0u;
        return TileRef{rec.start + lo, rec.start, valid, rec.size, rec.tile_start, seg};
    }
    __device__ uint32_t dbase(const TileRef &r, uint32_t t) const
    {
        return seg_base[((uint64_t)r.seg * d + pass) * bins + t];
    }
};

template <typename K, typename V, bool HAS_V, typename C>
__global__ __launch_bounds__(C::kThreads) void k_seg_pass(SegPassArgs a)
{
    __shared__ PassLds<K, C, HAS_V> L;
    PassArgs pa{};
    pa.ctrl = a.ctrl + (kSegPassCounter - kCtrlTileCounter);
    pa.pass = a.pass;
    pa.claims = a.claims;
    pa.num_tiles = std::min(a.ctrl[kSegTiles], a.max_tiles);
    pa.num_groups = (pa.num_tiles + C::kGroup - 1) / C::kGroup;
    const SegTiles res{a.large,        a.tile_seg,         a.seg_base,      (uint32_t)C::kTile,
                       (uint32_t)a.pass, (uint32_t)a.d, (uint32_t)C::kBins};
    run_pass<K, V, HAS_V, C>(L, pa, res, (const K *)a.src_k, (const V *)a.src_v, (K *)a.dst_k,
                             (V *)a.dst_v, a.status, a.shift, false);
}

// In-place segmented sort with an odd number of passes: the large segments
// end in the scratch copy; copy them back, tile by tile.
struct SegCopyArgs {
    const void *src_k;
    const void *src_v;
    void *dst_k;
    void *dst_v;
    const SegLarge *large;
    const uint32_t *tile_seg;
    const uint32_t *ctrl;  // segmented control block
    uint32_t max_tiles;
    uint32_t tile;  // elements per tile
};

template <typename K, bool HAS_V>
__global__ __launch_bounds__(256) void k_seg_copy(SegCopyArgs a)
{
    const uint32_t tiles = std::min(a.ctrl[kSegTiles], a.max_tiles);
    for (uint32_t tl = blockIdx.x; tl < tiles; tl += gridDim.x) {
        const SegLarge rec = a.large[a.tile_seg[tl]];
        const uint64_t lo = (uint64_t)(tl - rec.tile_start) * a.tile;
        if (lo >= rec.size)
            continue;
        const uint64_t hi = std::min<uint64_t>(lo + a.tile, rec.size);
        copy_range((const K *)a.src_k + rec.start, (K *)a.dst_k + rec.start, lo, hi, threadIdx.x,
                   256);
        if constexpr (HAS_V)
            copy_range((const K *)a.src_v + rec.start, (K *)a.dst_v + rec.start, lo, hi,
                       threadIdx.x, 256);
    }
}

}  // namespace rs
