// Digit-pass kernels of the LSD radix sort, templated on the configuration
// (digit width R, tile shape THREADS x ITEMS).
//
// Method (paper, Section 2.6): d = ceil(K/R) passes of R-bit digits, least
// significant first, each a stable counting sort.  The GPU realisation:
//
//   k_hist     one read of the keys -> histograms of all d digit positions
//              (added into one histogram, or for small sorts one row block
//              per workgroup); also clears the look-back words of every pass
//   k_plan     one workgroup: sums the row blocks if any, scans each
//              histogram row into digit_base (the counting sort's exclusive
//              prefix sums) and writes a plan: which passes move data (a pass
//              whose histogram has a single non-empty digit is the identity
//              and is skipped) and which buffer each pass reads and writes
//   k_pass     one per digit position: a single sweep over the data that
//              counts, scans (decoupled look-back across tiles) and places
//              each tile; see rs_device.h.
//   k_seg_hist / k_seg_scan / k_seg_pass
//              the same for the large segments of a segmented sort, every
//              segment with its own histograms and look-back chain.
#pragma once

#include <algorithm>
#include <cstddef>

#include "rs_device.h"
#include "rs_segmented.h"

namespace rs {

// Consecutive tiles claimed as a group (see claim_tile).
constexpr int kClaimGroup = 8;
// Passes of at most this many tiles claim them in arrival order (see
// claim_tile; measured on MI355X: faster or equal up to 1024 tiles on every
// kind, 2^24 keys of 16384-key tiles).
constexpr uint32_t kFlatClaimTiles = 1024;

// Per-XCD claim counters (XCC_ID has 3 bits; gfx950 has 8 XCDs).
constexpr uint32_t kXcdSlots = 8;

// One wave in kBallotShare ranks with ballots (see PassCfg::kBallotWaves).
constexpr int kBallotShare = 4;

// Configuration of the digit passes.
//   kLookback  predecessor tiles read per look-back round trip
//   kGroup     consecutive tiles claimed as a group (see claim_tile)
// The tile is staged in LDS in rank order (pairs as one (key, value) word
// per element) and written out after one barrier; the per-wave lane-mask
// tables are only live while ranking and share the staging memory.  Big
// tiles amortise the per-tile latencies (tile claim, look-back) and make
// the digit runs of the scatter longer.
template <int R, int THREADS, int ITEMS>
struct PassCfg {
    static_assert(R >= 4 && R <= 11, "digit widths of 4..11 bits");
    static_assert(THREADS % kWave == 0 && THREADS >= 256 && THREADS <= 1024, "256..1024 threads");
    static_assert(R <= 8 || THREADS == 1024, "wide digits use 1024-thread tiles");
    // digits of more than 8 bits take the wide layout (rs_wide.h)
    static constexpr bool kWide = R > 8;
    static constexpr int kRadixBits = R;
    static constexpr int kBins = 1 << R;
    static constexpr int kThreads = THREADS;
    static constexpr int kItems = ITEMS;
    static constexpr int kTile = THREADS * ITEMS;
    static constexpr int kLookback = 4;  // predecessors read per look-back round trip
    static constexpr int kGroup = kClaimGroup;
    // waves that find their digit peers with ballots (VALU) instead of the
    // LDS lane-mask table: the two methods give the same masks, and splitting
    // the waves between them keeps both the VALU and the LDS busy
    static constexpr int kBallotWaves = THREADS / kWave / kBallotShare;
};

constexpr int kHistThreads = 1024;

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
    uint32_t *hist;       // [d][2^R], accumulated with atomics (cleared before)
    uint32_t *part;       // or, when not null: [grid][d][2^R], one row block per
                          // workgroup, plain stores (nothing to clear first)
    uint4 *status;        // look-back words of all passes, cleared here
    uint64_t status_vec;  // number of uint4 in status
    uint32_t kmap;        // key order (kMap*), applied to every key read
    uint32_t fine;        // small sorts: up to 16 keys per thread, key by key,
                          // instead of batches (n <= 16 * grid * kHistThreads)
};

// Counters of k_hist: per digit position and per bin, kHistCols columns of
// 32-bit counters, column = lane % kHistCols.  Only the kWave / kHistCols
// lanes of a column can meet on one word, so a digit shared by the whole
// wave (zero, sorted or reverse keys) serialises kWave / kHistCols ways, not
// kWave; spread digits mostly land in different banks.
constexpr int kHistCols = 16;

// Columns per bin for D digit positions of R bits: 16 up to 8-bit digits;
// wide digits have 8x the bins, so fewer columns keep the table within
// 96 KB (4 for 32-bit keys at 11 bits, 2 for 64-bit keys).
template <int D, int R>
constexpr int hist_cols()
{
    if (R <= 8)
        return kHistCols;
    return (size_t)D * (1u << R) * 4 * 4 <= 96 * 1024 ? 4 : 2;
}

template <int R, int COLS = kHistCols>
__device__ __forceinline__ void hist_add(uint32_t *tab, int p, uint32_t dg, uint32_t col)
{
    atomicAdd(&tab[(((uint32_t)p << R) + dg) * COLS + col], 1u);
}

// Adds the counters into hist ([d][2^R]).  Row r (position r >> R, bin
// r % 2^R) is summed by one thread, which starts at column r so that
// neighbouring threads read different banks.
template <int D, int R, int COLS = kHistCols>
__device__ __forceinline__ void hist_flush(const uint32_t *tab, uint32_t *hist, uint32_t t)
{
    for (uint32_t r = t; r < (uint32_t)D << R; r += kHistThreads) {
        uint32_t s = 0;
#pragma unroll
        for (uint32_t c = 0; c < COLS; ++c)
            s += tab[r * COLS + ((c + r) & (COLS - 1))];
        if (s)
            atomicAdd(&hist[r], s);
    }
}

// Stores this workgroup's counters as its own row block of part ([d][2^R]),
// zero rows included.
template <int D, int R, int COLS = kHistCols>
__device__ __forceinline__ void hist_store(const uint32_t *tab, uint32_t *part, uint32_t t)
{
    for (uint32_t r = t; r < (uint32_t)D << R; r += kHistThreads) {
        uint32_t s = 0;
#pragma unroll
        for (uint32_t c = 0; c < COLS; ++c)
            s += tab[r * COLS + ((c + r) & (COLS - 1))];
        part[r] = s;
    }
}

// Up to this many k_hist workgroups (small sorts) write row blocks that
// k_plan sums, instead of adding into a histogram cleared by a launch of its
// own; beyond it the sum would cost k_plan more than that launch.
constexpr uint32_t kHistPartsMax = 16;

template <typename K, int R>
__global__ __launch_bounds__(kHistThreads) void k_hist(HistArgs a)
{
    constexpr int D = num_passes<K, R>();
    constexpr int KPV = 16 / (int)sizeof(K);  // keys per 16-byte vector
    constexpr int VPT = 16 / KPV;             // vectors per thread per batch
    constexpr int NK = VPT * KPV;             // 16 keys per thread per batch
    constexpr uint32_t BATCH = kHistThreads * VPT;
    constexpr int COLS = hist_cols<D, R>();
    constexpr uint32_t TAB = (D << R) * COLS;
    __shared__ uint32_t tab[TAB];

    const uint32_t t = threadIdx.x;
    const uint32_t col = t % COLS;
    for (uint32_t i = t; i < TAB; i += kHistThreads)
        tab[i] = 0;

    // clear the look-back words of every pass
    const uint64_t gtid = (uint64_t)blockIdx.x * kHistThreads + t;
    const uint64_t gstride = (uint64_t)gridDim.x * kHistThreads;
    for (uint64_t i = gtid; i < a.status_vec; i += gstride)
        a.status[i] = make_uint4(0, 0, 0, 0);
    __syncthreads();

    const K *keys = (const K *)a.keys;
    if (a.fine) {
        // all of the thread's loads in flight before its first count
        constexpr int FK = 16;
        K key[FK];
#pragma unroll
        for (int j = 0; j < FK; ++j) {
            const uint64_t idx = gtid + (uint64_t)j * gstride;
            key[j] = idx < a.n ? keys[idx] : (K)0;
        }
#pragma unroll
        for (int j = 0; j < FK; ++j) {
            if (gtid + (uint64_t)j * gstride < a.n) {
                const K k = map_in(key[j], a.kmap);
#pragma unroll
                for (int p = 0; p < D; ++p)
                    hist_add<R, COLS>(tab, p, digit_of<R>(k, p * R), col);
            }
        }
        __syncthreads();
        if (a.part)
            hist_store<D, R, COLS>(tab, a.part + (uint64_t)blockIdx.x * ((uint32_t)D << R), t);
        else
            hist_flush<D, R, COLS>(tab, a.hist, t);
        return;
    }
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
        if (a.kmap) {
#pragma unroll
            for (int i = 0; i < NK; ++i)
                key[i] = map_in(key[i], a.kmap);
        }
#pragma unroll
        for (int p = 0; p < D; ++p) {
#pragma unroll
            for (int i = 0; i < NK; ++i)
                hist_add<R, COLS>(tab, p, digit_of<R>(key[i], p * R), col);
        }
    }
    // the rest: unaligned head, vectors after the last full batch, ragged
    // tail -- element by element, spread over the whole grid
    const uint64_t rest0 = (uint64_t)a.head + full_batches * BATCH * KPV;
    const uint64_t extra = a.head + (a.n - rest0);
    for (uint64_t i = gtid; i < extra; i += gstride) {
        const uint64_t idx = i < a.head ? i : rest0 + (i - a.head);
        const K key = map_in(keys[idx], a.kmap);
#pragma unroll
        for (int p = 0; p < D; ++p)
            hist_add<R, COLS>(tab, p, digit_of<R>(key, p * R), col);
    }
    __syncthreads();
    if (a.part)
        hist_store<D, R, COLS>(tab, a.part + (uint64_t)blockIdx.x * ((uint32_t)D << R), t);
    else
        hist_flush<D, R, COLS>(tab, a.hist, t);
}

// ---------------------------------------------------------------------------
// k_plan (one workgroup, 256 threads per row group): digit_base = exclusive scan of each
// histogram row (the counting sort's starting offsets), and the plan of
// every pass.  A pass whose digit is the same for all n keys is the identity
// permutation and is skipped; the remaining passes alternate between the
// output and the scratch copy so that the last one lands in the output.

struct PlanArgs {
    uint32_t *hist;         // [d][2^R]: read; or written, as the sum of part
    const uint32_t *part;   // k_hist's row blocks ([parts][d][2^R]) when parts > 0
    uint32_t parts;
    uint32_t *digit_base;
    uint32_t *ctrl;
    uint32_t n;
    int keys_in_place;  // keys_out == keys_in
    int vals_in_place;  // pairs with vals_out == vals_in (0 for keys only)
    int limit;          // digit positions [0, limit) are sorted (the whole key: d)
};

// Rows are scanned side by side: row group g (threads [256 g, 256 g + 256))
// takes rows g, g + G, g + 2 G, ... (G = plan_groups row groups); a group's
// 256 threads hold up to 256 bins one each, wide digits several consecutive
// bins per thread.
template <typename K, int R>
constexpr int plan_groups()
{
    return num_passes<K, R>() < 4 ? num_passes<K, R>() : 4;
}

template <typename K, int R>
__global__ __launch_bounds__(kRadix * 4) void k_plan(PlanArgs a)
{
    constexpr int D = num_passes<K, R>();
    constexpr int NB = 1 << R;
    constexpr int G = plan_groups<K, R>();
    constexpr int ROUNDS = (D + G - 1) / G;
    constexpr int BPT = NB > kRadix ? NB / kRadix : 1;
    constexpr int WPG = kRadix / kWave;  // waves per group
    __shared__ uint32_t s_tot[G][WPG];
    __shared__ unsigned long long s_sq[G][WPG];
    __shared__ int s_trivial[D];
    __shared__ int s_skewed[D];
    const uint32_t t = threadIdx.x;
    const uint32_t g = t / kRadix;
    const uint32_t lt = t % kRadix;
    const uint32_t w = lt / kWave;
    const bool active = lt * BPT < (uint32_t)NB;
    if (t < (uint32_t)D)
        s_trivial[t] = 0;
    // the control block starts cleared (claim counters, error word); the
    // plan words are written at the end, after barriers
    for (uint32_t i = t; i < (uint32_t)kCtrlWords; i += blockDim.x)
        a.ctrl[i] = 0;
    // every row's load in flight at once, not one latency per digit position
    uint32_t cnt[ROUNDS][BPT];
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        const int p = r * G + (int)g;
#pragma unroll
        for (int i = 0; i < BPT; ++i)
            cnt[r][i] = (active && p < D && !a.parts) ? a.hist[p * NB + lt * BPT + i] : 0u;
    }
    if (a.parts) {
        // sum the row blocks of k_hist's workgroups, 8 blocks' loads in
        // flight at once (unconditional loads of in-range words, masked
        // after); hist then holds the sum
        constexpr uint32_t CHUNK = 8;
        for (uint32_t b0 = 0; b0 < a.parts; b0 += CHUNK) {
            uint32_t v[CHUNK][ROUNDS][BPT];
#pragma unroll
            for (uint32_t j = 0; j < CHUNK; ++j) {
                const uint32_t b = min(b0 + j, a.parts - 1);
                const uint32_t *pb = a.part + (uint64_t)b * (D * NB);
#pragma unroll
                for (int r = 0; r < ROUNDS; ++r) {
                    const int p = min(r * G + (int)g, D - 1);
#pragma unroll
                    for (int i = 0; i < BPT; ++i)
                        v[j][r][i] = pb[p * NB + min(lt * BPT + i, (uint32_t)NB - 1)];
                }
            }
#pragma unroll
            for (uint32_t j = 0; j < CHUNK; ++j) {
#pragma unroll
                for (int r = 0; r < ROUNDS; ++r) {
                    const bool use = b0 + j < a.parts && active && r * G + (int)g < D;
#pragma unroll
                    for (int i = 0; i < BPT; ++i)
                        cnt[r][i] += use ? v[j][r][i] : 0u;
                }
            }
        }
#pragma unroll
        for (int r = 0; r < ROUNDS; ++r) {
            const int p = r * G + (int)g;
#pragma unroll
            for (int i = 0; i < BPT; ++i)
                if (active && p < D)
                    a.hist[p * NB + lt * BPT + i] = cnt[r][i];
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        const int p = r * G + (int)g;
        uint32_t sum = 0;
        bool full = false;
        unsigned long long sq = 0;
#pragma unroll
        for (int i = 0; i < BPT; ++i) {
            sum += cnt[r][i];
            full = full || cnt[r][i] == a.n;
            sq += (unsigned long long)cnt[r][i] * cnt[r][i];
        }
        // exclusive scan of the row over the group's threads
        const uint32_t inc = wave_inclusive_scan(sum);
        // chance that two keys share this digit: sum_b (c_b / n)^2
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
            sq += __shfl_xor(sq, off);
        if ((lt & (kWave - 1)) == kWave - 1)
            s_tot[g][w] = inc;
        if ((lt & (kWave - 1)) == 0)
            s_sq[g][w] = sq;
        if (full && p < D)
            s_trivial[p] = 1;  // every writer stores the same value
        __syncthreads();
        uint32_t ex = inc - sum;
        for (uint32_t i = 0; i < w; ++i)
            ex += s_tot[g][i];
        if (active && p < D) {
#pragma unroll
            for (int i = 0; i < BPT; ++i) {
                a.digit_base[p * NB + lt * BPT + i] = ex;
                ex += cnt[r][i];
            }
        }
        if (lt == 0 && p < D) {
            unsigned long long tot = 0;
            for (int i = 0; i < WPG; ++i)
                tot += s_sq[g][i];
            // above 1/100 many lanes of a wave share a slot of the LDS lane-mask
            // table, whose same-address atomics serialise; ballots do not
            // (n < 2^30, so n^2 fits 64 bits; tot <= n^2)
            s_skewed[p] = tot > (unsigned long long)a.n * a.n / 100ull;
        }
        __syncthreads();
    }
    __syncthreads();
    if (t == 0) {
        const int limit = a.limit < D ? a.limit : D;
        int q_total = 0;
        for (int p = 0; p < limit; ++p)
            q_total += !s_trivial[p];
        // in place if either array is: the first moving pass must not write
        // its own input
        const bool in_place = a.keys_in_place || a.vals_in_place;
        const bool odd_in_place = in_place && (q_total & 1);
        int q = 0;
        uint32_t prev = kBufIn;
        for (int p = 0; p < D; ++p) {
            uint32_t plan = 0;
            if (p < limit && !s_trivial[p]) {
                uint32_t dst;
                if (odd_in_place)
                    dst = (q & 1) ? kBufOut : kBufTmp;
                else
                    dst = ((q_total - 1 - q) & 1) ? kBufTmp : kBufOut;
                plan = kPlanRun | (prev << kPlanSrcShift) | (dst << kPlanDstShift) |
                       (s_skewed[p] ? kPlanBallot : 0u) | (q == 0 ? kPlanFirst : 0u) |
                       (q == q_total - 1 && dst == kBufOut ? kPlanLast : 0u);
                prev = dst;
                ++q;
            }
            a.ctrl[kCtrlPlan + p] = plan;
        }
        // no pass moves data: the output is the input, so each array that is
        // not sorted in place is copied by the last pass launched
        if (q_total == 0)
            a.ctrl[kCtrlPlan + (limit > 0 ? limit - 1 : 0)] =
                (a.keys_in_place ? 0u : kPlanCopyIn) | (a.vals_in_place ? 0u : kPlanCopyInV);
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
    uint32_t *gagg;              // [tiles / kGroup][2^R] group aggregates (see lookback_digit)
    uint32_t *claims;            // per-XCD claim counters and group lists
    uint32_t num_tiles;
    uint32_t num_groups;
    uint32_t flat;  // claim tiles from one counter in arrival order (few tiles)
    uint32_t kmap;  // key order (kMap*), 0 = unsigned ascending
    uint32_t *err;        // error word of the control block (kErrWait)
    uint32_t spin_limit;  // polls without progress before a wait gives up
    uint32_t stall;       // test-only kStall* bits; 0 in every working call
};

// Which compute die (XCD) this wave runs on, from the XCC_ID hardware register.
__device__ __forceinline__ uint32_t xcc_id()
{
    return __builtin_amdgcn_s_getreg(20 | (0 << 6) | ((4 - 1) << 11)) & (kXcdSlots - 1);
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
// the look-back waits cannot depend on a workgroup that has not started.
//
// claims layout: [0, 8) per-XCD claim counters, then [8 + x*G + j] the id+1
// of group j of XCD x (0 = not yet published, kNoTile = no group left).
//
// Both waits are bounded: after a.spin_limit polls the claim records
// kErrWait and returns kNoTile (an opener that gives up still publishes
// kNoTile for its group, so nobody waits on it).
//
// A pass of up to kFlatClaimTiles tiles (a.flat) takes them from the global
// counter in arrival order instead: one atomic per claim rather than the
// opener's two and the others' wait for the group id, and no group opening
// in order.  Up to that size this costs less than the partly shared lines
// it leaves between XCDs; at 2048-4096 tiles (2^25-2^26 keys) the groups
// pay, except for 32-bit keys without values.
// Arrival order keeps the property above: every tile below a claimed one is
// held by a running workgroup.
template <int GROUP>
__device__ __forceinline__ uint32_t claim_tile(const PassArgs &a, uint32_t xcc)
{
    uint32_t *ctr = &a.ctrl[kCtrlTileCounter + a.pass];
    if (GROUP == 1 || a.flat) {
        (void)xcc;
        const uint32_t t = atomicAdd(ctr, 1u);
        return t < a.num_tiles ? t : kNoTile;
    } else {
        uint32_t *list = a.claims + kXcdSlots + (uint64_t)xcc * a.num_groups;
        while (true) {
            const uint32_t k = atomicAdd(&a.claims[xcc], 1u);
            const uint32_t j = k / GROUP, i = k % GROUP;
            if (j >= a.num_groups)
                return kNoTile;
            uint32_t v;
            if (i == 0) {
                uint32_t prev = 1;
                if (j > 0) {
                    uint32_t spins = 0;
                    while ((prev = __hip_atomic_load(&list[j - 1], __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT)) == 0 ||
                           (a.stall & kStallClaim)) {
                        if (++spins > a.spin_limit) {
                            atomicOr(a.err, kErrWait);
                            prev = kNoTile;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
                }
                if (prev == kNoTile) {
                    v = kNoTile;
                } else {
                    const uint32_t g = atomicAdd(ctr, 1u);
                    v = g < a.num_groups ? g + 1 : kNoTile;
                }
                __hip_atomic_store(&list[j], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                uint32_t spins = 0;
                while ((v = __hip_atomic_load(&list[j], __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT)) == 0 ||
                       (a.stall & kStallClaim)) {
                    if (++spins > a.spin_limit) {
                        atomicOr(a.err, kErrWait);
                        v = kNoTile;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
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

// Load a tile's keys (mapped to the sort order with kmap) and values;
// positions past `valid` get padding keys that sort after every real key.
template <typename K, typename V, bool HAS_V, int ITEMS>
__device__ __forceinline__ void load_tile(const K *tk, const V *tv, uint32_t valid, uint32_t off0,
                                          K (&key)[ITEMS], V (&val)[HAS_V ? ITEMS : 1], bool full,
                                          uint32_t kmap)
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
        // mapped after every load is issued, and not at all in the unsigned
        // ascending order: the loads stay in flight together
        if (kmap) {
#pragma unroll
            for (int j = 0; j < ITEMS; ++j)
                key[j] = map_in(key[j], kmap);
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
        // vmcnt(0) (expcnt and lgkmcnt left at their maximum): the loads
        // above sit behind branches, so after this path joins the full one
        // the compiler could not tell how many of them are still in flight
        // and would wait for every load, values included, before ranking
        // the first key.  Waiting here, on the partial tile only, keeps the
        // full tile's waits per item: item j is ranked once its own key has
        // arrived, while the values are still on their way.
        __builtin_amdgcn_s_waitcnt(0xF70);
        if (kmap) {
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) {
                const K mk = map_in(key[j], kmap);
                key[j] = off0 + j * kWave < valid ? mk : key[j];
            }
        }
    }
}

// Group aggregate word of the two-level look-back: [31:24] how many tiles
// of the group have added their count, [23:0] the sum of those counts (a
// group holds at most kClaimGroup x 16384 < 2^24 elements).
constexpr uint32_t kGroupTileOne = 1u << 24;
constexpr uint32_t kGroupCountMask = kGroupTileOne - 1;

// Exclusive prefix of digit d over tiles [first_tile, tile): the counting
// sort's running offset of this tile (Section 2.6), found by a decoupled
// look-back over the status words of earlier tiles.
//
// Flat form (gagg == nullptr): read LBW predecessors per round trip, add
// their counts in order up to the first inclusive word; on a tile that has
// not published yet, wait and re-read from there.
//
// Two-level form: tiles form groups of GROUP consecutive tiles (the tiles
// one XCD claims together, so a group's tiles run at the same time), and
// every tile also adds its count to its group's aggregate word.  The walk
// goes tile by tile only inside the tile's own group; before the group it
// takes a whole group per step: the inclusive word of the group's last tile
// if published (then done), else the group's aggregate once all GROUP
// tiles are in it.  A walk over the many tiles in flight then takes few
// round trips of LBW words each, not one per LBW tiles.  (Reading the whole
// group and several earlier groups in one round trip measured slower: the
// wait is mostly for the group's own earlier tiles to publish their counts,
// not for round trips.)
//
// Every wait is bounded: after wait.spin_limit rounds without progress the
// error word records kErrWait and the prefix found so far is returned.
template <int LBW, int GROUP>
__device__ __forceinline__ uint32_t lookback_digit(const uint32_t *status, const uint32_t *gagg,
                                                   uint32_t nb, uint32_t d, uint32_t tile,
                                                   uint32_t first_tile, const PassArgs &wait)
{
    uint32_t prefix = 0;
    uint32_t spins = 0;
    const bool stall = (wait.stall & kStallLookback) != 0;
    const int64_t glo = gagg ? std::max<int64_t>(first_tile, (int64_t)(tile - tile % GROUP))
                             : (int64_t)first_tile;
    // tiles of this group before this one (all earlier tiles in flat form)
    int64_t k = (int64_t)tile - 1;
    while (k >= glo) {
        uint32_t st[LBW];
#pragma unroll
        for (int i = 0; i < LBW; ++i)
            st[i] = (k - i >= glo) ? __hip_atomic_load(&status[(uint64_t)(k - i) * nb + d],
                                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                   : 0u;
        int used = 0;
        bool done = false;
        if (!stall) {
#pragma unroll
            for (int i = 0; i < LBW; ++i) {
                if (!done && used == i && k - i >= glo) {
                    const uint32_t f = st[i] & kFlagMask;
                    if (f != 0) {
                        prefix += st[i] & kCountMask;
                        done = f == kFlagInc;
                        used = i + 1;
                    }
                }
            }
        }
        if (done)
            return prefix;
        k -= used;
        if (k < glo)
            break;
        if (used == 0 && ++spins > wait.spin_limit) {
            atomicOr(wait.err, kErrWait);
            return prefix;
        }
        if (used < LBW)
            __builtin_amdgcn_s_sleep(1);
    }
    if (!gagg)
        return prefix;  // reached first_tile: no earlier tile
    // earlier groups, newest first, LBW per round trip
    int64_t g = (int64_t)(tile / GROUP) - 1;
    const int64_t g_lo = (int64_t)(first_tile / GROUP);
    while (g >= g_lo) {
        uint32_t last[LBW], agg[LBW];
#pragma unroll
        for (int i = 0; i < LBW; ++i) {
            const bool in = g - i >= g_lo;
            const uint64_t gi = (uint64_t)(in ? g - i : 0);
            last[i] = in ? __hip_atomic_load(&status[(gi * GROUP + GROUP - 1) * nb + d],
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                         : 0u;
            agg[i] = in ? __hip_atomic_load(&gagg[gi * nb + d], __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT)
                        : 0u;
        }
        int used = 0;
        bool done = false;
        if (!stall) {
#pragma unroll
            for (int i = 0; i < LBW; ++i) {
                if (!done && used == i && g - i >= g_lo) {
                    if ((last[i] & kFlagMask) == kFlagInc) {
                        prefix += last[i] & kCountMask;
                        done = true;
                        used = i + 1;
                    } else if ((agg[i] >> 24) == (uint32_t)GROUP) {
                        prefix += agg[i] & kGroupCountMask;
                        used = i + 1;
                    }
                }
            }
        }
        if (done)
            return prefix;
        g -= used;
        if (g < g_lo)
            break;
        if (used == 0 && ++spins > wait.spin_limit) {
            atomicOr(wait.err, kErrWait);
            return prefix;
        }
        if (used < LBW)
            __builtin_amdgcn_s_sleep(1);
    }
    return prefix;
}

// A staged (key, value) pair: one 8- or 16-byte LDS word.
template <typename K>
struct alignas(2 * sizeof(K)) KvPair {
    K k;
    K v;
};

// LDS of one digit pass: the per-wave counters, the digits' global bases and
// the staging memory: a key buffer (which holds the lane-mask tables while
// ranking) and a value buffer right after it, which pairs use as one array
// of (key, value) words, staged in one step and written out after one
// barrier.
template <typename K, typename C, bool HAS_V>
struct PassLds {
    static constexpr int W = C::kThreads / kWave;
    static constexpr size_t kStageBytes = (size_t)C::kTile * sizeof(K);
    static_assert(C::kWide || (size_t)W * C::kBins * 8 <= kStageBytes,
                  "the lane-mask tables live in the staging buffer");
    uint32_t wcnt[W * C::kBins];  // per wave and digit: count, then base in tile
    uint32_t gbase[C::kBins];
    uint32_t tmp[8];
    uint32_t tile;
    __attribute__((aligned(16))) unsigned char stage[kStageBytes];
    __attribute__((aligned(16))) unsigned char stage_v[HAS_V ? kStageBytes : 16];
};

// One tile of a digit pass (the paper's counting sort, Section 2.6, spread
// over workgroups): rank, publish the tile's digit counts, decoupled
// look-back over tiles [first_tile, tile), stage in LDS, write the digit
// runs.  after_lookback(t) runs in every thread once the look-back is done,
// before the writes (the plain pass claims its next tile there).  The tile's elements are tk/tv[0, valid); destination index i of the
// digit-sorted sequence is dk/dv[i] for i < limit.  dbase (threads < 2^R) is
// the digit's starting offset in that sequence.  Ends with a barrier.
template <typename K, typename V, bool HAS_V, typename C, typename Hook>
__device__ __forceinline__ void pass_tile(PassLds<K, C, HAS_V> &L, const K *tk, const V *tv, K *dk,
                                          V *dv, uint32_t valid, uint32_t limit, uint32_t tile,
                                          uint32_t first_tile, uint32_t *status, uint32_t *gagg,
                                          uint32_t dbase, int shift, bool ballot_rank,
                                          uint32_t map_load, uint32_t map_store,
                                          const PassArgs &wait, Hook &&after_lookback)
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
    V *s_v = (V *)L.stage_v;
    // pairs: one (key, value) word per element across both staging buffers,
    // so staging is one LDS write per element at its rank and the writes
    // read the pairs back in order
    constexpr bool KV = HAS_V;
    using Lds = PassLds<K, C, HAS_V>;
    static_assert(!KV || offsetof(Lds, stage_v) == offsetof(Lds, stage) + Lds::kStageBytes,
                  "the value buffer follows the key buffer");
    KvPair<K> *s_kv = (KvPair<K> *)L.stage;
    uint64_t *s_mask = (uint64_t *)L.stage;
    const uint32_t t = threadIdx.x;
    const uint32_t w = t / kWave;
    const uint32_t lane = t % kWave;
    const uint32_t off0 = w * (kWave * ITEMS) + lane;
    uint32_t *wc = L.wcnt + w * NB;

    // this wave's counters and lane-mask table are its own: it clears them
    // itself (after the previous tile's closing barrier), no barrier needed
    for (uint32_t i = lane; i < NB; i += kWave) {
        wc[i] = 0;
        s_mask[w * NB + i] = 0;
    }
    // load: item j of lane l is element j*64 + l of this wave's run
    K key[ITEMS];
    V val[HAS_V ? ITEMS : 1];
    load_tile<K, V, HAS_V, ITEMS>(tk, tv, valid, off0, key, val, valid == (uint32_t)T, map_load);

    // count: stable rank of every item among the wave's items of its digit
    uint32_t rank[ITEMS];
    if (ballot_rank || w < (uint32_t)C::kBallotWaves)
        wave_rank_ballot<R, K, ITEMS>(key, shift, wc, rank);
    else
        wave_rank<R, K, ITEMS>(key, shift, wc, s_mask + w * NB, lane, rank);
    __syncthreads();

    // scan: wave offsets per digit, tile count, publish the aggregate,
    // tile-local offsets
    uint32_t cnt = 0;
    if (t < NB) {
#pragma unroll
        for (int ww = 0; ww < W; ++ww) {
            const uint32_t c = L.wcnt[ww * NB + t];
            L.wcnt[ww * NB + t] = cnt;
            cnt += c;
        }
        __hip_atomic_store(&status[(uint64_t)tile * NB + t],
                           (tile == first_tile ? kFlagInc : kFlagAgg) | cnt, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        if (gagg)
            __hip_atomic_fetch_add(&gagg[(uint64_t)(tile / C::kGroup) * NB + t],
                                   kGroupTileOne | cnt, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
    }
    const uint32_t excl = bins_exclusive_scan<NB>(cnt, L.tmp);
    if (t < NB) {
        // tile-local offsets: wave offset + the digit's start in the tile
#pragma unroll
        for (int ww = 0; ww < W; ++ww)
            L.wcnt[ww * NB + t] += excl;
    }
    __syncthreads();
    // stage the keys and values in rank order; the digit owners first look
    // back (the other waves stage meanwhile), since only the global base
    // needs it
    if (t >= NB) {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            rank[j] += wc[digit_of<R>(key[j], shift)];  // position in the tile
            if constexpr (KV) {
                s_kv[rank[j]] = KvPair<K>{key[j], (K)val[j]};
            } else {
                s_k[rank[j]] = key[j];
                if constexpr (HAS_V)
                    s_v[rank[j]] = val[j];
            }
        }
    }
    if (t < NB) {
        // decoupled look-back over the tiles before this one
        const uint32_t prefix =
            tile == first_tile
                ? 0u
                : lookback_digit<LBW, C::kGroup>(status, gagg, NB, t, tile, first_tile, wait);
        if (tile != first_tile)
            __hip_atomic_store(&status[(uint64_t)tile * NB + t], kFlagInc | (prefix + cnt),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        L.gbase[t] = dbase + prefix - excl;
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            rank[j] += wc[digit_of<R>(key[j], shift)];
            if constexpr (KV) {
                s_kv[rank[j]] = KvPair<K>{key[j], (K)val[j]};
            } else {
                s_k[rank[j]] = key[j];
                if constexpr (HAS_V)
                    s_v[rank[j]] = val[j];
            }
        }
    }
    __syncthreads();
    after_lookback(t);

    // place: write each digit run out with consecutive lanes on consecutive
    // addresses; then the values
    uint32_t dst[ITEMS];
    V vk[KV ? ITEMS : 1];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t pos = i * THREADS + t;
        K k;
        if constexpr (KV) {
            const KvPair<K> kv = s_kv[pos];
            k = kv.k;
            vk[i] = (V)kv.v;
        } else {
            k = s_k[pos];
        }
        dst[i] = L.gbase[digit_of<R>(k, shift)] + pos;
        if (dst[i] < limit)
            store_at(dk, dst[i], map_out(k, map_store));
    }
    if constexpr (HAS_V) {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i)
            if (dst[i] < limit) {
                if constexpr (KV)
                    store_at(dv, dst[i], vk[i]);
                else
                    store_at(dv, dst[i], s_v[i * THREADS + t]);
            }
    }
    __syncthreads();  // LDS is reused by the next tile
}

}  // namespace rs

#include "rs_wide.h"

namespace rs {

template <typename K, typename V, bool HAS_V, typename C>
__global__ __launch_bounds__(C::kThreads) void k_pass(PassArgs a)
{
    constexpr int THREADS = C::kThreads;
    constexpr int T = C::kTile;
    using Lds = std::conditional_t<C::kWide, WideLds<K, C, HAS_V>, PassLds<K, C, HAS_V>>;
    __shared__ Lds L;

    const uint32_t t = threadIdx.x;
    const uint32_t plan = a.ctrl[kCtrlPlan + a.pass];
    if (!(plan & kPlanRun)) {
        if (plan & (kPlanCopyIn | kPlanCopyInV)) {
            // no pass moves data: copy in -> out (each array not sorted in place)
            for (uint64_t tl = blockIdx.x; tl < a.num_tiles; tl += gridDim.x) {
                const uint64_t lo = tl * T;
                const uint64_t hi = std::min<uint64_t>(lo + T, a.n);
                if (plan & kPlanCopyIn)
                    copy_range(pick<const K>(a.b, kBufIn, false), pick<K>(a.b, kBufOut, false),
                               lo, hi, t, THREADS);
                if constexpr (HAS_V) {
                    if (plan & kPlanCopyInV)
                        copy_range(pick<const V>(a.b, kBufIn, true), pick<V>(a.b, kBufOut, true),
                                   lo, hi, t, THREADS);
                }
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
    // the starting offsets of this thread's digits, fetched early (used
    // after the look-back): digit t, or digits 2t and 2t+1 of a wide pass
    uint32_t dbase = 0;
    uint32_t db[2] = {0, 0};
    if constexpr (C::kWide) {
        const uint2 d2 = ((const uint2 *)a.digit_base)[t];
        db[0] = d2.x;
        db[1] = d2.y;
    } else {
        dbase = t < (uint32_t)C::kBins ? a.digit_base[t] : 0u;
    }
    const uint32_t xcc = t == 0 ? xcc_id() : 0u;
    // the next tile is claimed once the current tile's look-back is done:
    // the claim's round trips overlap the writes, and the workgroup waits
    // on nothing while it holds the claimed tile
    if (t == 0)
        L.tile = claim_tile<C::kGroup>(a, xcc);
    __syncthreads();
    while (true) {
        // the claim made during the previous tile is visible after its
        // closing barrier
        const uint32_t tile = L.tile;
        if (tile == kNoTile)
            break;
        const uint64_t tb = (uint64_t)tile * T;
        const uint32_t valid = (uint32_t)std::min<uint64_t>(T, a.n - tb);
        auto claim_next = [&](uint32_t tt) {
            if (tt == 0)
                L.tile = claim_tile<C::kGroup>(a, xcc);
        };
        if constexpr (C::kWide)
            pass_tile_wide<K, V, HAS_V, C>(L, sk + tb, HAS_V ? sv + tb : nullptr, dk, dv, valid,
                                           a.n, tile, 0, a.status, db, a.shift,
                                           (plan & kPlanBallot) != 0,
                                           (plan & kPlanFirst) ? a.kmap : 0u,
                                           (plan & kPlanLast) ? a.kmap : 0u, a, claim_next);
        else
            pass_tile<K, V, HAS_V, C>(L, sk + tb, HAS_V ? sv + tb : nullptr, dk, dv, valid, a.n,
                                      tile, 0, a.status, a.gagg, dbase, a.shift,
                                      (plan & kPlanBallot) != 0,
                                      (plan & kPlanFirst) ? a.kmap : 0u,
                                      (plan & kPlanLast) ? a.kmap : 0u, a, claim_next);
    }
}

// ---------------------------------------------------------------------------
// Segmented sort: digit histograms of the large segments, chunk by chunk.
// Persistent workgroups claim chunks of kSegChunk elements, count all digit
// positions in the column table of k_hist and add the counts to the
// segment's histogram (global atomics).

struct SegHistArgs {
    const void *kin;
    const SegLarge *large;
    const uint32_t *chunk_seg;
    uint32_t max_chunks;
    uint32_t *ctrl;
    uint32_t *seg_hist;   // [large segment][d][2^R], zeroed
    uint32_t *seg_base;   // [large segment][d][2^R]
    uint32_t *seg_flags;  // [large segment]: bit p pass p's digit is the same for the
                          // whole segment; bit 16 + p pass p's digits are skewed
    uint32_t kmap;        // key order applied to every key read
};

constexpr int kSegSkewShift = 16;

constexpr int kSegHistThreads = 1024;

template <typename K, int R>
__global__ __launch_bounds__(kSegHistThreads) void k_seg_hist(SegHistArgs a)
{
    constexpr int D = num_passes<K, R>();
    constexpr int NB = 1 << R;
    constexpr int NK = 16;  // keys per thread per round, all loaded before counting
    constexpr uint32_t ROUND = kSegHistThreads * NK;
    constexpr uint32_t TAB = (D << R) * kHistCols;
    __shared__ uint32_t tab[TAB];
    __shared__ uint32_t s_item;
    const uint32_t t = threadIdx.x;
    const uint32_t col = t % kHistCols;
    const K *keys = (const K *)a.kin;
    const uint32_t chunks = min(a.ctrl[kSegChunks], a.max_chunks);
    for (uint32_t i = t; i < TAB; i += kSegHistThreads)
        tab[i] = 0;
    while (true) {
        // the barrier also ends the previous chunk's flush in every thread
        if (t == 0)
            s_item = atomicAdd(&a.ctrl[kSegChunkClaim], 1u);
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
        for (uint32_t r0 = 0; r0 < len; r0 += ROUND) {
            if (r0 + ROUND <= len) {
                K key[NK];
#pragma unroll
                for (int j = 0; j < NK; ++j)
                    key[j] = sk[r0 + j * kSegHistThreads + t];
                if (a.kmap) {
#pragma unroll
                    for (int j = 0; j < NK; ++j)
                        key[j] = map_in(key[j], a.kmap);
                }
#pragma unroll
                for (int p = 0; p < D; ++p) {
#pragma unroll
                    for (int j = 0; j < NK; ++j)
                        hist_add<R>(tab, p, digit_of<R>(key[j], p * R), col);
                }
            } else {
                for (uint32_t e = r0 + t; e < len; e += kSegHistThreads) {
                    const K key = map_in(sk[e], a.kmap);
#pragma unroll
                    for (int p = 0; p < D; ++p)
                        hist_add<R>(tab, p, digit_of<R>(key, p * R), col);
                }
            }
        }
        __syncthreads();
        // add the chunk's counts to its segment's histogram and clear them
        uint32_t *out = a.seg_hist + (uint64_t)seg * D * NB;
        for (uint32_t r = t; r < (uint32_t)D << R; r += kSegHistThreads) {
            uint32_t s = 0;
#pragma unroll
            for (uint32_t c = 0; c < kHistCols; ++c) {
                const uint32_t i = r * kHistCols + ((c + r) & (kHistCols - 1));
                s += tab[i];
                tab[i] = 0;
            }
            if (s)
                atomicAdd(&out[r], s);
        }
    }
}

// seg_base[seg][p] = exclusive scan of seg_hist[seg][p], one workgroup per
// large segment (persistent).
template <typename K, int R>
__global__ __launch_bounds__(256) void k_seg_scan(SegHistArgs a)
{
    constexpr int D = num_passes<K, R>();
    constexpr int NB = 1 << R;
    static_assert(D <= kSegSkewShift, "pass flags fit 16 bits each");
    __shared__ uint32_t s_tmp[8];
    __shared__ uint32_t s_item;
    __shared__ unsigned long long s_sq[256 / kWave];
    const uint32_t t = threadIdx.x;
    while (true) {
        if (t == 0)
            s_item = atomicAdd(&a.ctrl[kSegScanClaim], 1u);
        __syncthreads();
        const uint32_t item = s_item;
        if (item >= a.ctrl[kSegLargeLen])
            break;
        const uint32_t size = a.large[item].size;
        uint32_t flags = 0;
        for (int p = 0; p < D; ++p) {
            const uint64_t i = ((uint64_t)item * D + p) * NB + t;
            const uint32_t c = t < (uint32_t)NB ? a.seg_hist[i] : 0u;
            const uint32_t ex = bins_exclusive_scan<NB>(c, s_tmp);
            if (t < (uint32_t)NB)
                a.seg_base[i] = ex;
            // one digit for the whole segment: this pass is the identity
            const bool trivial = __syncthreads_or(c == size) != 0;
            // skewed: sum of squared counts above size^2 / 100 (as k_plan)
            unsigned long long sq = (unsigned long long)c * c;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1)
                sq += __shfl_xor(sq, off);
            if ((t & (kWave - 1)) == 0)
                s_sq[t / kWave] = sq;
            __syncthreads();
            unsigned long long tot = 0;
#pragma unroll
            for (int w = 0; w < 256 / kWave; ++w)
                tot += s_sq[w];
            const bool skewed = tot > (unsigned long long)size * size / 100ull;
            flags |= (trivial ? 1u << p : 0u) | (skewed ? 1u << (kSegSkewShift + p) : 0u);
            __syncthreads();
        }
        if (t == 0)
            a.seg_flags[item] = flags;
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
    const uint32_t *seg_flags; // [large segment]: trivial and skewed passes (k_seg_scan)
    uint32_t *ctrl;            // segmented control block
    uint32_t *status;          // look-back words of this pass
    uint32_t *claims;          // claim counters of this pass
    uint32_t max_tiles;        // tiles the workspace holds
    int pass;
    int shift;
    int d;
    uint32_t map_load;   // key order applied to the keys read (first pass)
    uint32_t map_store;  // key order undone on the keys written (last pass into the output)
    uint32_t spin_limit;  // polls without progress before a wait gives up
    uint32_t stall;       // test-only kStall* bits; 0 in every working call
};

template <typename K, typename V, bool HAS_V, typename C>
__global__ __launch_bounds__(C::kThreads) void k_seg_pass(SegPassArgs a)
{
    constexpr int T = C::kTile;
    constexpr uint32_t NB = C::kBins;
    __shared__ PassLds<K, C, HAS_V> L;
    const uint32_t t = threadIdx.x;
    PassArgs pa{};
    pa.ctrl = a.ctrl + (kSegPassCounter - kCtrlTileCounter);
    pa.pass = a.pass;
    pa.claims = a.claims;
    pa.num_tiles = std::min(a.ctrl[kSegTiles], a.max_tiles);
    pa.num_groups = (pa.num_tiles + C::kGroup - 1) / C::kGroup;
    pa.err = a.ctrl + kSegError;
    pa.spin_limit = a.spin_limit;
    pa.stall = a.stall;
    const uint32_t xcc = t == 0 ? xcc_id() : 0u;
    while (true) {
        if (t == 0)
            L.tile = claim_tile<C::kGroup>(pa, xcc);
        __syncthreads();
        const uint32_t tile = L.tile;
        if (tile == kNoTile)
            break;
        const uint32_t seg = a.tile_seg[tile];
        const SegLarge rec = a.large[seg];
        const uint32_t lt = tile - rec.tile_start;
        const uint32_t first = lt * T;
        const uint32_t valid = rec.size > first ? std::min<uint32_t>(T, rec.size - first) : 0u;
        const uint32_t flags = a.seg_flags[seg];
        const uint64_t off = rec.start + (uint64_t)lt * T;
        if ((flags >> a.pass) & 1u) {
            // the segment's digit is the same everywhere: the pass is the
            // identity permutation, so the tile is copied (no rank, no
            // look-back; the segment's other tiles do the same).  All of a
            // thread's loads are in flight before its first store.
            const uint32_t off0 = (t / kWave) * (kWave * C::kItems) + t % kWave;
            K key[C::kItems];
            V val[HAS_V ? C::kItems : 1];
            load_tile<K, V, HAS_V, C::kItems>((const K *)a.src_k + off,
                                              HAS_V ? (const V *)a.src_v + off : nullptr, valid,
                                              off0, key, val, valid == (uint32_t)T, a.map_load);
            K *dk = (K *)a.dst_k + off;
            V *dv = HAS_V ? (V *)a.dst_v + off : nullptr;
#pragma unroll
            for (int j = 0; j < C::kItems; ++j) {
                const uint32_t i = off0 + j * kWave;
                if (i < valid) {
                    dk[i] = map_out(key[j], a.map_store);
                    if constexpr (HAS_V)
                        dv[i] = val[j];
                }
            }
            __syncthreads();  // every thread has read this tile's id
            continue;
        }
        const uint32_t dbase = t < NB ? a.seg_base[((uint64_t)seg * a.d + a.pass) * NB + t] : 0u;
        pass_tile<K, V, HAS_V, C>(L, (const K *)a.src_k + off,
                                  HAS_V ? (const V *)a.src_v + off : nullptr,
                                  (K *)a.dst_k + rec.start,
                                  HAS_V ? (V *)a.dst_v + rec.start : nullptr, valid, rec.size,
                                  tile, rec.tile_start, a.status, nullptr, dbase, a.shift,
                                  ((flags >> (kSegSkewShift + a.pass)) & 1u) != 0, a.map_load,
                                  a.map_store, pa, [](uint32_t) {});
    }
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
    uint32_t kmap;  // key order undone on the keys copied out
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
        if (a.kmap) {
            const K *sk = (const K *)a.src_k + rec.start;
            K *dk = (K *)a.dst_k + rec.start;
            for (uint64_t i = lo + threadIdx.x; i < hi; i += 256)
                dk[i] = map_out(sk[i], a.kmap);
        } else {
            copy_range((const K *)a.src_k + rec.start, (K *)a.dst_k + rec.start, lo, hi,
                       threadIdx.x, 256);
        }
        if constexpr (HAS_V)
            copy_range((const K *)a.src_v + rec.start, (K *)a.dst_v + rec.start, lo, hi,
                       threadIdx.x, 256);
    }
}

}  // namespace rs
