// Stable merge sort (paper, Section 2.4: cut the sequence into runs, sort
// each, merge sorted runs with a stable merge until one remains), the
// comparison-based counterpart of the radix path.
//
//   k_merge_tile   one workgroup sorts a tile of THREADS x ITEMS elements:
//                  each thread sorts its ITEMS in registers with an odd-even
//                  transposition network, then the workgroup merges runs of
//                  ITEMS, 2 ITEMS, ... in LDS until the tile is one run;
//   k_merge_split  for one merge level (runs of w elements merged pairwise),
//                  the merge-path split of every output tile: how many of the
//                  tile's first outputs come from the left run;
//   k_merge_pass   one workgroup per output tile: stage the tile's share of
//                  both runs in LDS, each thread merges ITEMS outputs from its
//                  own splits, then a coalesced store.
//
// Every merge is stable: on equal keys the left run's element goes first,
// and in a split the left run gives every element <= the right run's next.
// Keys are compared after the key-order map (applied on the tile sort's
// load, undone on the last store).  Positions are 32-bit (n < 2^30).
#pragma once

#include "rs_device.h"

namespace rs {

// Shapes measured on MI355X (2^26 32-bit and 2^25 64-bit pairs): short
// per-thread merges and many waves hide the LDS latency of the merge better
// than long ones; more than one merge chain per thread (interleaved chains,
// each with its own split) costs more ALU than it hides.  Tile sorts of 8192
// elements; merge-pass workgroups of 2048 outputs.
template <typename K, bool HAS_V>
struct MergeShape {
    static constexpr int kTileThreads = 1024;
    static constexpr int kTileItems = 8;
    static constexpr int kTileChains = 1;  // independent merge chains per thread
    static constexpr int kPassThreads = sizeof(K) == 8 ? 512 : 256;
    static constexpr int kPassItems = sizeof(K) == 8 ? 4 : 8;
    static constexpr int kPassChains = 1;
    static constexpr int kTile = kTileThreads * kTileItems;      // elements per tile sort
    static constexpr int kPassTile = kPassThreads * kPassItems;  // outputs per merge-pass tile
};

// LDS slot of element e: one element of padding after every ITEMS, so that
// the lanes of a wave reading their own ITEMS consecutive elements hit
// different banks (lane stride ITEMS + 1 elements).
template <int ITEMS>
__device__ __forceinline__ uint32_t lds_slot(uint32_t e)
{
    return e + e / ITEMS;
}

template <int N, int ITEMS>
struct PaddedLen {
    static constexpr int value = N + N / ITEMS;
};

// ITEMS outputs of one thread as C interleaved chains of ITEMS / C outputs,
// each from its own merge-path split: the LDS reads of different chains are
// independent, so C of them are in flight where one chain would wait for
// each.  Runs are [0, na) and [na, na + nb) of the LDS positions starting
// at `base`; the thread's first output is `diag` (<= na + nb).
//
// The merge-path split of output d is the number i of left-run elements
// among the first d outputs of the stable merge: every A[x], x < i,
// precedes B[d - i] (A[x] <= B[d - i]) and every B[y], y < d - i, precedes
// A[i] (B[y] < A[i]); a binary search finds it.  From there the merge takes
// the left element whenever it is <= the right one.
template <typename K, int ITEMS, int C, int PAD_ITEMS>
__device__ __forceinline__ void merge_chains(const K *s_k, uint32_t base, uint32_t na, uint32_t nb,
                                             uint32_t diag, K (&key)[ITEMS],
                                             uint32_t (&src)[ITEMS])
{
    constexpr int L = ITEMS / C;
    static_assert(L * C == ITEMS, "chains split the items evenly");
    const uint32_t total = na + nb;
    uint32_t d[C], lo[C], hi[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        d[c] = min(diag + c * L, total);
        lo[c] = d[c] > nb ? d[c] - nb : 0u;
        hi[c] = d[c] < na ? d[c] : na;
    }
    // C binary searches side by side
    while (true) {
        bool more = false;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            if (lo[c] < hi[c]) {
                const uint32_t mid = (lo[c] + hi[c]) >> 1;
                const K x = s_k[lds_slot<PAD_ITEMS>(base + mid)];
                const K y = s_k[lds_slot<PAD_ITEMS>(base + na + d[c] - 1 - mid)];
                if (x <= y)
                    lo[c] = mid + 1;
                else
                    hi[c] = mid;
                more |= lo[c] < hi[c];
            }
        }
        if (!more)
            break;
    }
    uint32_t ia[C], ib[C];
    K a[C], b[C];
    const uint32_t ea = base + na, eb = base + total;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        ia[c] = base + lo[c];
        ib[c] = base + na + (d[c] - lo[c]);
        a[c] = ia[c] < ea ? s_k[lds_slot<PAD_ITEMS>(ia[c])] : (K)0;
        b[c] = ib[c] < eb ? s_k[lds_slot<PAD_ITEMS>(ib[c])] : (K)0;
    }
#pragma unroll
    for (int j = 0; j < L; ++j) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const bool take_a = ib[c] >= eb || (ia[c] < ea && a[c] <= b[c]);
            key[c * L + j] = take_a ? a[c] : b[c];
            src[c * L + j] = take_a ? ia[c] : ib[c];
            ia[c] += take_a;
            ib[c] += !take_a;
            const uint32_t nx = take_a ? ia[c] : ib[c];
            const bool has = take_a ? ia[c] < ea : ib[c] < eb;
            const K nk = has ? s_k[lds_slot<PAD_ITEMS>(nx)] : (K)0;
            a[c] = take_a ? nk : a[c];
            b[c] = take_a ? b[c] : nk;
        }
    }
}

// Orders this wave's LDS accesses before and after it: waits for the wave's
// outstanding LDS operations and keeps the compiler from moving LDS
// accesses across it (the lanes of one wave then see each other's writes).
__device__ __forceinline__ void wave_lds_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Stable odd-even transposition sort of ITEMS registers: ITEMS rounds of
// compare-exchanges between neighbours, exchanging only strictly greater
// keys, so equal keys never pass each other.
template <typename K, typename V, bool HAS_V, int ITEMS>
__device__ __forceinline__ void register_sort(K (&key)[ITEMS], V (&val)[HAS_V ? ITEMS : 1])
{
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
#pragma unroll
        for (int j = r & 1; j + 1 < ITEMS; j += 2) {
            const bool sw = key[j] > key[j + 1];
            const K lo = sw ? key[j + 1] : key[j];
            const K hi = sw ? key[j] : key[j + 1];
            key[j] = lo;
            key[j + 1] = hi;
            if constexpr (HAS_V) {
                const V vl = sw ? val[j + 1] : val[j];
                const V vh = sw ? val[j] : val[j + 1];
                val[j] = vl;
                val[j + 1] = vh;
            }
        }
    }
}

struct MergeTileArgs {
    const void *kin;
    const void *vin;
    void *kout;
    void *vout;
    uint32_t n;
    uint32_t map_load;   // key order applied on load
    uint32_t map_store;  // key order undone on store (when no merge level follows)
};

template <typename K, typename V, bool HAS_V, int THREADS, int ITEMS, int CHAINS>
__global__ __launch_bounds__(THREADS) void k_merge_tile(MergeTileArgs a)
{
    constexpr uint32_t T = THREADS * ITEMS;
    constexpr int SLOTS = PaddedLen<T, ITEMS>::value;
    __shared__ K s_k[SLOTS];
    __shared__ V s_v[HAS_V ? SLOTS : 1];

    const uint32_t t = threadIdx.x;
    const uint32_t base = blockIdx.x * T;
    const uint32_t valid = min(T, a.n - base);
    const K *kin = (const K *)a.kin + base;
    const V *vin = HAS_V ? (const V *)a.vin + base : nullptr;

    // coalesced load into LDS; padding keys (all ones) stay behind every
    // real key because they come last and every merge is stable
    {
        K key[ITEMS];
        V val[HAS_V ? ITEMS : 1];
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t e = j * THREADS + t;
            key[j] = e < valid ? kin[e] : KeyTraits<K>::kPad;
            if constexpr (HAS_V)
                val[j] = e < valid ? vin[e] : (V)0;
        }
        if (a.map_load) {
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) {
                const K mk = map_in(key[j], a.map_load);
                key[j] = j * THREADS + t < valid ? mk : key[j];
            }
        }
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t e = j * THREADS + t;
            s_k[lds_slot<ITEMS>(e)] = key[j];
            if constexpr (HAS_V)
                s_v[lds_slot<ITEMS>(e)] = val[j];
        }
    }
    __syncthreads();

    // each thread: its ITEMS consecutive elements, sorted in registers
    K key[ITEMS];
    V val[HAS_V ? ITEMS : 1];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        key[j] = s_k[lds_slot<ITEMS>(t * ITEMS + j)];
        if constexpr (HAS_V)
            val[j] = s_v[lds_slot<ITEMS>(t * ITEMS + j)];
    }
    register_sort<K, V, HAS_V, ITEMS>(key, val);

    // merge runs of w elements pairwise in LDS, w = ITEMS, 2 ITEMS, ...
    // While a pair of runs (2w elements) lies within one wave's kWave x ITEMS
    // elements, a round reads only what its own wave wrote: a wave-level
    // fence orders it (LDS accesses of one wave complete in order once the
    // compiler waits for them); larger rounds need the workgroup barrier.
    constexpr uint32_t kWaveSpan = kWave * ITEMS;
    for (uint32_t w = ITEMS; w < T; w *= 2) {
        const bool in_wave = 2 * w <= kWaveSpan;
        if (in_wave)
            wave_lds_fence();
        else
            __syncthreads();  // every read of the previous round is done
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            s_k[lds_slot<ITEMS>(t * ITEMS + j)] = key[j];
            if constexpr (HAS_V)
                s_v[lds_slot<ITEMS>(t * ITEMS + j)] = val[j];
        }
        if (in_wave)
            wave_lds_fence();
        else
            __syncthreads();
        const uint32_t o = t * ITEMS;          // first output of this thread
        const uint32_t pb = o & ~(2 * w - 1);  // its pair of runs
        uint32_t src[ITEMS];
        merge_chains<K, ITEMS, CHAINS, ITEMS>(s_k, pb, w, w, o - pb, key, src);
        if constexpr (HAS_V) {
#pragma unroll
            for (int j = 0; j < ITEMS; ++j)
                val[j] = s_v[lds_slot<ITEMS>(src[j])];
        }
    }

    // blocked registers -> LDS -> coalesced store
    __syncthreads();
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        s_k[lds_slot<ITEMS>(t * ITEMS + j)] = key[j];
        if constexpr (HAS_V)
            s_v[lds_slot<ITEMS>(t * ITEMS + j)] = val[j];
    }
    __syncthreads();
    K *kout = (K *)a.kout + base;
    V *vout = HAS_V ? (V *)a.vout + base : nullptr;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const uint32_t e = j * THREADS + t;
        if (e < valid) {
            kout[e] = map_out(s_k[lds_slot<ITEMS>(e)], a.map_store);
            if constexpr (HAS_V)
                vout[e] = s_v[lds_slot<ITEMS>(e)];
        }
    }
}

// One merge level: runs [q 2w, q 2w + w) and [q 2w + w, q 2w + 2w) (clipped
// to n) merge into [q 2w, q 2w + 2w).
struct MergeLevelArgs {
    const void *sk;
    const void *sv;
    void *dk;
    void *dv;
    uint32_t *split;  // per output-tile boundary: absolute position in the left run
    uint32_t n;
    uint32_t w;          // run length of this level
    uint32_t tiles;      // output tiles of the merge pass
    uint32_t map_store;  // key order undone on store (last level only)
};

// Pair of runs holding output position g, and the lengths of its two runs.
struct PairRuns {
    uint32_t base, na, nb;
};

__device__ __forceinline__ PairRuns pair_runs(uint32_t g, uint32_t w, uint32_t n)
{
    PairRuns p;
    p.base = g / (2 * w) * (2 * w);
    const uint32_t left = n - p.base;
    p.na = min(w, left);
    p.nb = left > w ? min(w, left - w) : 0u;
    return p;
}

// One thread per split: a binary search for the first x in [lo, hi) with
// A[x] > B[diag - 1 - x] (hi if none), the merge-path split of merge_chains.
// Measured on MI355X, searches with several probes per step (8 per thread,
// or 64 per wave) fetch so many more scattered lines that they take longer
// than this one, whose deep probes mostly hit lines shared by neighbouring
// splits.
template <typename K, int TILE>
__global__ __launch_bounds__(256) void k_merge_split(MergeLevelArgs a)
{
    const uint32_t b = blockIdx.x * 256 + threadIdx.x;
    if (b >= a.tiles)
        return;
    // the split at the start of output tile b (tiles never straddle a pair:
    // TILE divides 2w)
    const uint32_t g = b * TILE;
    const PairRuns p = pair_runs(g, a.w, a.n);
    const K *A = (const K *)a.sk + p.base;
    const K *B = A + a.w;
    const uint32_t diag = g - p.base;
    uint32_t lo = diag > p.nb ? diag - p.nb : 0u;
    uint32_t hi = diag < p.na ? diag : p.na;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (A[mid] <= B[diag - 1 - mid])
            lo = mid + 1;
        else
            hi = mid;
    }
    a.split[b] = p.base + lo;
}

template <typename K, typename V, bool HAS_V, int THREADS, int ITEMS, int CHAINS>
__global__ __launch_bounds__(THREADS) void k_merge_pass(MergeLevelArgs a)
{
    constexpr uint32_t T = THREADS * ITEMS;
    constexpr int SLOTS = PaddedLen<T, ITEMS>::value;
    __shared__ K s_k[SLOTS];
    __shared__ V s_v[HAS_V ? SLOTS : 1];

    const uint32_t t = threadIdx.x;
    const uint32_t b = blockIdx.x;
    const uint32_t g0 = b * T;
    const uint32_t g1 = min(g0 + T, a.n);
    const PairRuns p = pair_runs(g0, a.w, a.n);
    const uint32_t a_begin = p.base, b_begin = p.base + a.w;
    // this tile's share of each run
    const uint32_t a0 = a.split[b];
    const uint32_t b0 = b_begin + (g0 - p.base) - (a0 - a_begin);
    uint32_t a1, b1;
    if (g1 == p.base + p.na + p.nb) {  // the tile ends its pair
        a1 = a_begin + p.na;
        b1 = b_begin + p.nb;
    } else {
        a1 = a.split[b + 1];
        b1 = b_begin + (g1 - p.base) - (a1 - a_begin);
    }
    const uint32_t ca = a1 - a0, cb = b1 - b0;  // ca + cb = g1 - g0

    const K *sk = (const K *)a.sk;
    const V *sv = HAS_V ? (const V *)a.sv : nullptr;
    // stage A's share at [0, ca) and B's at [ca, ca + cb), coalesced
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const uint32_t e = j * THREADS + t;
        if (e < ca + cb) {
            const uint32_t s = e < ca ? a0 + e : b0 + (e - ca);
            s_k[lds_slot<ITEMS>(e)] = sk[s];
            if constexpr (HAS_V)
                s_v[lds_slot<ITEMS>(e)] = sv[s];
        }
    }
    __syncthreads();

    const uint32_t o = t * ITEMS;
    K key[ITEMS];
    V val[HAS_V ? ITEMS : 1];
    uint32_t src[ITEMS];
    merge_chains<K, ITEMS, CHAINS, ITEMS>(s_k, 0, ca, cb, min(o, ca + cb), key, src);
    if constexpr (HAS_V) {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j)
            val[j] = o + j < ca + cb ? s_v[lds_slot<ITEMS>(src[j])] : (V)0;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        if (o + j < ca + cb) {
            s_k[lds_slot<ITEMS>(o + j)] = key[j];
            if constexpr (HAS_V)
                s_v[lds_slot<ITEMS>(o + j)] = val[j];
        }
    }
    __syncthreads();
    K *dk = (K *)a.dk + g0;
    V *dv = HAS_V ? (V *)a.dv + g0 : nullptr;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const uint32_t e = j * THREADS + t;
        if (e < ca + cb) {
            dk[e] = map_out(s_k[lds_slot<ITEMS>(e)], a.map_store);
            if constexpr (HAS_V)
                dv[e] = s_v[lds_slot<ITEMS>(e)];
        }
    }
}

// Host-side table of the merge sort's kernels for one kind.
struct MergeOps {
    int tile;       // elements per tile sort
    int pass_tile;  // outputs per merge-pass workgroup
    void (*tile_sort)(const MergeTileArgs &, uint32_t grid, hipStream_t);
    void (*split)(const MergeLevelArgs &, uint32_t grid, hipStream_t);
    void (*pass)(const MergeLevelArgs &, uint32_t grid, hipStream_t);
};

const MergeOps &merge_ops(int key_bytes, bool has_values);

}  // namespace rs
