// Bitonic sorting network (paper, Section 2.1; Batcher) for the tiny
// segments of a segmented sort: one wave per segment of up to 1024
// elements, held in registers as 64 lanes x R slots (element e = j * 64 +
// lane in slot j), R = 1, 2, ..., 16 by the segment's size.
//
// Stage k = 2, 4, ..., 64 R builds sorted runs of length k; its steps of
// distance s = k/2, ..., 1 compare element e with e XOR s and order each
// pair ascending when bit k of e is clear, descending when it is set.  A
// distance of 64 or more pairs two slots of the same lane; a smaller one
// pairs the same slot of two lanes (a cross-lane shuffle).
//
// The network alone is not stable; every element is the pair (key, position
// in the segment), compared lexicographically, so all elements differ and
// the sorted order is the stable sort.  Values do not travel through the
// network: each output gathers its value by the position it carries.  Slots
// past the segment hold a padding element greater than every real one.
#pragma once

#include "rs_block.h"
#include "rs_device.h"

namespace rs {

// Largest segment the network sorts (64 lanes x 16 slots).
constexpr uint32_t kTinyMax = 1024;

// (key, position) as one comparable word: 32-bit keys pack into a 64-bit
// integer; 64-bit keys keep the position beside the key.
template <typename K>
struct BitonicElem;

template <>
struct BitonicElem<uint32_t> {
    using T = uint64_t;
    static __device__ __forceinline__ T make(uint32_t k, uint32_t pos)
    {
        return ((uint64_t)k << 32) | pos;
    }
    static __device__ __forceinline__ T pad() { return ~0ull; }
    static __device__ __forceinline__ uint32_t key(T e) { return (uint32_t)(e >> 32); }
    static __device__ __forceinline__ uint32_t pos(T e) { return (uint32_t)e; }
    static __device__ __forceinline__ bool less(T a, T b) { return a < b; }
    static __device__ __forceinline__ T sel(bool c, T a, T b) { return c ? a : b; }
    static __device__ __forceinline__ T shfl_xor(T e, uint32_t s)
    {
        return __shfl_xor((unsigned long long)e, (int)s);
    }
};

template <>
struct BitonicElem<uint64_t> {
    struct T {
        uint64_t k;
        uint32_t p;
    };
    static __device__ __forceinline__ T make(uint64_t k, uint32_t pos) { return T{k, pos}; }
    static __device__ __forceinline__ T pad() { return T{~0ull, ~0u}; }
    static __device__ __forceinline__ uint64_t key(T e) { return e.k; }
    static __device__ __forceinline__ uint32_t pos(T e) { return e.p; }
    static __device__ __forceinline__ bool less(T a, T b)
    {
        return a.k < b.k || (a.k == b.k && a.p < b.p);
    }
    // field by field: a select of the whole struct would go through memory
    static __device__ __forceinline__ T sel(bool c, T a, T b)
    {
        return T{c ? a.k : b.k, c ? a.p : b.p};
    }
    static __device__ __forceinline__ T shfl_xor(T e, uint32_t s)
    {
        return T{(uint64_t)__shfl_xor((unsigned long long)e.k, (int)s),
                 (uint32_t)__shfl_xor((int)e.p, (int)s)};
    }
};

struct TinyArgs {
    const void *kin;
    const void *vin;
    void *kout;
    void *vout;
    const SegRange *list;     // the tiny segments (2 .. kTinyMax elements)
    const uint32_t *list_len; // their number (a device counter)
    uint32_t *claim;          // claim counter, zero at launch
    uint32_t kmap;            // key order: applied on load, undone on store
};

template <typename K, typename V, bool HAS_V, int R>
__device__ __forceinline__ void bitonic_wave(const TinyArgs &a, uint64_t start, uint32_t m,
                                             uint32_t lane)
{
    using E = BitonicElem<K>;
    using T = typename E::T;
    constexpr uint32_t N = kWave * R;
    const K *kin = (const K *)a.kin + start;

    K raw[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const uint32_t e = j * kWave + lane;
        raw[j] = e < m ? kin[e] : (K)0;
    }
    T x[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const uint32_t e = j * kWave + lane;
        x[j] = E::sel(e < m, E::make(map_in(raw[j], a.kmap), e), E::pad());
    }

    for (uint32_t k = 2; k <= N; k <<= 1) {
        // distances of 64 and more: two slots of this lane
#pragma unroll
        for (int sr = R / 2; sr >= 1; sr >>= 1) {
            if ((uint32_t)sr * kWave < k) {
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    if (j & sr)
                        continue;
                    const bool up = ((j * kWave + lane) & k) == 0;
                    const T lo = x[j], hi = x[j | sr];
                    const bool sw = up ? E::less(hi, lo) : E::less(lo, hi);
                    x[j] = E::sel(sw, hi, lo);
                    x[j | sr] = E::sel(sw, lo, hi);
                }
            }
        }
        // distances below 64: the same slot of lane XOR s
        for (uint32_t s = min(k >> 1, (uint32_t)kWave / 2); s >= 1; s >>= 1) {
            const bool lower = (lane & s) == 0;
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const bool up = ((j * kWave + lane) & k) == 0;
                const T y = E::shfl_xor(x[j], s);
                // the lower element of an ascending pair keeps the smaller
                const bool take_y = (lower == up) == E::less(y, x[j]);
                x[j] = E::sel(take_y, y, x[j]);
            }
        }
    }

    // every value is read before any is written (in place: vin == vout)
    V val[HAS_V ? R : 1];
    if constexpr (HAS_V) {
        const V *vin = (const V *)a.vin + start;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const uint32_t e = j * kWave + lane;
            val[j] = e < m ? vin[E::pos(x[j])] : (V)0;
        }
    }
    K *kout = (K *)a.kout + start;
    V *vout = HAS_V ? (V *)a.vout + start : nullptr;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const uint32_t e = j * kWave + lane;
        if (e < m) {
            kout[e] = map_out((K)E::key(x[j]), a.kmap);
            if constexpr (HAS_V)
                vout[e] = val[j];
        }
    }
}

// Persistent workgroups of 4 waves; each wave claims one tiny segment at a
// time until the list is exhausted.
template <typename K, typename V, bool HAS_V>
__global__ __launch_bounds__(256) void k_seg_bitonic(TinyArgs a)
{
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t len = *a.list_len;
    while (true) {
        uint32_t item = 0;
        if (lane == 0)
            item = atomicAdd(a.claim, 1u);
        item = (uint32_t)__shfl((int)item, 0);
        if (item >= len)
            break;
        const uint64_t start = a.list[item].start;
        const uint32_t m = a.list[item].size;
        if (m <= 64)
            bitonic_wave<K, V, HAS_V, 1>(a, start, m, lane);
        else if (m <= 128)
            bitonic_wave<K, V, HAS_V, 2>(a, start, m, lane);
        else if (m <= 256)
            bitonic_wave<K, V, HAS_V, 4>(a, start, m, lane);
        else if (m <= 512)
            bitonic_wave<K, V, HAS_V, 8>(a, start, m, lane);
        else
            bitonic_wave<K, V, HAS_V, 16>(a, start, m, lane);
    }
}

}  // namespace rs
