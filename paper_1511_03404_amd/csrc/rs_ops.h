// Host-side tables of the compiled digit-pass configurations.  Each entry
// enqueues the kernels of one configuration (digit width, tile shape); the
// entries follow the order of the lists in rs_configs.h.  The kernels are
// instantiated in four translation units (32/64-bit keys x plain/segmented)
// that compile in parallel.
#pragma once

#include "rs_kernels.h"

namespace rs {

struct SortOps {
    int r;        // digit bits
    int threads;  // workgroup size of the digit pass
    int items;    // elements per thread
    int tile;     // threads x items
    int d;        // digit passes
    void (*hist)(const HistArgs &, uint32_t grid, hipStream_t);
    void (*plan)(const PlanArgs &, hipStream_t);
    void (*pass)(const PassArgs &, uint32_t grid, hipStream_t);
    const void *pass_kernel;  // for occupancy queries
};

struct SegOps {
    int r, threads, items, tile, d;
    void (*hist)(const SegHistArgs &, uint32_t grid, hipStream_t);
    void (*scan)(const SegHistArgs &, uint32_t grid, hipStream_t);
    void (*pass)(const SegPassArgs &, uint32_t grid, hipStream_t);
    const void *hist_kernel, *scan_kernel, *pass_kernel;
};

// Tables of the plain and segmented sorts for 32- and 64-bit keys.
const SortOps *sort_ops_u32(bool has_values, int *count);
const SortOps *sort_ops_u64(bool has_values, int *count);
const SegOps *seg_ops_u32(bool has_values, int *count);
const SegOps *seg_ops_u64(bool has_values, int *count);

template <typename K, bool HAS_V, int R, int THREADS, int ITEMS>
struct SortLaunch {
    using C = PassCfg<R, THREADS, ITEMS>;
    static void hist(const HistArgs &a, uint32_t grid, hipStream_t s)
    {
        hipLaunchKernelGGL((k_hist<K, R>), dim3(grid), dim3(kHistThreads), 0, s, a);
    }
    static void plan(const PlanArgs &a, hipStream_t s)
    {
        hipLaunchKernelGGL((k_plan<K, R>), dim3(1), dim3(kRadix * plan_groups<K, R>()), 0, s, a);
    }
    static void pass(const PassArgs &a, uint32_t grid, hipStream_t s)
    {
        hipLaunchKernelGGL((k_pass<K, K, HAS_V, C>), dim3(grid), dim3(THREADS), 0, s, a);
    }
    static SortOps ops()
    {
        return SortOps{R, THREADS, ITEMS, C::kTile, num_passes<K, R>(), &hist, &plan, &pass,
                       (const void *)k_pass<K, K, HAS_V, C>};
    }
};

template <typename K, bool HAS_V, int R, int THREADS, int ITEMS>
struct SegLaunch {
    using C = PassCfg<R, THREADS, ITEMS>;
    static void hist(const SegHistArgs &a, uint32_t grid, hipStream_t s)
    {
        hipLaunchKernelGGL((k_seg_hist<K, R>), dim3(grid), dim3(kSegHistThreads), 0, s, a);
    }
    static void scan(const SegHistArgs &a, uint32_t grid, hipStream_t s)
    {
        hipLaunchKernelGGL((k_seg_scan<K, R>), dim3(grid), dim3(256), 0, s, a);
    }
    static void pass(const SegPassArgs &a, uint32_t grid, hipStream_t s)
    {
        hipLaunchKernelGGL((k_seg_pass<K, K, HAS_V, C>), dim3(grid), dim3(THREADS), 0, s, a);
    }
    static SegOps ops()
    {
        return SegOps{R,
                      THREADS,
                      ITEMS,
                      C::kTile,
                      num_passes<K, R>(),
                      &hist,
                      &scan,
                      &pass,
                      (const void *)k_seg_hist<K, R>,
                      (const void *)k_seg_scan<K, R>,
                      (const void *)k_seg_pass<K, K, HAS_V, C>};
    }
};

}  // namespace rs
