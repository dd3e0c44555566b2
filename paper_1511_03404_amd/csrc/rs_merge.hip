// Merge-sort kernels of every key kind (32/64-bit keys, with and without
// values) and their launch table.
#include "rs_merge.h"

namespace rs {

template <typename K, bool HAS_V>
struct MergeLaunch {
    using S = MergeShape<K, HAS_V>;
    static void tile_sort(const MergeTileArgs &a, uint32_t grid, hipStream_t s)
    {
        hipLaunchKernelGGL((k_merge_tile<K, K, HAS_V, S::kTileThreads, S::kTileItems, S::kTileChains>), dim3(grid),
                           dim3(S::kTileThreads), 0, s, a);
    }
    static void split(const MergeLevelArgs &a, uint32_t grid, hipStream_t s)
    {
        hipLaunchKernelGGL((k_merge_split<K, S::kPassTile>), dim3(grid), dim3(256), 0, s, a);
    }
    static void pass(const MergeLevelArgs &a, uint32_t grid, hipStream_t s)
    {
        hipLaunchKernelGGL((k_merge_pass<K, K, HAS_V, S::kPassThreads, S::kPassItems, S::kPassChains>), dim3(grid),
                           dim3(S::kPassThreads), 0, s, a);
    }
    static MergeOps ops() { return MergeOps{S::kTile, S::kPassTile, &tile_sort, &split, &pass}; }
};

const MergeOps &merge_ops(int key_bytes, bool has_values)
{
    static const MergeOps table[4] = {MergeLaunch<uint32_t, false>::ops(),
                                      MergeLaunch<uint32_t, true>::ops(),
                                      MergeLaunch<uint64_t, false>::ops(),
                                      MergeLaunch<uint64_t, true>::ops()};
    return table[(key_bytes == 8 ? 2 : 0) + (has_values ? 1 : 0)];
}

}  // namespace rs
