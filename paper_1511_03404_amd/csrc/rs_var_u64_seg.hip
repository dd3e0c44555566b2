// Segmented-sort kernels of every compiled configuration, u64 keys.
#include "rs_configs.h"
#include "rs_ops.h"

namespace rs {

#define RS_KEYS_OPS(R, T, I) SegLaunch<uint64_t, false, R, T, I>::ops(),
#define RS_PAIRS_OPS(R, T, I) SegLaunch<uint64_t, true, R, T, I>::ops(),

const SegOps *seg_ops_u64(bool has_values, int *count)
{
    static const SegOps keys[] = {RS_SEG_CONFIGS_U64_KEYS(RS_KEYS_OPS)};
    static const SegOps pairs[] = {RS_SEG_CONFIGS_U64_PAIRS(RS_PAIRS_OPS)};
    if (has_values) {
        *count = (int)(sizeof pairs / sizeof pairs[0]);
        return pairs;
    }
    *count = (int)(sizeof keys / sizeof keys[0]);
    return keys;
}

}  // namespace rs
