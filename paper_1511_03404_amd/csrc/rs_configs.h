// The compiled configurations of the digit-pass kernels, per key type and
// with or without values: X(R, THREADS, ITEMS) = R-bit digits, tiles of
// THREADS x ITEMS elements.  The first entry of each list is the default;
// the others are what the tuner may choose (every digit width 4..7 at the
// default tile, other tile shapes at 8 bits, and 11-bit digits).  The order is the index
// of a configuration in the C-ABI (rs_config_get, rs_tune_set).
//
// Limits: a tile's key staging (THREADS x ITEMS x key bytes) must hold the
// per-wave lane-mask tables (ITEMS >= 2^R / 32) and, with the counters, fit
// the 160 KB of LDS of a gfx950 workgroup; ITEMS keys and values per thread
// must fit the registers at THREADS threads per workgroup.
#pragma once

#define RS_SEG_CONFIGS_U32_KEYS(X)                                                       \
    X(8, 1024, 16) X(4, 1024, 16) X(5, 1024, 16) X(6, 1024, 16) X(7, 1024, 16)          \
    X(8, 512, 16) X(8, 1024, 8) X(8, 256, 16) X(8, 512, 32)

#define RS_SEG_CONFIGS_U32_PAIRS(X) RS_SEG_CONFIGS_U32_KEYS(X)

#define RS_SEG_CONFIGS_U64_KEYS(X)                                                       \
    X(8, 1024, 16) X(4, 1024, 16) X(5, 1024, 16) X(6, 1024, 16) X(7, 1024, 16)          \
    X(8, 512, 16) X(8, 1024, 8) X(8, 256, 16) X(8, 512, 24)

// 64-bit pairs: 16 keys and 16 values per thread need more registers than
// 1024 threads leave, so the default tile is 512 x 16.
#define RS_SEG_CONFIGS_U64_PAIRS(X)                                                      \
    X(8, 512, 16) X(4, 512, 16) X(5, 512, 16) X(6, 512, 16) X(7, 512, 16)               \
    X(8, 1024, 8) X(8, 256, 16) X(8, 512, 8) X(8, 256, 32)

// The plain sort also has wide digits (11 bits, the layout of rs_wide.h):
// three passes for 32-bit keys, six for 64-bit keys; and for 32-bit keys
// alone, whose 16384-key tiles use 64 KB of staging, tiles of 24576 keys
// (the built-in choice from 2^26 keys).  They follow the segmented lists,
// so an index below the segmented list's length names the same
// configuration in both.
#define RS_CONFIGS_U32_KEYS(X) RS_SEG_CONFIGS_U32_KEYS(X) X(11, 1024, 16) X(8, 1024, 24)
#define RS_CONFIGS_U32_PAIRS(X) RS_SEG_CONFIGS_U32_PAIRS(X) X(11, 1024, 16)
#define RS_CONFIGS_U64_KEYS(X) RS_SEG_CONFIGS_U64_KEYS(X) X(11, 1024, 16)
#define RS_CONFIGS_U64_PAIRS(X) RS_SEG_CONFIGS_U64_PAIRS(X) X(11, 1024, 8)
