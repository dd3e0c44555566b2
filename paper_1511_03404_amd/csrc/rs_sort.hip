// LSD radix sort for gfx950 (MI355X) behind the C-ABI declared in rs.h:
// argument validation, workspace layout, the per-context tune table and the
// launch sequences.  The digit-pass kernels (paper, Section 2.6) are in
// rs_kernels.h, instantiated for every configuration of rs_configs.h in the
// rs_var_*.hip units; the one-workgroup LDS sort is in rs_block.h.
//
// A plain sort of n elements, n above the one-workgroup limit:
//   k_init      zero the control block and the digit histograms (sorts whose
//               k_hist adds into one histogram; small sorts skip it)
//   k_hist      all digit histograms in one read; clears the look-back words
//   k_plan      digit_base scans, skipped passes, buffer ping-pong
//   k_pass x d  one sweep per digit
//   k_finalize  in-place sorts with an odd number of moving passes only
//
// Everything after argument validation is enqueued on the caller's stream
// with no host synchronisation.
#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "rs.h"
#include "rs_bitonic.h"
#include "rs_block.h"
#include "rs_configs.h"
#include "rs_device.h"
#include "rs_merge.h"
#include "rs_ops.h"
#include "rs_segmented.h"

namespace rs {

// ---------------------------------------------------------------------------
// k_init: clear the control block and the histograms.

__global__ void k_init(uint32_t *ctrl, uint32_t *hist, int hist_words)
{
    for (int i = threadIdx.x; i < kCtrlWords; i += blockDim.x)
        ctrl[i] = 0;
    for (int i = threadIdx.x; i < hist_words; i += blockDim.x)
        hist[i] = 0;
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
__global__ void k_finalize(Bufs b, uint32_t n, const uint32_t *ctrl, uint32_t kmap)
{
    if (ctrl[kCtrlFinal] != 1u)
        return;
    const K *tk = (const K *)b.tmp_k;
    K *ok = (K *)b.out_k;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        ok[i] = map_out(tk[i], kmap);
        if constexpr (HAS_V)
            ((V *)b.out_v)[i] = ((const V *)b.tmp_v)[i];
    }
}

// k_copy_ceiling: a plain copy of 16-byte words, each thread with ITEMS loads
// in flight before its stores; the measuring stick of the copy ceiling.
template <int THREADS, int ITEMS>
__global__ __launch_bounds__(THREADS) void k_copy_ceiling(const uint4 *src, uint4 *dst,
                                                          uint64_t nvec)
{
    const uint64_t per_block = (uint64_t)THREADS * ITEMS;
    for (uint64_t base = (uint64_t)blockIdx.x * per_block; base < nvec;
         base += (uint64_t)gridDim.x * per_block) {
        uint4 v[ITEMS];
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint64_t i = base + (uint64_t)j * THREADS + threadIdx.x;
            if (i < nvec)
                v[j] = src[i];
        }
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint64_t i = base + (uint64_t)j * THREADS + threadIdx.x;
            if (i < nvec)
                dst[i] = v[j];
        }
    }
}

}  // namespace rs

// ===========================================================================
// Host side: validation, workspace layout, launches.

using namespace rs;

// Size classes of the tune table: ceil(log2 n) = 0 .. 39.
constexpr int kTuneClasses = 40;

struct ProfRecord {
    const char *name;
    int tag;
    size_t ev;  // index of the first of two events in the pool
};

// Scratch the context allocates for calls made with ws == NULL: one buffer
// per stream, so that sorts on different streams never share one.
struct OwnWorkspace {
    hipStream_t stream;
    void *ptr;
    size_t bytes;
};

struct rs_context {
    int device = 0;
    std::vector<OwnWorkspace> own;
    // per-kernel timing (rs_profile_*)
    bool prof = false;
    int prof_tag = 0;
    std::vector<ProfRecord> recs;
    std::vector<hipEvent_t> events;  // grow-only pool, reused after a reset
    size_t events_used = 0;
    uint32_t cus = 0;  // compute units, queried on first use
    // tune table: configuration index per [64-bit keys][values][segmented]
    // [ceil(log2 n)], -1 = the default (index 0)
    int8_t tune[2][2][2][kTuneClasses];
    // segments of 2 .. tiny_cap elements go to the bitonic network (0: none)
    uint32_t tiny_cap = kTinyMax;
    // bound of the waits on other workgroups, and test-only stalls
    uint32_t spin_limit = kDefaultSpinLimit;
    uint32_t stall = 0;
    rs_context() { memset(tune, -1, sizeof tune); }
};

// ceil(log2 n) for n >= 1 (0 for n <= 1).
static int size_class(uint64_t n)
{
    int c = 0;
    while (c < 63 && ((uint64_t)1 << c) < n)
        ++c;
    return c;
}

static const SortOps *sort_table(int key_bytes, bool has_values, int *count)
{
    return key_bytes == 4 ? sort_ops_u32(has_values, count) : sort_ops_u64(has_values, count);
}

static const SegOps *seg_table(int key_bytes, bool has_values, int *count)
{
    return key_bytes == 4 ? seg_ops_u32(has_values, count) : seg_ops_u64(has_values, count);
}

// The configuration the context's tune table selects (the first one of the
// table unless set otherwise).
// The configuration a size class gets when its table entry is unset: what
// the autotuner selected on MI355X for plain sorts of uniform keys.  Tiles
// of 8192 elements (1024 x 8) up to 2^21 elements (all sizes for 64-bit
// pairs, as 512 x 8 up to 2^19): a small sort has few tiles, and a tile's
// latency, not HBM, sets the pass time.  Above, the list's default (index
// 0), except 32-bit keys without values from 2^26 keys on: tiles of
// 1024 x 24 (a pass 6.7% faster at 2^26, 3% slower at 2^25, where fewer
// tiles are in flight).  Looked up by shape, so a different list falls
// back to index 0.
static int default_index(int key_bytes, bool has_values, bool segmented, int c)
{
    if (segmented)
        return 0;
    int threads = 0, items = 0;
    if (key_bytes == 8 && has_values) {
        if (c <= 19)
            threads = 512, items = 8;
        else
            threads = 1024, items = 8;
    } else if (c <= 21) {
        threads = 1024, items = 8;
    } else if (key_bytes == 4 && !has_values && c >= 26) {
        threads = 1024, items = 24;
    }
    if (threads == 0)
        return 0;
    int count = 0;
    const SortOps *t = sort_table(key_bytes, has_values, &count);
    for (int i = 0; i < count; ++i)
        if (t[i].r == 8 && t[i].threads == threads && t[i].items == items)
            return i;
    return 0;
}

static int tuned_index(const rs_context *ctx, int key_bytes, bool has_values, bool segmented,
                       uint64_t n, int count)
{
    const int c = std::min(size_class(n), kTuneClasses - 1);
    const int i = ctx->tune[key_bytes == 8][has_values][segmented][c];
    if (i >= 0 && i < count)
        return i;
    const int d = default_index(key_bytes, has_values, segmented, c);
    return d < count ? d : 0;
}

static const SortOps &pick_sort(const rs_context *ctx, int key_bytes, bool has_values, uint64_t n)
{
    int count = 0;
    const SortOps *t = sort_table(key_bytes, has_values, &count);
    return t[tuned_index(ctx, key_bytes, has_values, false, n, count)];
}

static const SegOps &pick_seg(const rs_context *ctx, int key_bytes, bool has_values,
                              uint64_t total)
{
    int count = 0;
    const SegOps *t = seg_table(key_bytes, has_values, &count);
    return t[tuned_index(ctx, key_bytes, has_values, true, total, count)];
}

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
    uint32_t bins;  // 2^r
    uint32_t tile;
    uint64_t tiles;
    uint64_t off_ctrl, off_hist, off_base, off_part, off_status, off_tmp_k, off_tmp_v, total;
    uint32_t hist_blocks;   // workgroups of k_hist
    bool hist_fine;         // k_hist counts key by key (small sorts), not in batches
    uint32_t parts;         // hist_blocks if k_hist writes row blocks, else 0
    uint64_t status_bytes;  // look-back words, claim counters, group aggregates of all passes
    uint64_t claim_words;
    uint64_t groups;        // tile groups of the two-level look-back
};

static Layout make_layout(int key_bytes, bool has_values, uint64_t n, const SortOps &op)
{
    Layout L{};
    L.d = op.d;
    L.bins = 1u << op.r;
    L.tile = (uint32_t)op.tile;
    L.tiles = (n + L.tile - 1) / L.tile;
    uint64_t o = 0;
    L.off_ctrl = o;
    o = align_up(o + kCtrlWords * 4, 256);
    L.off_hist = o;
    o = align_up(o + (uint64_t)L.d * L.bins * 4, 256);
    L.off_base = o;
    o = align_up(o + (uint64_t)L.d * L.bins * 4, 256);
    // k_hist: batches of 16384 keys per workgroup; up to 2^16 keys, one
    // workgroup per 4096 keys, 4 per thread (a small sort's histogram then
    // takes one short count, not one full batch: 1-3% of a 2^15-2^16 sort;
    // with 8-16 keys per thread it is slower than the batches)
    L.hist_fine = n <= 65536;
    L.hist_blocks = L.hist_fine
                        ? (uint32_t)std::max<uint64_t>(
                              1, std::min<uint64_t>(kHistPartsMax, (n + 4095) / 4096))
                        : (uint32_t)std::min<uint64_t>(512, (n + 16383) / 16384);
    L.parts = L.hist_blocks <= kHistPartsMax ? L.hist_blocks : 0u;
    L.off_part = o;
    o = align_up(o + (uint64_t)L.parts * L.d * L.bins * 4, 256);
    L.off_status = o;
    L.claim_words = kXcdSlots * (1 + L.tiles);  // per-XCD counters + per-XCD group lists
    L.groups = (L.tiles + kClaimGroup - 1) / kClaimGroup;
    L.status_bytes = align_up(
        (uint64_t)L.d * (L.tiles * L.bins + L.claim_words + L.groups * L.bins) * 4, 16);
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

// Workgroups of `kernel` that fit on one CU at once (at least 1).
static uint32_t resident_blocks(const void *kernel, int threads)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess ||
        per_cu < 1) {
        (void)hipGetLastError();
        per_cu = 1;
    }
    return (uint32_t)per_cu;
}

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

static OwnWorkspace *own_workspace(rs_context *ctx, hipStream_t s)
{
    for (OwnWorkspace &o : ctx->own)
        if (o.stream == s)
            return &o;
    return nullptr;
}

// The caller's workspace, or the context's own one for this stream, grown
// to `need` bytes.  An own buffer is only ever used by sorts on its stream,
// so growing it waits for that stream alone before the old one is freed.
static rs_status get_workspace(rs_context *ctx, void *ws, uint64_t need, hipStream_t s,
                               void **out)
{
    if (ws) {
        *out = ws;
        return RS_OK;
    }
    OwnWorkspace *o = own_workspace(ctx, s);
    if (!o) {
        ctx->own.push_back({s, nullptr, 0});
        o = &ctx->own.back();
    }
    if (o->bytes < need) {
        if (o->ptr) {
            (void)hipStreamSynchronize(s);
            (void)hipFree(o->ptr);
            o->ptr = nullptr;
            o->bytes = 0;
        }
        if (hipMalloc(&o->ptr, need) != hipSuccess) {
            (void)hipGetLastError();
            o->ptr = nullptr;
            return fail(RS_ERR_OUT_OF_MEMORY, "could not allocate %llu bytes of scratch",
                        (unsigned long long)need);
        }
        o->bytes = need;
    }
    *out = o->ptr;
    return RS_OK;
}

// Pointer checks shared by every sort (n > 0).
static rs_status validate_data(int key_bytes, const void *kin, const void *vin, void *kout,
                               void *vout, bool has_values, uint64_t n)
{
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
    return RS_OK;
}

// Checks of a caller's workspace of `need` bytes (none given: the context's own).
static rs_status validate_ws(int key_bytes, const void *kin, const void *vin, const void *kout,
                             const void *vout, bool has_values, uint64_t n, const void *ws,
                             size_t ws_bytes, uint64_t need)
{
    if (!ws)
        return RS_OK;
    const uint64_t bytes = n * (uint64_t)key_bytes;
    if ((uintptr_t)ws & 255)
        return fail(RS_ERR_INVALID_ARGUMENT, "workspace must be 256-byte aligned");
    if (ws_bytes < need)
        return fail(RS_ERR_INVALID_ARGUMENT, "workspace of %zu bytes is below the %llu needed",
                    ws_bytes, (unsigned long long)need);
    if (overlaps(ws, need, kin, bytes) || overlaps(ws, need, kout, bytes) ||
        (has_values && (overlaps(ws, need, vin, bytes) || overlaps(ws, need, vout, bytes))))
        return fail(RS_ERR_INVALID_ARGUMENT, "workspace overlaps a data array");
    return RS_OK;
}

static rs_status validate_sort(const rs_context *ctx, int key_bytes, const void *kin,
                               const void *vin, void *kout, void *vout, bool has_values,
                               uint64_t n, const void *ws, size_t ws_bytes, const SortOps &op,
                               Layout *L)
{
    (void)ctx;
    if (n >= RS_MAX_ELEMENTS)
        return fail(RS_ERR_UNSUPPORTED, "n = %llu exceeds the limit of 2^30 - 1 elements",
                    (unsigned long long)n);
    *L = make_layout(key_bytes, has_values, n, op);
    if (n == 0)
        return RS_OK;
    rs_status st = validate_data(key_bytes, kin, vin, kout, vout, has_values, n);
    if (st != RS_OK)
        return st;
    return validate_ws(key_bytes, kin, vin, kout, vout, has_values, n, ws, ws_bytes, L->total);
}

template <typename K, bool HAS_V>
static const char *pass_name()
{
    if (sizeof(K) == 4)
        return HAS_V ? "k_pass_u32_pairs" : "k_pass_u32_keys";
    return HAS_V ? "k_pass_u64_pairs" : "k_pass_u64_keys";
}

// limit >= 0 and hist_out are for the per-kernel test entry point only:
// stop after `limit` digit positions (the state after that many passes lands
// in the output), copy the digit histograms to hist_out, and always take the
// multi-kernel path.
template <typename K, bool HAS_V>
static rs_status run_sort(rs_context *ctx, const K *kin, const K *vin, K *kout, K *vout,
                          uint64_t n, void *ws, size_t ws_bytes, void *stream, uint32_t kmap = 0,
                          int limit = -1, uint32_t *hist_out = nullptr)
{
    if (!ctx)
        return fail(RS_ERR_INVALID_ARGUMENT, "ctx is NULL");
    const SortOps &op = pick_sort(ctx, sizeof(K), HAS_V, n);
    Layout L;
    rs_status st =
        validate_sort(ctx, sizeof(K), kin, vin, kout, vout, HAS_V, n, ws, ws_bytes, op, &L);
    if (st != RS_OK || n == 0)
        return st;
    DeviceGuard guard(ctx->device);
    if (!guard.ok)
        return fail(RS_ERR_DEVICE, "cannot select HIP device %d", ctx->device);
    hipStream_t s = (hipStream_t)stream;
    using B = BlockShape<K, HAS_V>;
    const bool debug = limit >= 0 || hist_out != nullptr;
    if (n <= (uint64_t)B::kMediumCap && !debug) {
        // the whole array fits one workgroup's LDS: one launch, all passes.
        // The workspace is not needed; its error word is cleared.
        uint32_t *err_clear = nullptr;
        if (ws) {
            err_clear = (uint32_t *)ws + kCtrlError;
        } else if (OwnWorkspace *o = own_workspace(ctx, s)) {
            if (o->ptr)
                err_clear = (uint32_t *)o->ptr + kCtrlError;
        }
        BlockArgs ba{kin, vin, kout, vout, nullptr, nullptr, nullptr, n, kmap, err_clear};
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
    st = get_workspace(ctx, ws, L.total, (hipStream_t)stream, &w);
    if (st != RS_OK)
        return st;
    char *wb = (char *)w;
    uint32_t *ctrl = (uint32_t *)(wb + L.off_ctrl);
    uint32_t *hist = (uint32_t *)(wb + L.off_hist);
    uint32_t *base = (uint32_t *)(wb + L.off_base);
    uint32_t *status = (uint32_t *)(wb + L.off_status);
    // in place if either array is (the first moving pass must not write its
    // own input); an array not sorted in place is copied when no pass moves
    const bool keys_in_place = (const void *)kin == (const void *)kout;
    const bool vals_in_place = HAS_V && vin == vout;  // keys only: no values to place
    const bool in_place = keys_in_place || vals_in_place;
    const int run_passes = limit >= 0 ? std::min(limit, L.d) : L.d;

    Bufs b{kin, vin, kout, vout, wb + L.off_tmp_k, HAS_V ? (void *)(wb + L.off_tmp_v) : nullptr};

    // the histogram that k_hist adds into starts cleared; with row blocks
    // (small sorts) nothing needs clearing (k_plan clears the control block)
    if (!L.parts)
        launch(ctx, s, "k_init", [&] {
            hipLaunchKernelGGL(k_init, dim3(1), dim3(256), 0, s, ctrl, hist, (int)(L.d * L.bins));
        });

    HistArgs ha{};
    ha.keys = kin;
    ha.n = (uint32_t)n;
    const uint64_t mis = ((uintptr_t)kin & 15) / sizeof(K);
    ha.head = (uint32_t)std::min<uint64_t>(n, mis ? (16 / sizeof(K)) - mis : 0);
    ha.nvec = (uint32_t)((n - ha.head) / (16 / sizeof(K)));
    ha.hist = hist;
    ha.kmap = kmap;
    ha.status = (uint4 *)status;
    ha.status_vec = L.status_bytes / 16;
    uint32_t *part = (uint32_t *)(wb + L.off_part);
    ha.part = L.parts ? part : nullptr;
    ha.fine = L.hist_fine ? 1u : 0u;
    launch(ctx, s, sizeof(K) == 4 ? "k_hist_u32" : "k_hist_u64",
           [&] { op.hist(ha, L.hist_blocks, s); });

    PlanArgs pl{hist, part, L.parts, base, ctrl, (uint32_t)n, keys_in_place, vals_in_place,
                run_passes};
    launch(ctx, s, "k_plan", [&] { op.plan(pl, s); });
    // after k_plan: with row blocks, k_plan writes their sum into hist
    if (hist_out &&
        hipMemcpyAsync(hist_out, hist, (size_t)L.d * L.bins * 4, hipMemcpyDeviceToDevice, s) !=
            hipSuccess)
        return fail(RS_ERR_DEVICE, "histogram copy failed");

    // workgroups loop over claimed tiles: launch only what fits on the device
    // at once (more would start at the end just to find no work).  Tiles are
    // claimed in groups per XCD and workgroups are dealt to the XCDs in turn,
    // so a small sort launches up to one workgroup per tile on every XCD:
    // otherwise an XCD holding a group could have fewer workgroups than tiles
    // and process them one after another.  A pass of few tiles claims them
    // in arrival order: one workgroup per tile.  So do 32-bit keys without
    // values at every size (measured on MI355X at 2^25 and 2^26: 2-3.5%
    // faster in arrival order, while pairs and 64-bit keys are 3-18% faster
    // with the groups).
    const bool flat = L.tiles <= kFlatClaimTiles || (sizeof(K) == 4 && !HAS_V);
    const uint32_t pass_grid = (uint32_t)std::min<uint64_t>(
        flat ? L.tiles : L.tiles * kXcdSlots,
        (uint64_t)resident_blocks(op.pass_kernel, op.threads) * ctx_cus(ctx));
    // the passes of digit positions [0, run_passes); at least one is launched,
    // which copies the input when no pass moves data
    for (int p = 0; p < std::max(run_passes, 1); ++p) {
        PassArgs pa{};
        pa.b = b;
        pa.n = (uint32_t)n;
        pa.pass = p;
        pa.shift = p * op.r;
        pa.ctrl = ctrl;
        pa.digit_base = base + p * L.bins;
        pa.status = status + (uint64_t)p * L.tiles * L.bins;
        pa.claims = status + (uint64_t)L.d * L.tiles * L.bins + (uint64_t)p * L.claim_words;
        pa.gagg = status + (uint64_t)L.d * (L.tiles * L.bins + L.claim_words) +
                  (uint64_t)p * L.groups * L.bins;
        pa.num_tiles = (uint32_t)L.tiles;
        pa.num_groups = (uint32_t)((L.tiles + kClaimGroup - 1) / kClaimGroup);
        pa.flat = flat ? 1u : 0u;
        pa.kmap = kmap;
        pa.err = ctrl + kCtrlError;
        pa.spin_limit = ctx->spin_limit;
        pa.stall = ctx->stall;
        launch(ctx, s, pass_name<K, HAS_V>(), [&] { op.pass(pa, pass_grid, s); });
    }
    if (in_place) {
        const uint32_t blocks = (uint32_t)std::min<uint64_t>(4096, (n + 255) / 256);
        launch(ctx, s, "k_finalize", [&] {
            hipLaunchKernelGGL((k_finalize<K, K, HAS_V>), dim3(blocks), dim3(256), 0, s, b,
                               (uint32_t)n, (const uint32_t *)ctrl, kmap);
        });
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(RS_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return RS_OK;
}

// ---------------------------------------------------------------------------
// Merge sort host side: one tile-sort launch, then per merge level a split
// launch and a merge-pass launch, ping-ponging between the output and the
// scratch copy so that the last level writes the output.

struct MergeLayout {
    uint64_t tiles;       // tile sorts
    uint64_t pass_tiles;  // merge-pass workgroups per level
    int levels;           // merge levels: runs double from the tile size until >= n
    uint64_t off_split, off_tmp_k, off_tmp_v, total;
};

static MergeLayout make_merge_layout(int key_bytes, bool has_values, uint64_t n,
                                     const MergeOps &op)
{
    MergeLayout L{};
    L.tiles = (n + op.tile - 1) / op.tile;
    L.pass_tiles = (n + op.pass_tile - 1) / op.pass_tile;
    for (uint64_t w = op.tile; w < n; w *= 2)
        ++L.levels;
    uint64_t o = 0;
    L.off_split = o;
    o = align_up(o + (L.pass_tiles + 1) * 4, 256);
    L.off_tmp_k = o;
    o = align_up(o + n * key_bytes, 256);
    L.off_tmp_v = o;
    o = align_up(o + (has_values ? n * key_bytes : 0), 256);
    L.total = o;
    return L;
}

template <typename K, bool HAS_V>
static const char *merge_pass_name()
{
    if (sizeof(K) == 4)
        return HAS_V ? "k_merge_pass_u32_pairs" : "k_merge_pass_u32_keys";
    return HAS_V ? "k_merge_pass_u64_pairs" : "k_merge_pass_u64_keys";
}

template <typename K, bool HAS_V>
static rs_status run_merge(rs_context *ctx, const K *kin, const K *vin, K *kout, K *vout,
                           uint64_t n, void *ws, size_t ws_bytes, void *stream, uint32_t kmap)
{
    if (!ctx)
        return fail(RS_ERR_INVALID_ARGUMENT, "ctx is NULL");
    if (n >= RS_MAX_ELEMENTS)
        return fail(RS_ERR_UNSUPPORTED, "n = %llu exceeds the limit of 2^30 - 1 elements",
                    (unsigned long long)n);
    if (n == 0)
        return RS_OK;
    const MergeOps &op = merge_ops(sizeof(K), HAS_V);
    const MergeLayout L = make_merge_layout(sizeof(K), HAS_V, n, op);
    rs_status st = validate_data(sizeof(K), kin, vin, kout, vout, HAS_V, n);
    if (st != RS_OK)
        return st;
    st = validate_ws(sizeof(K), kin, vin, kout, vout, HAS_V, n, ws, ws_bytes, L.total);
    if (st != RS_OK)
        return st;
    DeviceGuard guard(ctx->device);
    if (!guard.ok)
        return fail(RS_ERR_DEVICE, "cannot select HIP device %d", ctx->device);
    hipStream_t s = (hipStream_t)stream;
    char *wb = nullptr;
    if (L.levels > 0) {
        void *w = nullptr;
        st = get_workspace(ctx, ws, L.total, (hipStream_t)stream, &w);
        if (st != RS_OK)
            return st;
        wb = (char *)w;
    }
    // buffers: 0 = output, 1 = scratch; the tile sort writes the one from
    // which an even or odd number of levels ends in the output
    K *bk[2] = {kout, wb ? (K *)(wb + L.off_tmp_k) : nullptr};
    K *bv[2] = {vout, (wb && HAS_V) ? (K *)(wb + L.off_tmp_v) : nullptr};
    int cur = L.levels & 1;
    MergeTileArgs ta{kin, vin, bk[cur], bv[cur], (uint32_t)n, kmap, L.levels == 0 ? kmap : 0u};
    launch(ctx, s, "k_merge_tile", [&] { op.tile_sort(ta, (uint32_t)L.tiles, s); });
    uint32_t *split = wb ? (uint32_t *)(wb + L.off_split) : nullptr;
    for (int lvl = 0; lvl < L.levels; ++lvl) {
        MergeLevelArgs la{};
        la.sk = bk[cur];
        la.sv = bv[cur];
        la.dk = bk[cur ^ 1];
        la.dv = bv[cur ^ 1];
        la.split = split;
        la.n = (uint32_t)n;
        la.w = (uint32_t)op.tile << lvl;
        la.tiles = (uint32_t)L.pass_tiles;
        la.map_store = lvl == L.levels - 1 ? kmap : 0u;
        launch(ctx, s, "k_merge_split",
               [&] { op.split(la, (uint32_t)((L.pass_tiles + 255) / 256), s); });
        launch(ctx, s, merge_pass_name<K, HAS_V>(),
               [&] { op.pass(la, (uint32_t)L.pass_tiles, s); });
        cur ^= 1;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(RS_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return RS_OK;
}

// ---------------------------------------------------------------------------
// Segmented sort host side.

static constexpr uint64_t kSegMaxTotal = (uint64_t)1 << 36;

struct SegLayout {
    int d;
    uint32_t bins;  // 2^r
    uint64_t max_tiles;
    uint64_t claim_words;
    uint64_t max_chunks;
    uint64_t off_ctrl, off_tiny, off_small, off_medium, off_large, off_base, off_tile_seg,
        off_status, status_bytes, off_tmp_k, off_tmp_v, total;
    uint64_t off_hist, off_chunk_seg, off_flags;
};

static SegLayout make_seg_layout(int key_bytes, bool has_values, uint64_t total, uint32_t nseg,
                                 const SegOps &op)
{
    SegLayout L{};
    L.d = op.d;
    L.bins = 1u << op.r;
    const uint64_t T = (uint64_t)op.tile;
    // every large segment adds at most one partial tile
    L.max_tiles = total / T + nseg + 1;
    L.claim_words = kXcdSlots * (1 + L.max_tiles);
    uint64_t o = 0;
    L.off_ctrl = o;
    o = align_up(o + kSegWords * 4, 256);
    L.off_tiny = o;
    o = align_up(o + (uint64_t)nseg * sizeof(SegRange), 256);
    L.off_small = o;
    o = align_up(o + (uint64_t)nseg * sizeof(SegRange), 256);
    L.off_medium = o;
    o = align_up(o + (uint64_t)nseg * sizeof(SegRange), 256);
    L.off_large = o;
    o = align_up(o + (uint64_t)nseg * sizeof(SegLarge), 256);
    L.off_base = o;
    o = align_up(o + (uint64_t)nseg * L.d * L.bins * 4, 256);
    L.off_flags = o;
    o = align_up(o + (uint64_t)nseg * 4, 256);
    L.off_tile_seg = o;
    o = align_up(o + L.max_tiles * 4, 256);
    L.max_chunks = total / kSegChunk + nseg + 1;
    L.off_chunk_seg = o;
    o = align_up(o + L.max_chunks * 4, 256);
    // zeroed region: look-back words, claim counters, segment histograms
    L.off_status = o;
    L.status_bytes = align_up((uint64_t)L.d * (L.max_tiles * L.bins + L.claim_words) * 4, 16);
    L.off_hist = L.off_status + L.status_bytes;
    L.status_bytes += align_up((uint64_t)nseg * L.d * L.bins * 4, 16);
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
                               void *ws, size_t ws_bytes, void *stream, uint32_t kmap = 0)
{
    if (!ctx)
        return fail(RS_ERR_INVALID_ARGUMENT, "ctx is NULL");
    if (total >= kSegMaxTotal)
        return fail(RS_ERR_UNSUPPORTED, "total exceeds 2^36 elements");
    if (HAS_V && (!vin || !vout))
        return fail(RS_ERR_INVALID_ARGUMENT, "values need both vals_in and vals_out");
    const SegOps &op = pick_seg(ctx, sizeof(K), HAS_V, total);
    const SegLayout L = make_seg_layout(sizeof(K), HAS_V, total, nseg, op);
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
    rs_status st = get_workspace(ctx, ws, L.total, (hipStream_t)stream, &w);
    if (st != RS_OK)
        return st;
    hipStream_t s = (hipStream_t)stream;
    char *wb = (char *)w;
    uint32_t *ctrl = (uint32_t *)(wb + L.off_ctrl);
    SegRange *tiny_list = (SegRange *)(wb + L.off_tiny);
    SegRange *small_list = (SegRange *)(wb + L.off_small);
    SegRange *medium_list = (SegRange *)(wb + L.off_medium);
    SegLarge *large = (SegLarge *)(wb + L.off_large);
    uint32_t *seg_base = (uint32_t *)(wb + L.off_base);
    uint32_t *seg_flags = (uint32_t *)(wb + L.off_flags);
    uint32_t *tile_seg = (uint32_t *)(wb + L.off_tile_seg);
    uint32_t *chunk_seg = (uint32_t *)(wb + L.off_chunk_seg);
    uint32_t *seg_hist = (uint32_t *)(wb + L.off_hist);
    uint32_t *status = (uint32_t *)(wb + L.off_status);
    void *tmp_k = wb + L.off_tmp_k;
    void *tmp_v = HAS_V ? (void *)(wb + L.off_tmp_v) : nullptr;
    using B = BlockShape<K, HAS_V>;
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
    SegClassifyArgs ca{offsets,   nseg,        total,     (uint32_t)L.max_tiles,
                       ctrl,      tiny_list,   small_list, medium_list,
                       large,     tile_seg,    chunk_seg, (uint32_t)L.max_chunks,
                       kin,       vin,         kout,      vout,
                       ctx->tiny_cap, (uint32_t)B::kSmallCap, (uint32_t)B::kMediumCap,
                       (uint32_t)op.tile};
    launch(ctx, s, "k_seg_classify", [&] {
        const uint32_t g = std::min<uint32_t>(1024, (nseg + 255) / 256);
        hipLaunchKernelGGL((k_seg_classify<K, HAS_V>), dim3(std::max(1u, g)), dim3(256), 0, s, ca);
    });
    // tiny, small and medium segments: persistent workgroups over the device lists
    auto grid_of = [&](const void *kernel, int threads) {
        return resident_blocks(kernel, threads) * cus;
    };
    if (ctx->tiny_cap > 0) {
        TinyArgs ta{kin, vin, kout, vout, tiny_list, ctrl + kSegTinyLen, ctrl + kSegTinyClaim,
                    kmap};
        auto kern = k_seg_bitonic<K, K, HAS_V>;
        const uint32_t g =
            std::min<uint32_t>(grid_of((const void *)kern, 256), (nseg + 3) / 4);
        launch(ctx, s, "k_seg_bitonic", [&] {
            hipLaunchKernelGGL(kern, dim3(std::max(1u, g)), dim3(256), 0, s, ta);
        });
    }
    {
        BlockArgs ba{kin, vin, kout, vout, small_list, ctrl + kSegSmallLen, ctrl + kSegSmallClaim,
                     0, kmap, nullptr};
        auto kern = k_block_sort<K, K, HAS_V, B::kSmallThreads, B::kItems>;
        const uint32_t g = std::min<uint32_t>(grid_of((const void *)kern, B::kSmallThreads), nseg);
        launch(ctx, s, "k_block_sort_small", [&] {
            hipLaunchKernelGGL(kern, dim3(g), dim3(B::kSmallThreads), 0, s, ba);
        });
    }
    {
        BlockArgs ba{kin, vin, kout, vout, medium_list, ctrl + kSegMediumLen,
                     ctrl + kSegMediumClaim, 0, kmap, nullptr};
        auto kern = k_block_sort<K, K, HAS_V, B::kMediumThreads, B::kItems>;
        const uint32_t g = std::min<uint32_t>(grid_of((const void *)kern, B::kMediumThreads), nseg);
        launch(ctx, s, "k_block_sort_medium", [&] {
            hipLaunchKernelGGL(kern, dim3(g), dim3(B::kMediumThreads), 0, s, ba);
        });
    }
    // large segments: per-segment histograms, then the batched digit passes.
    // Pass p writes the output when d - 1 - p is even, the scratch copy
    // otherwise, so the last pass lands in the output; in place (the first
    // pass may not write its own input) with an odd d, the passes start in
    // the scratch copy and the large segments are copied back at the end.
    {
        SegHistArgs ha{kin,      large,    chunk_seg, (uint32_t)L.max_chunks, ctrl,
                       seg_hist, seg_base, seg_flags, kmap};
        const uint32_t g = std::min<uint64_t>(grid_of(op.hist_kernel, kSegHistThreads), L.max_chunks);
        launch(ctx, s, "k_seg_hist", [&] { op.hist(ha, g, s); });
        const uint32_t gs = std::min<uint32_t>(grid_of(op.scan_kernel, 256), nseg);
        launch(ctx, s, "k_seg_scan", [&] { op.scan(ha, gs, s); });
    }
    const bool in_place = kin == (const void *)kout || (HAS_V && vin == (const void *)vout);
    const bool copy_back = in_place && (L.d & 1);
    {
        const uint32_t g = grid_of(op.pass_kernel, op.threads);
        const void *src_k = kin, *src_v = vin;
        for (int p = 0; p < L.d; ++p) {
            const bool to_out = copy_back ? (p & 1) != 0 : ((L.d - 1 - p) & 1) == 0;
            SegPassArgs pa{};
            pa.src_k = src_k;
            pa.src_v = src_v;
            pa.dst_k = to_out ? kout : tmp_k;
            pa.dst_v = to_out ? vout : tmp_v;
            pa.large = large;
            pa.tile_seg = tile_seg;
            pa.seg_base = seg_base;
            pa.seg_flags = seg_flags;
            pa.ctrl = ctrl;
            pa.status = status + (uint64_t)p * L.max_tiles * L.bins;
            pa.claims = status + (uint64_t)L.d * L.max_tiles * L.bins + (uint64_t)p * L.claim_words;
            pa.max_tiles = (uint32_t)L.max_tiles;
            pa.pass = p;
            pa.shift = p * op.r;
            pa.d = L.d;
            pa.map_load = p == 0 ? kmap : 0u;
            pa.map_store = (p == L.d - 1 && to_out) ? kmap : 0u;
            pa.spin_limit = ctx->spin_limit;
            pa.stall = ctx->stall;
            launch(ctx, s, sizeof(K) == 4 ? "k_seg_pass_u32" : "k_seg_pass_u64",
                   [&] { op.pass(pa, g, s); });
            src_k = pa.dst_k;
            src_v = pa.dst_v;
        }
    }
    if (copy_back) {
        SegCopyArgs cp{tmp_k, tmp_v, kout, vout, large, tile_seg, ctrl, (uint32_t)L.max_tiles,
                       (uint32_t)op.tile, kmap};
        const uint32_t g = (uint32_t)std::min<uint64_t>(L.max_tiles, 4096);
        launch(ctx, s, "k_seg_copy", [&] {
            hipLaunchKernelGGL((k_seg_copy<K, HAS_V>), dim3(g), dim3(256), 0, s, cp);
        });
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(RS_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return RS_OK;
}

// ---------------------------------------------------------------------------
// Scratch of rs_sort_noalloc: a fixed device array instead of an allocation.
// Every GPU the library runs on holds its own copy until the process ends.
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address comes from hipGetSymbolAddress, once per device, and only
// that address is handed to kernels.

constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

// The device address of this device's copy of `scratch` (the device must be
// current).  Looked up on the first call for a device, then reused.
static rs_status scratch_address(int device, void **out)
{
    if (device < 0 || device >= kMaxDevices)
        return fail(RS_ERR_UNSUPPORTED, "device %d is beyond the %d the library tracks", device,
                    kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(RS_ERR_DEVICE, "hipGetSymbolAddress(scratch) failed: %s",
                        hipGetErrorString(e));
        }
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
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
    if (!ctx->own.empty() || !ctx->events.empty()) {
        DeviceGuard g(ctx->device);
        for (OwnWorkspace &o : ctx->own)
            if (o.ptr)
                (void)hipFree(o.ptr);
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
    const int kb = key_type == RS_KEY_U32 ? 4 : 8;
    *bytes = (size_t)make_layout(kb, has_values != 0, n, pick_sort(ctx, kb, has_values != 0, n))
                 .total;
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

static uint32_t order_map(rs_key_type key_type, uint32_t order, rs_status *st)
{
    *st = RS_OK;
    if (order & ~(uint32_t)(RS_ORDER_SIGNED | RS_ORDER_FLOAT | RS_ORDER_DESCENDING)) {
        *st = fail(RS_ERR_INVALID_ARGUMENT, "unknown order flags 0x%x", order);
        return 0;
    }
    if ((order & RS_ORDER_SIGNED) && (order & RS_ORDER_FLOAT)) {
        *st = fail(RS_ERR_INVALID_ARGUMENT, "RS_ORDER_SIGNED and RS_ORDER_FLOAT exclude each other");
        return 0;
    }
    if (key_type != RS_KEY_U32 && key_type != RS_KEY_U64) {
        *st = fail(RS_ERR_INVALID_ARGUMENT, "unknown key type %d", (int)key_type);
        return 0;
    }
    return ((order & RS_ORDER_SIGNED) ? kMapSigned : 0u) | ((order & RS_ORDER_FLOAT) ? kMapFloat : 0u) |
           ((order & RS_ORDER_DESCENDING) ? kMapDescending : 0u);
}

rs_status rs_sort(rs_context *ctx, rs_key_type key_type, uint32_t order, const void *keys_in,
                  const void *vals_in, void *keys_out, void *vals_out, uint64_t n, void *ws,
                  size_t ws_bytes, void *stream)
{
    rs_status st;
    const uint32_t kmap = order_map(key_type, order, &st);
    if (st != RS_OK)
        return st;
    if ((vals_in != nullptr) != (vals_out != nullptr))
        return fail(RS_ERR_INVALID_ARGUMENT, "vals_in and vals_out must both be given or both NULL");
    if (key_type == RS_KEY_U32) {
        if (vals_in)
            return run_sort<uint32_t, true>(ctx, (const uint32_t *)keys_in, (const uint32_t *)vals_in,
                                            (uint32_t *)keys_out, (uint32_t *)vals_out, n, ws,
                                            ws_bytes, stream, kmap);
        return run_sort<uint32_t, false>(ctx, (const uint32_t *)keys_in, nullptr,
                                         (uint32_t *)keys_out, nullptr, n, ws, ws_bytes, stream,
                                         kmap);
    }
    if (vals_in)
        return run_sort<uint64_t, true>(ctx, (const uint64_t *)keys_in, (const uint64_t *)vals_in,
                                        (uint64_t *)keys_out, (uint64_t *)vals_out, n, ws, ws_bytes,
                                        stream, kmap);
    return run_sort<uint64_t, false>(ctx, (const uint64_t *)keys_in, nullptr, (uint64_t *)keys_out,
                                     nullptr, n, ws, ws_bytes, stream, kmap);
}

rs_status rs_sort_noalloc(rs_context *ctx, rs_key_type key_type, uint32_t order,
                          const void *keys_in, const void *vals_in, void *keys_out,
                          void *vals_out, uint64_t n, void *stream)
{
    if (!ctx)
        return fail(RS_ERR_INVALID_ARGUMENT, "ctx is NULL");
    rs_status st;
    (void)order_map(key_type, order, &st);
    if (st != RS_OK)
        return st;
    if ((vals_in != nullptr) != (vals_out != nullptr))
        return fail(RS_ERR_INVALID_ARGUMENT, "vals_in and vals_out must both be given or both NULL");
    if (n >= RS_MAX_ELEMENTS)
        return fail(RS_ERR_UNSUPPORTED, "n = %llu exceeds the limit of 2^30 - 1 elements",
                    (unsigned long long)n);
    if (n == 0)
        return RS_OK;
    const int kb = key_type == RS_KEY_U32 ? 4 : 8;
    const bool has_v = vals_in != nullptr;
    const uint64_t need = make_layout(kb, has_v, n, pick_sort(ctx, kb, has_v, n)).total;
    if (need > kNoAllocScratchBytes)
        return fail(RS_ERR_UNSUPPORTED,
                    "n = %llu needs %llu bytes of scratch, above the fixed %llu of "
                    "rs_sort_noalloc (use rs_sort with a workspace)",
                    (unsigned long long)n, (unsigned long long)need,
                    (unsigned long long)kNoAllocScratchBytes);
    DeviceGuard guard(ctx->device);
    if (!guard.ok)
        return fail(RS_ERR_DEVICE, "cannot select HIP device %d", ctx->device);
    void *ws = nullptr;
    st = scratch_address(ctx->device, &ws);
    if (st != RS_OK)
        return st;
    // no profiling events either: nothing is created on this path
    const bool prof = ctx->prof;
    ctx->prof = false;
    st = rs_sort(ctx, key_type, order, keys_in, vals_in, keys_out, vals_out, n, ws,
                 kNoAllocScratchBytes, stream);
    ctx->prof = prof;
    return st;
}

uint64_t rs_sort_noalloc_scratch_bytes(void)
{
    return kNoAllocScratchBytes;
}

rs_status rs_segmented_sort_order(rs_context *ctx, rs_key_type key_type, uint32_t order,
                                  const void *keys_in, const void *vals_in, void *keys_out,
                                  void *vals_out, const uint64_t *offsets, uint32_t num_segments,
                                  uint64_t total, void *ws, size_t ws_bytes, void *stream)
{
    rs_status st;
    const uint32_t kmap = order_map(key_type, order, &st);
    if (st != RS_OK)
        return st;
    if (key_type == RS_KEY_U32) {
        if (vals_in || vals_out)
            return run_segmented<uint32_t, true>(ctx, keys_in, vals_in, keys_out, vals_out, offsets,
                                                 num_segments, total, ws, ws_bytes, stream, kmap);
        return run_segmented<uint32_t, false>(ctx, keys_in, vals_in, keys_out, vals_out, offsets,
                                              num_segments, total, ws, ws_bytes, stream, kmap);
    }
    if (vals_in || vals_out)
        return run_segmented<uint64_t, true>(ctx, keys_in, vals_in, keys_out, vals_out, offsets,
                                             num_segments, total, ws, ws_bytes, stream, kmap);
    return run_segmented<uint64_t, false>(ctx, keys_in, vals_in, keys_out, vals_out, offsets,
                                          num_segments, total, ws, ws_bytes, stream, kmap);
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
    const int kb = key_type == RS_KEY_U32 ? 4 : 8;
    *bytes = (size_t)make_seg_layout(kb, has_values != 0, total, num_segments,
                                     pick_seg(ctx, kb, has_values != 0, total))
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

rs_status rs_workspace_status(rs_context *ctx, const void *ws, void *stream)
{
    if (!ctx)
        return fail(RS_ERR_INVALID_ARGUMENT, "ctx is NULL");
    if (ws && ((uintptr_t)ws & 255))
        return fail(RS_ERR_INVALID_ARGUMENT, "workspace must be 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    const void *w = ws;
    if (!w) {
        OwnWorkspace *o = own_workspace(ctx, s);
        if (!o || !o->ptr)
            return RS_OK;  // no sort with the context's own scratch ran on this stream
        w = o->ptr;
    }
    DeviceGuard guard(ctx->device);
    if (!guard.ok)
        return fail(RS_ERR_DEVICE, "cannot select HIP device %d", ctx->device);
    uint32_t word = 0;
    hipError_t e = hipMemcpyAsync(&word, (const uint32_t *)w + kCtrlError, sizeof word,
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(RS_ERR_DEVICE, "stream failed: %s", hipGetErrorString(e));
    }
    if (word & kErrWait)
        return fail(RS_ERR_DEVICE, "a wait on another workgroup reached its bound; the output "
                                   "is not valid");
    if (word & kErrSegTiles)
        return fail(RS_ERR_INVALID_ARGUMENT, "the segments need more tiles than the workspace "
                                             "holds (overlapping offsets); some were not sorted");
    if (word & kErrSegTooLarge)
        return fail(RS_ERR_UNSUPPORTED, "a segment of 2^30 or more elements was left unsorted");
    return RS_OK;
}

rs_status rs_device_copy(rs_context *ctx, const void *src, void *dst, uint64_t bytes,
                         void *stream)
{
    if (!ctx)
        return fail(RS_ERR_INVALID_ARGUMENT, "ctx is NULL");
    if (bytes == 0)
        return RS_OK;
    if (!src || !dst)
        return fail(RS_ERR_INVALID_ARGUMENT, "NULL pointer with bytes > 0");
    if ((((uintptr_t)src) | ((uintptr_t)dst) | bytes) & 15)
        return fail(RS_ERR_INVALID_ARGUMENT, "pointers and size must be multiples of 16 bytes");
    if (overlaps(src, bytes, dst, bytes))
        return fail(RS_ERR_INVALID_ARGUMENT, "source and destination overlap");
    DeviceGuard guard(ctx->device);
    if (!guard.ok)
        return fail(RS_ERR_DEVICE, "cannot select HIP device %d", ctx->device);
    hipStream_t s = (hipStream_t)stream;
    // 1024 x 2 words in flight per workgroup and 8192 workgroups measured
    // fastest among 256..1024 threads x 2..16 words and 1024..16384 groups
    constexpr int kThreads = 1024, kItems = 2;
    const uint64_t nvec = bytes / 16;
    const uint32_t grid = (uint32_t)std::max<uint64_t>(
        1, std::min<uint64_t>(8192, (nvec + kThreads * kItems - 1) / (kThreads * kItems)));
    launch(ctx, s, "k_copy_ceiling", [&] {
        hipLaunchKernelGGL((k_copy_ceiling<kThreads, kItems>), dim3(grid), dim3(kThreads), 0, s,
                           (const uint4 *)src, (uint4 *)dst, nvec);
    });
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(RS_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return RS_OK;
}

rs_status rs_debug_wait_set(rs_context *ctx, uint32_t spin_limit, uint32_t stall)
{
    if (!ctx)
        return fail(RS_ERR_INVALID_ARGUMENT, "ctx is NULL");
    if (spin_limit == 0)
        return fail(RS_ERR_INVALID_ARGUMENT, "spin_limit must be at least 1");
    if (stall & ~(kStallLookback | kStallClaim))
        return fail(RS_ERR_INVALID_ARGUMENT, "unknown stall bits 0x%x", stall);
    ctx->spin_limit = spin_limit;
    ctx->stall = stall;
    return RS_OK;
}

rs_status rs_debug_sort_stages(rs_context *ctx, rs_key_type key_type, const void *keys_in,
                               const void *vals_in, void *keys_out, void *vals_out, uint64_t n,
                               int passes, uint32_t *hist_out, void *ws, size_t ws_bytes,
                               void *stream)
{
    if (key_type != RS_KEY_U32 && key_type != RS_KEY_U64)
        return fail(RS_ERR_INVALID_ARGUMENT, "unknown key type %d", (int)key_type);
    if (passes < 0)
        return fail(RS_ERR_INVALID_ARGUMENT, "passes must be >= 0");
    if ((vals_in != nullptr) != (vals_out != nullptr))
        return fail(RS_ERR_INVALID_ARGUMENT, "vals_in and vals_out must both be given or both NULL");
    if (key_type == RS_KEY_U32) {
        if (vals_in)
            return run_sort<uint32_t, true>(ctx, (const uint32_t *)keys_in,
                                            (const uint32_t *)vals_in, (uint32_t *)keys_out,
                                            (uint32_t *)vals_out, n, ws, ws_bytes, stream, 0,
                                            passes, hist_out);
        return run_sort<uint32_t, false>(ctx, (const uint32_t *)keys_in, nullptr,
                                         (uint32_t *)keys_out, nullptr, n, ws, ws_bytes, stream, 0,
                                         passes, hist_out);
    }
    if (vals_in)
        return run_sort<uint64_t, true>(ctx, (const uint64_t *)keys_in, (const uint64_t *)vals_in,
                                        (uint64_t *)keys_out, (uint64_t *)vals_out, n, ws,
                                        ws_bytes, stream, 0, passes, hist_out);
    return run_sort<uint64_t, false>(ctx, (const uint64_t *)keys_in, nullptr, (uint64_t *)keys_out,
                                     nullptr, n, ws, ws_bytes, stream, 0, passes, hist_out);
}

rs_status rs_merge_workspace_bytes(const rs_context *ctx, rs_key_type key_type, int has_values,
                                   uint64_t n, size_t *bytes)
{
    if (!ctx || !bytes)
        return fail(RS_ERR_INVALID_ARGUMENT, "ctx or bytes is NULL");
    if (key_type != RS_KEY_U32 && key_type != RS_KEY_U64)
        return fail(RS_ERR_INVALID_ARGUMENT, "unknown key type %d", (int)key_type);
    if (n >= RS_MAX_ELEMENTS)
        return fail(RS_ERR_UNSUPPORTED, "n = %llu exceeds the limit of 2^30 - 1 elements",
                    (unsigned long long)n);
    const int kb = key_type == RS_KEY_U32 ? 4 : 8;
    *bytes = (size_t)make_merge_layout(kb, has_values != 0, n, merge_ops(kb, has_values != 0))
                 .total;
    return RS_OK;
}

rs_status rs_merge_sort(rs_context *ctx, rs_key_type key_type, uint32_t order,
                        const void *keys_in, const void *vals_in, void *keys_out, void *vals_out,
                        uint64_t n, void *ws, size_t ws_bytes, void *stream)
{
    rs_status st;
    const uint32_t kmap = order_map(key_type, order, &st);
    if (st != RS_OK)
        return st;
    if ((vals_in != nullptr) != (vals_out != nullptr))
        return fail(RS_ERR_INVALID_ARGUMENT, "vals_in and vals_out must both be given or both NULL");
    if (key_type == RS_KEY_U32) {
        if (vals_in)
            return run_merge<uint32_t, true>(ctx, (const uint32_t *)keys_in,
                                             (const uint32_t *)vals_in, (uint32_t *)keys_out,
                                             (uint32_t *)vals_out, n, ws, ws_bytes, stream, kmap);
        return run_merge<uint32_t, false>(ctx, (const uint32_t *)keys_in, nullptr,
                                          (uint32_t *)keys_out, nullptr, n, ws, ws_bytes, stream,
                                          kmap);
    }
    if (vals_in)
        return run_merge<uint64_t, true>(ctx, (const uint64_t *)keys_in, (const uint64_t *)vals_in,
                                         (uint64_t *)keys_out, (uint64_t *)vals_out, n, ws,
                                         ws_bytes, stream, kmap);
    return run_merge<uint64_t, false>(ctx, (const uint64_t *)keys_in, nullptr,
                                      (uint64_t *)keys_out, nullptr, n, ws, ws_bytes, stream, kmap);
}

rs_status rs_segmented_tiny_cap_set(rs_context *ctx, uint32_t cap)
{
    if (!ctx)
        return fail(RS_ERR_INVALID_ARGUMENT, "ctx is NULL");
    if (cap > kTinyMax)
        return fail(RS_ERR_INVALID_ARGUMENT, "tiny cap %u exceeds %u", cap, kTinyMax);
    ctx->tiny_cap = cap < 2 ? 0u : cap;
    return RS_OK;
}

rs_status rs_segmented_tiny_cap_get(const rs_context *ctx, uint32_t *cap)
{
    if (!ctx || !cap)
        return fail(RS_ERR_INVALID_ARGUMENT, "ctx or cap is NULL");
    *cap = ctx->tiny_cap;
    return RS_OK;
}

rs_status rs_config_count(rs_key_type key_type, int has_values, int *count)
{
    if (!count)
        return fail(RS_ERR_INVALID_ARGUMENT, "count is NULL");
    if (key_type != RS_KEY_U32 && key_type != RS_KEY_U64)
        return fail(RS_ERR_INVALID_ARGUMENT, "unknown key type %d", (int)key_type);
    (void)sort_table(key_type == RS_KEY_U32 ? 4 : 8, has_values != 0, count);
    return RS_OK;
}

rs_status rs_segmented_config_count(rs_key_type key_type, int has_values, int *count)
{
    if (!count)
        return fail(RS_ERR_INVALID_ARGUMENT, "count is NULL");
    if (key_type != RS_KEY_U32 && key_type != RS_KEY_U64)
        return fail(RS_ERR_INVALID_ARGUMENT, "unknown key type %d", (int)key_type);
    (void)seg_table(key_type == RS_KEY_U32 ? 4 : 8, has_values != 0, count);
    return RS_OK;
}

rs_status rs_config_get(rs_key_type key_type, int has_values, int index, rs_config *config)
{
    if (!config)
        return fail(RS_ERR_INVALID_ARGUMENT, "config is NULL");
    if (key_type != RS_KEY_U32 && key_type != RS_KEY_U64)
        return fail(RS_ERR_INVALID_ARGUMENT, "unknown key type %d", (int)key_type);
    int count = 0;
    const SortOps *t = sort_table(key_type == RS_KEY_U32 ? 4 : 8, has_values != 0, &count);
    if (index < 0 || index >= count)
        return fail(RS_ERR_INVALID_ARGUMENT, "configuration index %d outside [0, %d)", index,
                    count);
    config->radix_bits = t[index].r;
    config->threads = t[index].threads;
    config->items = t[index].items;
    return RS_OK;
}

rs_status rs_tune_set(rs_context *ctx, rs_key_type key_type, int has_values, int segmented,
                      int size_log2, int index)
{
    if (!ctx)
        return fail(RS_ERR_INVALID_ARGUMENT, "ctx is NULL");
    if (key_type != RS_KEY_U32 && key_type != RS_KEY_U64)
        return fail(RS_ERR_INVALID_ARGUMENT, "unknown key type %d", (int)key_type);
    if (size_log2 < -1 || size_log2 >= kTuneClasses)
        return fail(RS_ERR_INVALID_ARGUMENT, "size_log2 %d outside [-1, %d)", size_log2,
                    kTuneClasses);
    int count = 0;
    // the segmented sort's list is the prefix of the plain sort's without
    // the wide-digit configurations
    if (segmented)
        (void)seg_table(key_type == RS_KEY_U32 ? 4 : 8, has_values != 0, &count);
    else
        (void)sort_table(key_type == RS_KEY_U32 ? 4 : 8, has_values != 0, &count);
    if (index < -1 || index >= count)
        return fail(RS_ERR_INVALID_ARGUMENT, "configuration index %d outside [-1, %d)%s", index,
                    count, segmented ? " for the segmented sort" : "");
    int8_t *row = ctx->tune[key_type == RS_KEY_U64][has_values != 0][segmented != 0];
    for (int c = 0; c < kTuneClasses; ++c)
        if (size_log2 < 0 || c == size_log2)
            row[c] = (int8_t)index;
    return RS_OK;
}

rs_status rs_tune_get(const rs_context *ctx, rs_key_type key_type, int has_values, int segmented,
                      int size_log2, int *index)
{
    if (!ctx || !index)
        return fail(RS_ERR_INVALID_ARGUMENT, "ctx or index is NULL");
    if (key_type != RS_KEY_U32 && key_type != RS_KEY_U64)
        return fail(RS_ERR_INVALID_ARGUMENT, "unknown key type %d", (int)key_type);
    if (size_log2 < 0 || size_log2 >= kTuneClasses)
        return fail(RS_ERR_INVALID_ARGUMENT, "size_log2 %d outside [0, %d)", size_log2,
                    kTuneClasses);
    int count = 0;
    const int kb = key_type == RS_KEY_U32 ? 4 : 8;
    (void)sort_table(kb, has_values != 0, &count);
    const int i = ctx->tune[key_type == RS_KEY_U64][has_values != 0][segmented != 0][size_log2];
    *index = (i >= 0 && i < count) ? i : default_index(kb, has_values != 0, segmented != 0, size_log2);
    return RS_OK;
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
