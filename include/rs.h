/*
 * rs.h -- C-ABI of the MI355X (gfx950) LSD radix sort library (librs.so).
 *
 * The operation is the least-significant-digit radix sort described in the
 * paper (Bozidar & Dobravec, "Comparison of parallel sorting algorithms",
 * Section 2.6): keys are split into r-bit digits and sorted digit by digit
 * from the least significant one, each pass being a stable counting sort.
 * Inputs are 32-bit or 64-bit unsigned keys, alone or with a value of the
 * same width (Sections 1 and 3), of any length (Section 1).  The result is
 * the ascending, stable sort by unsigned key: equal keys keep their input
 * order, and each value travels with its key.  Exactly one output is
 * correct, so results are bit-exact.
 *
 * Conventions shared by every entry point below:
 *
 *  - Pointers named *_in, *_out, ws and offsets are DEVICE pointers on the
 *    context's device (hipMalloc / torch allocations).  Keys and values are
 *    separate arrays (structure of arrays).  Alignment: 4 bytes for 32-bit
 *    data, 8 bytes for 64-bit data.
 *  - The caller owns every buffer.  The library never frees what it did not
 *    allocate.
 *  - *_out may equal *_in (in-place).  Any other overlap between an input
 *    and an output, or between keys and values, is RS_ERR_INVALID_ARGUMENT.
 *  - ws / ws_bytes: scratch memory of at least rs_workspace_bytes() bytes,
 *    256-byte aligned.  ws == NULL makes the context allocate and keep a
 *    scratch buffer of its own, one per stream (grow-only; growing waits for
 *    that stream; all are freed by rs_context_destroy), so calls on
 *    different streams never share scratch.  That mode calls hipMalloc and
 *    is therefore not usable under stream capture.  Calls that share one
 *    caller workspace must be ordered (same stream, or synchronised).
 *  - stream is a hipStream_t (NULL = the device's null stream).  Calls are
 *    asynchronous: the output is valid once the stream has completed.
 *    Device faults surface at the caller's next synchronisation.
 *  - Arguments are validated on the host before any HIP call; a rejected
 *    call enqueues nothing.  n = 0 is valid and enqueues nothing.
 *  - One sort handles n < 2^30 elements (RS_ERR_UNSUPPORTED above that).
 *  - Nothing is thrown across this interface.  rs_last_error() returns a
 *    thread-local description of the last failure.
 *  - Errors found on the device (a segment too large for one sort, a wait
 *    on another workgroup that reached its bound) are recorded in the
 *    workspace and reported by rs_workspace_status() once the stream has
 *    completed; the enqueueing call has already returned RS_OK.
 *  - A context may be used from one host thread at a time.
 */
#ifndef RS_H
#define RS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum rs_status {
    RS_OK = 0,
    RS_ERR_INVALID_ARGUMENT = 1, /* bad pointer, size, alignment, overlap, workspace */
    RS_ERR_UNSUPPORTED = 2,      /* valid request outside this version's limits */
    RS_ERR_OUT_OF_MEMORY = 3,    /* the context could not allocate its own scratch */
    RS_ERR_DEVICE = 4            /* a HIP call failed (launch, device selection) */
} rs_status;

typedef enum rs_key_type {
    RS_KEY_U32 = 0,
    RS_KEY_U64 = 1
} rs_key_type;

typedef struct rs_context rs_context; /* opaque */

/* Maximum elements in one sort or one segmented batch. */
#define RS_MAX_ELEMENTS ((uint64_t)1 << 30)

/*
 * Create a context bound to HIP device `device`.  HIP is touched lazily: the
 * device is only selected when the first sort is enqueued, so a context can
 * be created (and arguments validated) on a machine without a GPU.
 * *out receives the context; release it with rs_context_destroy.
 */
rs_status rs_context_create(int device, rs_context **out);

/* Release a context and any scratch memory it allocated.  NULL is a no-op. */
void rs_context_destroy(rs_context *ctx);

/*
 * Bytes of scratch memory one sort of n elements needs (look-back words,
 * digit histograms, one ping-pong copy of the keys and values) with the
 * configuration the context's tune table selects for n (see rs_tune_set:
 * query again after changing the table).  Pure host arithmetic; never
 * touches the device.
 */
rs_status rs_workspace_bytes(const rs_context *ctx, rs_key_type key_type, int has_values,
                             uint64_t n, size_t *bytes);

/*
 * Stable ascending sort of n 32-bit keys (Section 2.6): keys_out receives the
 * keys of keys_in in ascending unsigned order.  keys_in is read, never
 * written, unless keys_out == keys_in.
 */
rs_status rs_sort_keys_u32(rs_context *ctx, const uint32_t *keys_in, uint32_t *keys_out,
                           uint64_t n, void *ws, size_t ws_bytes, void *stream);

/* As rs_sort_keys_u32 for 64-bit keys. */
rs_status rs_sort_keys_u64(rs_context *ctx, const uint64_t *keys_in, uint64_t *keys_out,
                           uint64_t n, void *ws, size_t ws_bytes, void *stream);

/*
 * Stable sort of n (32-bit key, 32-bit value) pairs by key (Sections 1, 2.6):
 * output position i holds the pair with the i-th smallest (key, input index).
 */
rs_status rs_sort_pairs_u32(rs_context *ctx, const uint32_t *keys_in, const uint32_t *vals_in,
                            uint32_t *keys_out, uint32_t *vals_out, uint64_t n, void *ws,
                            size_t ws_bytes, void *stream);

/* As rs_sort_pairs_u32 for 64-bit keys with 64-bit values. */
rs_status rs_sort_pairs_u64(rs_context *ctx, const uint64_t *keys_in, const uint64_t *vals_in,
                            uint64_t *keys_out, uint64_t *vals_out, uint64_t n, void *ws,
                            size_t ws_bytes, void *stream);

/*
 * Batched segmented sort: num_segments independent stable sorts, segment s
 * being elements [offsets[s], offsets[s+1]) of the arrays, sorted within its
 * own range.  offsets is a DEVICE array of num_segments+1 uint64 values,
 * non-decreasing, offsets[0] >= 0 and offsets[num_segments] <= total; empty
 * segments are allowed.  vals_in/vals_out NULL = keys only.  Elements outside
 * every segment are left untouched in *_out.  Bytes of scratch:
 * rs_segmented_workspace_bytes().  Offsets are read on the device only (no
 * host round trip); a non-monotone offsets array is not detected and gives
 * unspecified (but in-bounds) results.  Segments are classified on the
 * device: up to the tiny cap (rs_segmented_tiny_cap_set, 1024 by default) a
 * bitonic network per wave (Section 2.1), up to 16384 elements (8192 for
 * 64-bit pairs) a one-workgroup LDS radix sort, larger ones batched digit
 * passes (Section 2.6); every class gives the same stable sort.  One
 * segment must hold fewer than 2^30 elements; a larger one is left
 * unsorted and reported by rs_workspace_status (RS_ERR_UNSUPPORTED).
 */
rs_status rs_segmented_sort(rs_context *ctx, rs_key_type key_type, const void *keys_in,
                            const void *vals_in, void *keys_out, void *vals_out,
                            const uint64_t *offsets, uint32_t num_segments, uint64_t total,
                            void *ws, size_t ws_bytes, void *stream);

/*
 * Device-side status of the last rs_sort_* / rs_sort / rs_segmented_sort*
 * call (n >= 1) that used workspace `ws` (NULL: the context's own scratch
 * of `stream`).  Synchronises `stream`, then reads the error word the
 * kernels leave in the workspace's control block:
 *   RS_OK                    the sort completed;
 *   RS_ERR_UNSUPPORTED       a segment of 2^30 or more elements was left
 *                            unsorted (one segment is one radix sort, whose
 *                            look-back count field has 30 bits);
 *   RS_ERR_INVALID_ARGUMENT  overlapping segment offsets needed more tiles
 *                            than the workspace holds; some segments were
 *                            left unsorted;
 *   RS_ERR_DEVICE            the stream failed, or a wait on another
 *                            workgroup (a tile claim or a look-back)
 *                            reached its bound: the output is not valid.
 * Not meaningful for rs_merge_sort workspaces (the merge sort never waits).
 */
rs_status rs_workspace_status(rs_context *ctx, const void *ws, void *stream);

/* Scratch bytes for rs_segmented_sort on `total` elements in num_segments
 * segments, with the configuration the tune table selects for `total`.
 * Pure host arithmetic. */
rs_status rs_segmented_workspace_bytes(const rs_context *ctx, rs_key_type key_type,
                                       int has_values, uint64_t total, uint32_t num_segments,
                                       size_t *bytes);

/*
 * Per-kernel timing for benchmarks and profiling.  While enabled, every
 * kernel the context launches is bracketed by two HIP events recorded on the
 * launch stream, and the pair is kept with the kernel's name and the tag set
 * by rs_profile_tag().  Disabled by default; enabling costs two event
 * records per launch and no synchronisation.
 */
rs_status rs_profile_enable(rs_context *ctx, int enable);

/* Tag attached to the records of later launches (e.g. an input id). */
rs_status rs_profile_tag(rs_context *ctx, int tag);

/* Drop all records. */
rs_status rs_profile_reset(rs_context *ctx);

/*
 * Synchronise on the recorded events and copy out up to `max` records:
 * names[i] points to a static kernel name, tags[i] is the tag, ms[i] the
 * elapsed time between the record's two events in milliseconds.  *count
 * receives the number of records held (which may exceed max).
 */
rs_status rs_profile_read(rs_context *ctx, const char **names, int *tags, float *ms, int max,
                          int *count);

/*
 * Key orders.  The entry points above sort unsigned keys ascending.  rs_sort
 * and rs_segmented_sort_order take `order`, a combination of:
 *   RS_ORDER_SIGNED      keys are two's-complement integers;
 *   RS_ORDER_FLOAT       keys are IEEE-754 floats (binary32 for 32-bit keys,
 *                        binary64 for 64-bit keys) ordered as a total order
 *                        of their bit patterns: -NaN < -inf < ... < -0 <
 *                        +0 < ... < +inf < +NaN (so -0 sorts before +0 and
 *                        NaNs sort at the ends by their sign);
 *   RS_ORDER_DESCENDING  largest first; equal keys keep their input order.
 * SIGNED and FLOAT exclude each other; 0 is unsigned ascending.  Each order
 * is an exact bijection of the key bits applied where keys are read and
 * undone where they are written, inside the same kernels (no extra pass
 * over the data); output keys are the input keys, reordered.  The sort
 * stays stable (Section 2.6's counting sorts on the mapped digits).
 */
typedef enum {
    RS_ORDER_UNSIGNED = 0,
    RS_ORDER_SIGNED = 1,
    RS_ORDER_FLOAT = 2,
    RS_ORDER_DESCENDING = 4
} rs_order;

/*
 * Stable sort of n keys (vals_in/vals_out both NULL) or key-value pairs of
 * key_type's width in the given order; otherwise as rs_sort_keys_u32 /
 * rs_sort_pairs_u32.  Unknown or conflicting order flags ->
 * RS_ERR_INVALID_ARGUMENT.
 */
rs_status rs_sort(rs_context *ctx, rs_key_type key_type, uint32_t order, const void *keys_in,
                  const void *vals_in, void *keys_out, void *vals_out, uint64_t n, void *ws,
                  size_t ws_bytes, void *stream);

/*
 * rs_sort for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments and result as rs_sort, without ws / ws_bytes: the scratch
 * (control block, histograms, look-back words and the ping-pong copy) is a
 * fixed device array inside the library, rs_sort_noalloc_scratch_bytes()
 * bytes (64 MiB) on each GPU it runs on, held until the process ends.  The
 * call allocates nothing (no hipMalloc, no hipFree, no profiling events).
 * A sort whose workspace (rs_workspace_bytes) exceeds that size is rejected
 * with RS_ERR_UNSUPPORTED before any HIP call: about 16M 32-bit keys, 8M
 * 32-bit pairs or 64-bit keys, 4M 64-bit pairs.  Every call on one GPU
 * shares that GPU's array and clears what must start at zero itself; calls
 * that overlap in time on one GPU (other streams, other host threads) race
 * and must not be made.  Device-side errors: rs_workspace_status is not
 * available for this scratch (the call never waits longer than the bound of
 * rs_debug_wait_set and then leaves an invalid output).
 */
rs_status rs_sort_noalloc(rs_context *ctx, rs_key_type key_type, uint32_t order,
                          const void *keys_in, const void *vals_in, void *keys_out,
                          void *vals_out, uint64_t n, void *stream);

/* Bytes of the fixed scratch array of rs_sort_noalloc. */
uint64_t rs_sort_noalloc_scratch_bytes(void);

/* rs_segmented_sort with a key order; same arguments otherwise. */
rs_status rs_segmented_sort_order(rs_context *ctx, rs_key_type key_type, uint32_t order,
                                  const void *keys_in, const void *vals_in, void *keys_out,
                                  void *vals_out, const uint64_t *offsets, uint32_t num_segments,
                                  uint64_t total, void *ws, size_t ws_bytes, void *stream);

/*
 * Tiny segments of a segmented sort.  Segments of 2 .. cap elements (cap at
 * most 1024; the default is 1024) are sorted by one wave each with Batcher's
 * bitonic network (Section 2.1) in registers, on (key, position in the
 * segment) pairs so that the result is the same stable sort as the radix
 * path's; cap 0 (or 1) sends them to the one-workgroup radix sort instead.
 * The setting belongs to the context and applies to later
 * rs_segmented_sort* calls and to graphs captured after it.
 * cap > 1024 -> RS_ERR_INVALID_ARGUMENT.
 */
rs_status rs_segmented_tiny_cap_set(rs_context *ctx, uint32_t cap);
rs_status rs_segmented_tiny_cap_get(const rs_context *ctx, uint32_t *cap);

/*
 * Stable merge sort (Section 2.4: the sequence is cut into runs, each run is
 * sorted, and sorted runs are merged pairwise with a stable merge until one
 * run remains), the comparison-based counterpart of the radix sort.  Same
 * result as rs_sort with the same arguments: the unique stable sort in the
 * given order (position i holds the pair with the i-th smallest key,
 * equal keys in input order).
 *
 * On the device: tiles of 8192 elements are sorted in one workgroup's LDS
 * (a stable odd-even transposition network per thread, then merge-path
 * merges in LDS), then ceil(log2(n / 8192)) merge levels each read and
 * write every element once.  keys_in may equal keys_out (and vals_in
 * vals_out): in place.  ws: a device buffer of at least
 * rs_merge_workspace_bytes() bytes (scratch copies of keys and values and
 * one split word per 2048 outputs), 256-byte aligned, or NULL for the
 * context's own; n <= 8192 needs none.  Errors as rs_sort.
 */
rs_status rs_merge_sort(rs_context *ctx, rs_key_type key_type, uint32_t order,
                        const void *keys_in, const void *vals_in, void *keys_out, void *vals_out,
                        uint64_t n, void *ws, size_t ws_bytes, void *stream);

/* Bytes of workspace rs_merge_sort needs for n elements of this kind. */
rs_status rs_merge_workspace_bytes(const rs_context *ctx, rs_key_type key_type, int has_values,
                                   uint64_t n, size_t *bytes);

/*
 * Kernel configurations and the tune table.
 *
 * The digit width r is a free parameter of the method (Section 2.6: the
 * keys are cut into r-bit digits and sorted with one counting sort per
 * digit; the result does not depend on r).  The library is compiled for a
 * fixed list of configurations per key type and values/no values: r of 4 to
 * 8 bits and of 11 bits (ceil(key bits / r) digit passes: three for 32-bit
 * keys at 11 bits) and tile shapes of threads x items elements per
 * workgroup.  Index 0 of each list is the default.  Each
 * context holds a tune table that picks one configuration per key type,
 * values or not, plain or segmented sort, and size class ceil(log2 n) (n of
 * the plain sort, `total` of the segmented one).  Sorts that fit one
 * workgroup's LDS (up to 16384 elements, 8192 for 64-bit pairs) and the
 * small and medium segments always use the one-workgroup sort, whatever the
 * table says.  Every configuration gives the same, bit-exact result.
 */
typedef struct rs_config {
    int radix_bits; /* digit width r, 4..11 */
    int threads;    /* workgroup size of the digit pass */
    int items;      /* elements per thread; a tile holds threads * items */
} rs_config;

/* Number of compiled configurations for this key type, with/without values. */
rs_status rs_config_count(rs_key_type key_type, int has_values, int *count);

/* How many of them (the first *count of the list) the segmented sort can
 * use: the configurations with digits of more than 8 bits are compiled for
 * the plain sort only. */
rs_status rs_segmented_config_count(rs_key_type key_type, int has_values, int *count);

/* Configuration `index` (0 <= index < count) of that list. */
rs_status rs_config_get(rs_key_type key_type, int has_values, int index, rs_config *config);

/*
 * Select configuration `index` (-1 = the built-in choice) for sorts of this
 * kind whose size class ceil(log2 n) is size_log2 (0..39), or for every
 * size class if size_log2 is -1.  segmented != 0 selects the table of
 * rs_segmented_sort.  The built-in choice of a plain sort is the one the
 * autotuner selected on MI355X: 1024 x 8 tiles up to size class 21 (from
 * class 18 up for 64-bit pairs), 256 x 16 or 512 x 8 tiles at the smallest
 * classes of some kinds, index 0 above; segmented sorts use index 0.  Takes effect for
 * calls enqueued afterwards; a workspace sized before the change may be too
 * small for the new choice (the sort then returns RS_ERR_INVALID_ARGUMENT).
 */
rs_status rs_tune_set(rs_context *ctx, rs_key_type key_type, int has_values, int segmented,
                      int size_log2, int index);

/* The configuration index in force for one size class (0..39): the table's
 * entry, or the built-in choice where it is unset. */
rs_status rs_tune_get(const rs_context *ctx, rs_key_type key_type, int has_values, int segmented,
                      int size_log2, int *index);

/*
 * Test entry points (for the library's own tests; a working caller needs
 * neither).
 *
 * rs_debug_wait_set: every wait of a digit pass on another workgroup (tile
 * claims, the decoupled look-back of Section 2.6's prefix sums spread over
 * tiles) polls at most spin_limit times without progress before it records
 * an error and lets the kernel finish (default 2^22 polls, several seconds).
 * stall bit 1 makes every look-back, bit 2 every tile claim after the
 * first, treat its predecessor as not yet published, so that each such wait
 * reaches its bound and the give-up path runs with every kernel still
 * exiting normally.  Only grouped claims wait: passes of more than 1024
 * tiles (not 32-bit keys without values) and the segmented sort; a smaller
 * pass claims its tiles from one counter without waiting.  Applies to later
 * calls on the context.
 * spin_limit 0 or unknown stall bits -> RS_ERR_INVALID_ARGUMENT.
 *
 * rs_debug_sort_stages: the plain radix sort's kernels stage by stage, for
 * per-kernel checks against the counting sort of Section 2.6.  Runs the
 * histogram kernel, copies the digit histograms (u32[d][2^r] for the
 * configuration the tune table selects, d = ceil(key bits / r)) to the
 * DEVICE array hist_out unless it is NULL, then only the digit passes of
 * positions [0, passes): keys_out/vals_out receive the state after those
 * passes (the input stably sorted by its low passes*r bits; passes = 0
 * copies the input).  Always takes the multi-kernel path, whatever n.
 * Unsigned ascending order; otherwise as rs_sort.
 */
rs_status rs_debug_wait_set(rs_context *ctx, uint32_t spin_limit, uint32_t stall);

/*
 * Measurement helper: a plain device copy of `bytes` bytes (a multiple of 16,
 * both pointers 16-byte aligned, no overlap), each thread keeping its loads
 * in flight before its stores.  The digit pass reads and writes every
 * element once, so this copy's rate is the ceiling it is compared with.
 * Asynchronous on `stream`; profiled like the sorts (kernel k_copy_ceiling).
 */
rs_status rs_device_copy(rs_context *ctx, const void *src, void *dst, uint64_t bytes,
                         void *stream);
rs_status rs_debug_sort_stages(rs_context *ctx, rs_key_type key_type, const void *keys_in,
                               const void *vals_in, void *keys_out, void *vals_out, uint64_t n,
                               int passes, uint32_t *hist_out, void *ws, size_t ws_bytes,
                               void *stream);

/* Static description of a status code. */
const char *rs_status_string(rs_status status);

/* Thread-local detail of the last failed call on this thread ("" if none). */
const char *rs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RS_H */
