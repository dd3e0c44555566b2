"""Exact O(n) certificate that a (keys, values) output is *the* stable sort.

With value[i] = i on input, the three conditions below together imply that
the output equals the unique stable ascending sort by unsigned key, with no
second implementation needed:

1. the output values are a permutation of [0, n);
2. out_key[i] == in_key[out_val[i]] for every i;
3. the keys never decrease, and within a run of equal keys the values
   strictly increase.

(1)+(2) make the output a rearrangement of the input pairs; (3) forces the
order among them, which is then unique.
"""
import numpy as np


def certify_stable_sort(in_keys, out_keys, out_vals):
    in_keys = np.asarray(in_keys)
    out_keys = np.asarray(out_keys)
    out_vals = np.asarray(out_vals).astype(np.int64, copy=False)
    n = in_keys.size
    if out_keys.size != n or out_vals.size != n:
        return "length mismatch"
    if n == 0:
        return None
    if out_vals.min() < 0 or out_vals.max() >= n:
        return "value out of range"
    seen = np.zeros(n, dtype=bool)
    seen[out_vals] = True
    if not seen.all():
        return "values are not a permutation"
    if not np.array_equal(out_keys, in_keys[out_vals]):
        return "a key does not travel with its value"
    if n > 1:
        dk = out_keys[1:] >= out_keys[:-1]
        if not dk.all():
            return "keys decrease at %d" % int(np.argmin(dk))
        eq = out_keys[1:] == out_keys[:-1]
        if (eq & (out_vals[1:] <= out_vals[:-1])).any():
            return "equal keys out of input order (unstable)"
    return None


def certify_sorted_keys(in_keys, out_keys):
    """Keys-only: non-decreasing and the same multiset (exact, via a
    library sort of the input -- a third-party cross-check)."""
    in_keys = np.asarray(in_keys)
    out_keys = np.asarray(out_keys)
    if in_keys.size != out_keys.size:
        return "length mismatch"
    if out_keys.size > 1 and not (out_keys[1:] >= out_keys[:-1]).all():
        return "keys decrease"
    if not np.array_equal(np.sort(in_keys), out_keys):
        return "multiset differs"
    return None


def multiset_hash(keys):
    """Order-independent 64-bit hash of a key multiset (sum and xor of a
    per-key mix), for quick checks where a full copy is not wanted."""
    k = np.asarray(keys).astype(np.uint64)
    with np.errstate(over="ignore"):
        x = k * np.uint64(0x9E3779B97F4A7C15)
        x ^= x >> np.uint64(29)
        x *= np.uint64(0xBF58476D1CE4E5B9)
        x ^= x >> np.uint64(32)
        return int(x.sum(dtype=np.uint64)), int(np.bitwise_xor.reduce(x)) if x.size else 0


def certify_segmented(in_keys, out_keys, out_vals, offsets):
    """Segmented form of the certificate, with value = index within the
    segment: every segment of the output is the unique stable sort of the
    same segment of the input.  Elements outside every segment are not
    checked here."""
    in_keys = np.asarray(in_keys)
    out_keys = np.asarray(out_keys)
    out_vals = np.asarray(out_vals).astype(np.int64)
    off = np.asarray(offsets, dtype=np.int64)
    sizes = np.diff(off)
    if (sizes < 0).any():
        return "offsets decrease"
    seg = np.repeat(np.arange(sizes.size), sizes)
    starts = np.repeat(off[:-1], sizes)
    lo, hi = int(off[0]), int(off[-1])
    ok_, ov = out_keys[lo:hi], out_vals[lo:hi]
    if ((ov < 0) | (ov >= np.repeat(sizes, sizes))).any():
        return "value out of its segment"
    g = starts + ov
    seen = np.zeros(hi - lo, dtype=bool)
    seen[g - lo] = True
    if not seen.all():
        return "values are not a permutation within each segment"
    if not np.array_equal(ok_, in_keys[g]):
        return "a key does not travel with its value"
    same = seg[1:] == seg[:-1]
    dk = ok_[1:] >= ok_[:-1]
    if (same & ~dk).any():
        return "keys decrease inside a segment"
    eq = same & (ok_[1:] == ok_[:-1])
    if (eq & (ov[1:] <= ov[:-1])).any():
        return "equal keys out of input order (unstable)"
    return None
