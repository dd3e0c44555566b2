"""Seeded synthetic inputs for the radix sort: the one module that both the
oracle and the HIP path draw their inputs from.

Nothing here sorts by digit, counts or scans: this module only draws numbers.
The generator is the 32-bit Mersenne Twister MT19937 (Matsumoto and Nishimura,
1998) in its standard seeding (``init_genrand``), reached through numpy's
frozen legacy ``RandomState`` stream.  A full-range ``uint32`` draw from that
stream is one raw MT19937 output, so a 64-bit key is built from two
consecutive outputs, the high word first.

The paper tests six input distributions (uniform, Gaussian, zero, bucket,
sorted, sorted descending; Section 4) drawn from a Mersenne Twister
(Section 3) but defines none of them; the recipes below are the reading this
project adopts:

* ``uniform``  key = u_K()
* ``gaussian`` key = floor((u_K()+u_K()+u_K()+u_K()) / 4), summed exactly
* ``zero``     key = 0 (draws nothing)
* ``sorted``   uniform keys, ascending
* ``reverse``  uniform keys, descending
* ``bucket``   a table of 64 distinct u_K() values (a repeat is redrawn), then
               key = table[g() >> 26]

Values are the input index (``value[i] = i``) so that stability can be read
off the output.
"""
from __future__ import annotations

import numpy as np

DISTRIBUTIONS = ("uniform", "gaussian", "zero", "sorted", "reverse", "bucket")


class MT19937:
    """Sequential MT19937 stream with the standard integer seeding."""

    def __init__(self, seed: int = 5489):
        if not 0 <= seed < 2**32:
            raise ValueError("seed must be in [0, 2^32)")
        self._rs = np.random.RandomState(seed)

    def u32(self, n: int) -> np.ndarray:
        """n raw 32-bit outputs, in stream order."""
        if n == 0:
            return np.zeros(0, dtype=np.uint32)
        return self._rs.randint(0, 2**32, size=n, dtype=np.uint32)

    def u64(self, n: int) -> np.ndarray:
        """n 64-bit words, each (first output << 32) | second output."""
        w = self.u32(2 * n).astype(np.uint64)
        return (w[0::2] << np.uint64(32)) | w[1::2]

    def uniform01(self, n: int) -> np.ndarray:
        """n doubles u = g() / 2^32 in [0, 1), one output each."""
        return self.u32(n).astype(np.float64) / 4294967296.0


def _draw(g: MT19937, bits: int, n: int) -> np.ndarray:
    return g.u32(n) if bits == 32 else g.u64(n)


def keys(dist: str, n: int, bits: int = 32, seed: int = 1) -> np.ndarray:
    """n keys of the given distribution and width (32 or 64 bits)."""
    if bits not in (32, 64):
        raise ValueError("bits must be 32 or 64")
    if dist not in DISTRIBUTIONS:
        raise ValueError(f"unknown distribution {dist!r}")
    dt = np.uint32 if bits == 32 else np.uint64
    g = MT19937(seed)
    if dist == "zero":
        return np.zeros(n, dtype=dt)
    if dist == "uniform":
        return _draw(g, bits, n)
    if dist == "gaussian":
        # four consecutive draws per key, in stream order
        u = _draw(g, bits, 4 * n).reshape(n, 4)
        if bits == 32:
            s = u.astype(np.uint64).sum(axis=1)  # < 2^34, exact
            return (s >> np.uint64(2)).astype(np.uint32)
        # exact floor of a 66-bit sum / 4 without 128-bit integers:
        # sum = 4*q + r, q = sum(u>>2) + (sum(u&3) >> 2)
        hi = (u >> np.uint64(2)).sum(axis=1, dtype=np.uint64)  # < 2^64
        lo = (u & np.uint64(3)).sum(axis=1, dtype=np.uint64)  # <= 12
        return hi + (lo >> np.uint64(2))
    if dist in ("sorted", "reverse"):
        k = np.sort(_draw(g, bits, n), kind="stable")
        return k if dist == "sorted" else k[::-1].copy()
    # bucket
    table: list[int] = []
    seen: set[int] = set()
    while len(table) < 64:
        v = int(_draw(g, bits, 1)[0])
        if v not in seen:
            seen.add(v)
            table.append(v)
    idx = (g.u32(n) >> np.uint32(26)).astype(np.int64)
    return np.asarray(table, dtype=dt)[idx]


def values(n: int, bits: int = 32) -> np.ndarray:
    """value[i] = i, in the key width."""
    return np.arange(n, dtype=np.uint32 if bits == 32 else np.uint64)


def segment_sizes(num_segments: int = 20000, lo_log2: int = 4, hi_log2: int = 20,
                  seed: int = 1, g: MT19937 | None = None) -> np.ndarray:
    """Log-uniform segment sizes floor(2^(lo + (hi-lo)*u)), clamped to
    [2^lo, 2^hi]; one draw per segment."""
    g = g or MT19937(seed)
    u = g.uniform01(num_segments)
    s = np.floor(np.exp2(lo_log2 + (hi_log2 - lo_log2) * u)).astype(np.int64)
    return np.clip(s, 1 << lo_log2, 1 << hi_log2)


def segmented(num_segments: int = 20000, lo_log2: int = 4, hi_log2: int = 20,
              bits: int = 32, seed: int = 1):
    """Batched-sort workload: all sizes first, then uniform keys segment by
    segment (one stream, so the keys are one contiguous draw); values are
    the index within the segment.  Returns (keys, values, offsets[S+1])."""
    g = MT19937(seed)
    sizes = segment_sizes(num_segments, lo_log2, hi_log2, g=g)
    offsets = np.zeros(num_segments + 1, dtype=np.uint64)
    np.cumsum(sizes, out=offsets[1:])
    total = int(offsets[-1])
    k = _draw(g, bits, total)
    dt = np.uint32 if bits == 32 else np.uint64
    v = np.empty(total, dtype=dt)
    ramp = np.arange(int(sizes.max()) if sizes.size else 0, dtype=dt)
    for a, n in zip(offsets[:-1].tolist(), sizes.tolist()):
        v[a:a + n] = ramp[:n]
    return k, v, offsets


def requests(num: int, rate_per_s: float, lo_log2: int = 10, hi_log2: int = 24,
             seed: int = 1):
    """Serving workload: Poisson arrivals at ``rate_per_s``; per request
    (dt, n, key bits, has_values, key seed) with dt = -ln(1-u)/rate,
    n = floor(2^(lo + (hi-lo)*u)), width and key-value each from one random
    bit.  Each request's keys come from their own seed so that they can be
    drawn lazily, request by request."""
    g = MT19937(seed)
    out = []
    t = 0.0
    for i in range(num):
        u_dt, u_n = g.uniform01(2)
        bits_word = int(g.u32(1)[0])
        t += -np.log1p(-u_dt) / rate_per_s
        n = int(np.floor(np.exp2(lo_log2 + (hi_log2 - lo_log2) * u_n)))
        n = min(max(n, 1 << lo_log2), 1 << hi_log2)
        out.append({
            "id": i,
            "arrival_s": t,
            "n": n,
            "bits": 64 if (bits_word & 1) else 32,
            "has_values": bool(bits_word & 2),
            "key_seed": int(g.u32(1)[0]),
        })
    return out
