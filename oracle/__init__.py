"""CPU oracle for the LSD radix sort -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library in
``paper_1511_03404_amd``) never loads it and shares no code with it.

The arithmetic lives in plain C compiled with gcc: ``lsd_oracle.c``, a
stable counting-sort LSD radix sort written from the paper's description
(Section 2.6), ``merge_oracle.c``, the stable merge sort of Section 2.4, and
``bitonic_oracle.c``, Batcher's bitonic network of Section 2.1.
This module only marshals numpy arrays into them (and holds the key-order
maps, written in numpy from their definitions).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "lsd_oracle.c"), os.path.join(_HERE, "merge_oracle.c"),
         os.path.join(_HERE, "bitonic_oracle.c")]
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-shared",
                               "-fPIC", *_SRCS, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        vp, u64, ci = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int
        lib.oracle_sort_u32.argtypes = [vp, vp, u64, ci, ci]
        lib.oracle_sort_u64.argtypes = [vp, vp, u64, ci, ci]
        lib.oracle_digit_histograms.argtypes = [vp, u64, ci, ci, vp]
        lib.oracle_segmented_sort.argtypes = [ci, vp, vp, vp, u64, ci]
        lib.oracle_merge_sort.argtypes = [ci, vp, vp, u64, u64, ci]
        lib.oracle_bitonic_sort.argtypes = [ci, vp, vp, u64]
        lib.oracle_bitonic_network.argtypes = [vp, u64]
        for f in (lib.oracle_sort_u32, lib.oracle_sort_u64, lib.oracle_digit_histograms,
                  lib.oracle_segmented_sort, lib.oracle_merge_sort, lib.oracle_bitonic_sort,
                  lib.oracle_bitonic_network):
            f.restype = ci
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check_pair(keys, vals):
    keys = np.asarray(keys)
    if keys.dtype not in (np.uint32, np.uint64):
        raise TypeError("keys must be uint32 or uint64")
    if vals is not None:
        vals = np.asarray(vals)
        if vals.dtype != keys.dtype or vals.shape != keys.shape:
            raise TypeError("values must match the keys' dtype and length")
    return keys, vals


def sort(keys, vals=None, r: int = 8, passes: int = -1):
    """Stable LSD sort by unsigned key.  Returns new arrays (keys, vals or None).

    ``passes`` < 0 runs all ceil(K/r) passes; a smaller count returns the
    state after that many counting-sort passes."""
    keys, vals = _check_pair(keys, vals)
    k = np.array(keys, copy=True, order="C")
    v = None if vals is None else np.array(vals, copy=True, order="C")
    f = _load().oracle_sort_u32 if k.dtype == np.uint32 else _load().oracle_sort_u64
    if f(_ptr(k), _ptr(v), k.size, r, passes) != 0:
        raise ValueError("oracle rejected the arguments")
    return k, v


def digit_histograms(keys, r: int = 8) -> np.ndarray:
    """hist[p, b] = number of input keys whose digit p equals b."""
    keys = np.ascontiguousarray(keys)
    bits = 32 if keys.dtype == np.uint32 else 64
    d = (bits + r - 1) // r
    h = np.zeros((d, 1 << r), dtype=np.uint64)
    if _load().oracle_digit_histograms(_ptr(keys), keys.size, bits, r, _ptr(h)) != 0:
        raise ValueError("oracle rejected the arguments")
    return h


def segmented_sort(keys, vals, offsets, r: int = 8):
    """Sort each segment [offsets[s], offsets[s+1]) on its own."""
    keys, vals = _check_pair(keys, vals)
    k = np.array(keys, copy=True, order="C")
    v = None if vals is None else np.array(vals, copy=True, order="C")
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    bits = 32 if k.dtype == np.uint32 else 64
    if off.size < 1 or int(off[-1]) > k.size:
        raise ValueError("offsets out of range")
    if _load().oracle_segmented_sort(bits, _ptr(k), _ptr(v), _ptr(off), off.size - 1, r) != 0:
        raise ValueError("oracle rejected the arguments")
    return k, v


def merge_sort(keys, vals=None, tile: int = 1, levels: int = -1):
    """Stable merge sort by unsigned key (paper, Section 2.4): runs of ``tile``
    elements sorted by insertion, then merged pairwise level by level.
    ``levels`` < 0 runs every level; otherwise returns the state after that
    many merge levels (runs of tile * 2^levels elements sorted)."""
    keys, vals = _check_pair(keys, vals)
    k = np.array(keys, copy=True, order="C")
    v = None if vals is None else np.array(vals, copy=True, order="C")
    bits = 32 if k.dtype == np.uint32 else 64
    if _load().oracle_merge_sort(bits, _ptr(k), _ptr(v), k.size, tile, levels) != 0:
        raise ValueError("oracle rejected the arguments")
    return k, v


def bitonic_sort(keys, vals=None):
    """Batcher's bitonic network (paper, Section 2.1) over the next power of
    two, on (key, input index) pairs: the stable sort by unsigned key."""
    keys, vals = _check_pair(keys, vals)
    k = np.array(keys, copy=True, order="C")
    v = None if vals is None else np.array(vals, copy=True, order="C")
    bits = 32 if k.dtype == np.uint32 else 64
    if _load().oracle_bitonic_sort(bits, _ptr(k), _ptr(v), k.size) != 0:
        raise ValueError("oracle rejected the arguments")
    return k, v


def bitonic_network(words):
    """The bare network (no index tie-break) on a power-of-two number of
    uint64 words."""
    w = np.array(words, dtype=np.uint64, copy=True, order="C")
    if _load().oracle_bitonic_network(_ptr(w), w.size) != 0:
        raise ValueError("oracle rejected the arguments")
    return w


def segmented_bitonic_sort(keys, vals, offsets):
    """bitonic_sort of every segment [offsets[s], offsets[s+1]) on its own."""
    keys, vals = _check_pair(keys, vals)
    k = np.array(keys, copy=True, order="C")
    v = None if vals is None else np.array(vals, copy=True, order="C")
    off = np.asarray(offsets, dtype=np.uint64)
    for a, b in zip(off[:-1], off[1:]):
        a, b = int(a), int(b)
        if b > a:
            ks, vs = bitonic_sort(k[a:b], None if v is None else v[a:b])
            k[a:b] = ks
            if v is not None:
                v[a:b] = vs
    return k, v


# ---------------------------------------------------------------------------
# Key orders other than unsigned ascending.  Each order is a bijection of the
# key bits that is monotone from the wanted order to the unsigned order, so
# the stable unsigned sort of the mapped keys, mapped back, is the stable sort
# in that order.  Written from the definitions:
#   signed      two's complement: adding 2^(K-1) (mod 2^K) -- flipping the
#               sign bit -- turns [-2^(K-1), 2^(K-1)) into [0, 2^K) in order;
#   float       IEEE 754 totalOrder on the bit patterns: non-negative values
#               grow with their bit pattern, negative ones shrink, so negative
#               patterns are complemented and the sign bit of the others set;
#   descending  complementing reverses the unsigned order; ties keep their
#               input order because the sort of the complemented keys is
#               stable.

ORDERS = ("unsigned", "signed", "float")


def order_key(keys, order="unsigned", descending=False):
    """Map unsigned key bit patterns (uint32/uint64) to the sort key."""
    k = np.asarray(keys)
    if k.dtype not in (np.uint32, np.uint64):
        raise TypeError("key bit patterns must be uint32 or uint64")
    if order not in ORDERS:
        raise ValueError(f"order must be one of {ORDERS}")
    sign = k.dtype.type(1) << k.dtype.type(8 * k.dtype.itemsize - 1)
    if order == "signed":
        m = k ^ sign
    elif order == "float":
        m = np.where((k & sign) != 0, ~k, k | sign).astype(k.dtype)
    else:
        m = k.copy()
    return ~m if descending else m


def order_unkey(mapped, order="unsigned", descending=False):
    """Inverse of order_key."""
    m = np.asarray(mapped)
    if descending:
        m = ~m
    sign = m.dtype.type(1) << m.dtype.type(8 * m.dtype.itemsize - 1)
    if order == "signed":
        return m ^ sign
    if order == "float":
        return np.where((m & sign) != 0, m ^ sign, ~m).astype(m.dtype)
    return m.copy()


def sort_ordered(keys, vals=None, order="unsigned", descending=False):
    """Stable sort of key bit patterns in the given order (values follow)."""
    keys, vals = _check_pair(keys, vals)
    k, v = sort(order_key(keys, order, descending), vals)
    return order_unkey(k, order, descending), v


def merge_sort_ordered(keys, vals=None, order="unsigned", descending=False, tile: int = 1):
    """merge_sort in the given order."""
    keys, vals = _check_pair(keys, vals)
    k, v = merge_sort(order_key(keys, order, descending), vals, tile)
    return order_unkey(k, order, descending), v


def segmented_sort_ordered(keys, vals, offsets, order="unsigned", descending=False):
    """segmented_sort in the given order."""
    keys, vals = _check_pair(keys, vals)
    mapped = order_key(keys, order, descending)
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    k, v = segmented_sort(mapped, vals, off)
    out = np.array(keys, copy=True)
    lo, hi = (int(off[0]), int(off[-1])) if off.size else (0, 0)
    out[lo:hi] = order_unkey(k[lo:hi], order, descending)
    return out, v
