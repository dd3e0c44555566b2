"""Pins of the oracle's merge sort (paper, Section 2.4) against things other
than itself: the definitional stable order by (key, input index) by brute
force, numpy's stable sort, the independently pinned radix oracle, the
sortedness of every run after each merge level, and mutants of its C source
that must each fail one of these pins."""
import ctypes
import itertools
import os
import subprocess

import numpy as np
import pytest

import datagen
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "merge_oracle.c")


def test_brute_force_every_arrangement():
    """All 7! arrangements of a multiset with duplicates and the 32-bit
    extremes, for several run lengths: the output is the stable sort."""
    ms = [0, 0, 2**31, 2**32 - 1, 5, 5, 1]
    for perm in itertools.permutations(range(len(ms))):
        keys = np.array([ms[i] for i in perm], dtype=np.uint32)
        want = sorted(range(len(ms)), key=lambda i: (int(keys[i]), i))
        for tile in (1, 2, 3, 7):
            k, v = oracle.merge_sort(keys, np.arange(len(ms), dtype=np.uint32), tile)
            assert v.tolist() == want and k.tolist() == [int(keys[i]) for i in want]


@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("dist", datagen.DISTRIBUTIONS)
def test_equals_numpy_and_the_radix_oracle(bits, dist):
    n = (1 << 13) + (1 << 12) + 5
    keys = datagen.keys(dist, n, bits, seed=7)
    vals = datagen.values(n, bits)
    order = np.argsort(keys, kind="stable")
    rk, rv = oracle.sort(keys, vals)
    for tile in (1, 5, 64, n):
        k, v = oracle.merge_sort(keys, vals, tile)
        assert np.array_equal(k, keys[order]) and np.array_equal(v.astype(np.int64), order)
        assert np.array_equal(k, rk) and np.array_equal(v, rv)


@pytest.mark.parametrize("tile", [1, 3, 16])
def test_each_level_sorts_runs_of_twice_the_length(tile):
    """After L merge levels every run of tile * 2^L elements is the stable sort
    of the same input range (the last run may be shorter)."""
    n = 1000
    keys = datagen.keys("bucket", n, 32, seed=3)
    vals = datagen.values(n, 32)
    for level in range(0, 8):
        k, v = oracle.merge_sort(keys, vals, tile, level)
        run = tile << level
        for lo in range(0, n, run):
            seg = keys[lo:lo + run]
            o = np.argsort(seg, kind="stable")
            assert np.array_equal(k[lo:lo + run], seg[o])
            assert np.array_equal(v[lo:lo + run].astype(np.int64), o + lo)


def test_edge_lengths():
    for n in (0, 1, 2, 3):
        keys = np.arange(n, dtype=np.uint64)[::-1].copy()
        k, v = oracle.merge_sort(keys, keys.copy(), 2)
        assert k.tolist() == sorted(keys.tolist())
    with pytest.raises(ValueError):
        oracle.merge_sort(np.zeros(4, dtype=np.uint32), None, 0)


MUTANTS = {
    # the merge takes the right run's element on equal keys
    "unstable_merge": ("if (ka[i] <= ka[j]) {", "if (ka[i] < ka[j]) {"),
    # insertion moves an element past equal keys
    "unstable_insertion": ("while (j > lo && key[j - 1] > k) {",
                           "while (j > lo && key[j - 1] >= k) {"),
    # the right run's tail is never copied (its slots keep the old contents)
    "dropped_tail": ("    while (j < hi) {\n        kb[o] = ka[j];",
                     "    while (0) {\n        kb[o] = ka[j];"),
    # the run length does not double: levels merge overlapping ranges
    "width_not_doubled": ("width < n && (levels < 0 || level < levels); width *= 2)",
                          "width < n && (levels < 0 || level < levels); width += 1)"),
    # values taken from the left run's index when the right run wins
    "value_from_wrong_run": ("                vb[o] = va[j];\n            ++j;",
                             "                vb[o] = va[i < mid ? i : j];\n            ++j;"),
}


def _compile(text, path):
    with open(path + ".c", "w") as f:
        f.write(text)
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-shared", "-fPIC", path + ".c", "-o", path])
    lib = ctypes.CDLL(path)
    vp, u64, ci = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int
    lib.oracle_merge_sort.argtypes = [ci, vp, vp, u64, u64, ci]
    lib.oracle_merge_sort.restype = ci
    return lib


def _pins_pass(lib):
    def run(keys, vals, tile):
        k, v = keys.copy(), vals.copy()
        rc = lib.oracle_merge_sort(32 if k.dtype == np.uint32 else 64,
                                   k.ctypes.data_as(ctypes.c_void_p),
                                   v.ctypes.data_as(ctypes.c_void_p), k.size, tile, -1)
        return rc, k, v
    ms = [0, 0, 2**31, 2**32 - 1, 5, 5, 1]
    for perm in itertools.permutations(range(len(ms))):
        keys = np.array([ms[i] for i in perm], dtype=np.uint32)
        want = sorted(range(len(ms)), key=lambda i: (int(keys[i]), i))
        for tile in (1, 2, 3):
            rc, k, v = run(keys, np.arange(len(ms), dtype=np.uint32), tile)
            if rc != 0 or v.tolist() != want:
                return False
    for bits in (32, 64):
        keys = datagen.keys("bucket", 3001, bits, seed=2)
        vals = datagen.values(3001, bits)
        order = np.argsort(keys, kind="stable")
        for tile in (1, 5):
            rc, k, v = run(keys, vals, tile)
            if rc != 0 or not np.array_equal(v.astype(np.int64), order) \
                    or not np.array_equal(k, keys[order]):
                return False
    return True


def test_unmodified_source_passes(tmp_path):
    assert _pins_pass(_compile(open(SRC).read(), str(tmp_path / "orig.so")))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_each_mutant_fails_a_pin(tmp_path, name):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation anchor of {name} not found once"
    assert not _pins_pass(_compile(text.replace(old, new), str(tmp_path / f"{name}.so")))
