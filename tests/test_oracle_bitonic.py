"""Pins of the oracle's bitonic network (paper, Section 2.1; Batcher): the
bare network sorts every 0/1 input of 2, 4, 8 and 16 slots (by the 0-1
principle it then sorts every input of those sizes), the (key, index)
network gives the stable sort by brute force and against numpy on every
distribution, and mutants of its C source fail these pins."""
import ctypes
import itertools
import os
import subprocess

import numpy as np
import pytest

import datagen
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "bitonic_oracle.c")


def zero_one_inputs(N):
    return ((np.arange(1 << N)[:, None] >> np.arange(N)[None, :]) & 1).astype(np.uint64)


@pytest.mark.parametrize("N", [2, 4, 8, 16])
def test_zero_one_principle(N):
    for row in zero_one_inputs(N):
        out = oracle.bitonic_network(row)
        assert np.all(out[:-1] <= out[1:]), row


def test_brute_force_every_arrangement():
    ms = [0, 0, 2**31, 2**32 - 1, 5, 5, 1]
    for perm in itertools.permutations(range(len(ms))):
        keys = np.array([ms[i] for i in perm], dtype=np.uint32)
        want = sorted(range(len(ms)), key=lambda i: (int(keys[i]), i))
        k, v = oracle.bitonic_sort(keys, np.arange(len(ms), dtype=np.uint32))
        assert v.tolist() == want and k.tolist() == [int(keys[i]) for i in want]


@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("dist", datagen.DISTRIBUTIONS)
def test_equals_numpy_and_the_radix_oracle(bits, dist):
    for n in (1, 2, 3, 63, 64, 65, 1000, 1024):
        keys = datagen.keys(dist, n, bits, seed=n)
        if bits == 64 and n > 5:
            keys[3] = np.uint64(2**64 - 1)  # a real key equal to the padding key
        vals = datagen.values(n, bits)
        order = np.argsort(keys, kind="stable")
        k, v = oracle.bitonic_sort(keys, vals)
        assert np.array_equal(k, keys[order]) and np.array_equal(v.astype(np.int64), order)
        rk, rv = oracle.sort(keys, vals)
        assert np.array_equal(k, rk) and np.array_equal(v, rv)


def test_segmented_equals_radix_oracle():
    sizes = [0, 1, 2, 17, 64, 100, 1024, 3]
    off = np.zeros(len(sizes) + 1, dtype=np.uint64)
    off[1:] = np.cumsum(sizes)
    keys = datagen.keys("bucket", int(off[-1]), 32, seed=2)
    vals = datagen.values(int(off[-1]), 32)
    a = oracle.segmented_bitonic_sort(keys, vals, off)
    b = oracle.segmented_sort(keys, vals, off)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


MUTANTS = {
    # the stage direction bit taken one too low
    "wrong_direction_bit": ("int ascending = (i & k) == 0;", "int ascending = (i & (k / 2)) == 0;"),
    # the last step of each stage (distance 1) is skipped
    "missing_last_step": ("for (uint64_t j = k / 2; j >= 1; j /= 2) {",
                          "for (uint64_t j = k / 2; j >= 2; j /= 2) {"),
    # the index tie-break is ignored: equal keys keep network order
    "no_tie_break": ("    return a.idx > b.idx;", "    return 0;"),
    # the last stage (the full-length merge) is skipped
    "missing_last_stage": ("for (uint64_t k = 2; k <= N; k *= 2) {",
                           "for (uint64_t k = 2; k < N; k *= 2) {"),
}


def _compile(text, path):
    with open(path + ".c", "w") as f:
        f.write(text)
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-shared", "-fPIC", path + ".c", "-o", path])
    lib = ctypes.CDLL(path)
    vp, u64, ci = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int
    lib.oracle_bitonic_sort.argtypes = [ci, vp, vp, u64]
    lib.oracle_bitonic_sort.restype = ci
    lib.oracle_bitonic_network.argtypes = [vp, u64]
    lib.oracle_bitonic_network.restype = ci
    return lib


def _pins_pass(lib):
    for N in (2, 4, 8, 16):
        for row in zero_one_inputs(N):
            w = row.copy()
            if lib.oracle_bitonic_network(w.ctypes.data_as(ctypes.c_void_p), N) != 0:
                return False
            if not np.all(w[:-1] <= w[1:]):
                return False
    ms = [0, 0, 2**31, 2**32 - 1, 5, 5, 1]
    for perm in itertools.permutations(range(len(ms))):
        keys = np.array([ms[i] for i in perm], dtype=np.uint32)
        vals = np.arange(len(ms), dtype=np.uint32)
        if lib.oracle_bitonic_sort(32, keys.ctypes.data_as(ctypes.c_void_p),
                                   vals.ctypes.data_as(ctypes.c_void_p), len(ms)) != 0:
            return False
        if vals.tolist() != sorted(range(len(ms)), key=lambda i: (ms[perm[i]], i)):
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
