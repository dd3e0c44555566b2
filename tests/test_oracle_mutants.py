"""Mutation check of the oracle's pins: each plausible mistake, planted in a
copy of the oracle's C source on the CPU, must fail at least one pin, while
the unmodified source passes all of them.  Mutations are chosen so that the
mutant stays in bounds (it computes a wrong answer, it does not crash)."""
import ctypes
import itertools
import os
import subprocess

import numpy as np
import pytest

import datagen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lsd_oracle.c")

MUTANTS = {
    # placement walks the input backwards: equal digits come out reversed
    "unstable_placement": ("for (uint64_t i = 0; i < n; ++i) { /* ascending i: stability */",
                           "for (uint64_t i = n; i-- > 0;) {"),
    # digit taken one bit too high
    "shifted_digit": ("int shift = p * r;", "int shift = p * r + 1;"),
    # the last, partial digit is dropped (floor instead of ceiling)
    "dropped_last_digit": ("return (key_bits + r - 1) / r;", "return key_bits / r;"),
    # digit mask loses its lowest bit
    "bad_mask": ("return (key >> shift) & ((UINT64_C(1) << r) - 1);",
                 "return (key >> shift) & ((UINT64_C(1) << r) - 2);"),
    # values read from the destination index instead of the source
    "value_from_wrong_index": ("vb[dst] = va[i];", "vb[dst] = va[dst < n ? dst : 0];"),
    # most significant digit first
    "msd_order": ("counting_pass(ka, va, kt, vt, n, p, r, cnt, start);",
                  "counting_pass(ka, va, kt, vt, n, passes_to_run - 1 - p, r, cnt, start);"),
    # count step skips the first element
    "count_skips_first": ("for (uint64_t i = 0; i < n; ++i)\n        cnt[digit_of(key[i], p, r)] += 1;",
                          "for (uint64_t i = 1; i < n; ++i)\n        cnt[digit_of(key[i], p, r)] += 1;\n    cnt[0] += n > 0;"),
}


def _compile(src_text, out_path):
    c_path = out_path + ".c"
    with open(c_path, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-shared", "-fPIC", c_path, "-o", out_path])
    lib = ctypes.CDLL(out_path)
    vp, u64, ci = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int
    lib.oracle_sort_u32.argtypes = [vp, vp, u64, ci, ci]
    lib.oracle_sort_u64.argtypes = [vp, vp, u64, ci, ci]
    return lib


def _sort(lib, keys, vals, r=8):
    k = keys.copy()
    v = vals.copy()
    f = lib.oracle_sort_u32 if k.dtype == np.uint32 else lib.oracle_sort_u64
    rc = f(k.ctypes.data_as(ctypes.c_void_p), v.ctypes.data_as(ctypes.c_void_p), k.size, r, -1)
    return rc, k, v


def _pins_pass(lib):
    # brute force against the definitional stable order (Python's sorted)
    ms = [0, 0, 2**31, 2**32 - 1, 5, 5, 1]
    for perm in itertools.permutations(range(len(ms))):
        keys = np.array([ms[i] for i in perm], dtype=np.uint32)
        vals = np.arange(len(ms), dtype=np.uint32)
        rc, k, v = _sort(lib, keys, vals)
        if rc != 0 or [int(x) for x in v] != sorted(range(len(ms)), key=lambda i: int(keys[i])):
            return False
    # library stable sort on seeded inputs, both widths, r = 8 and 11
    for bits in (32, 64):
        for r in (8, 11):
            keys = datagen.keys("bucket", 3000, bits, seed=2)
            keys[::5] = datagen.keys("uniform", keys[::5].size, bits, seed=3)
            vals = datagen.values(3000, bits)
            rc, k, v = _sort(lib, keys, vals, r)
            if rc != 0 or not np.array_equal(v.astype(np.int64), np.argsort(keys, kind="stable")):
                return False
            if not np.array_equal(k, np.sort(keys)):
                return False
    return True


def test_original_passes(tmp_path):
    with open(SRC) as f:
        lib = _compile(f.read(), str(tmp_path / "orig.so"))
    assert _pins_pass(lib)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_fails_a_pin(tmp_path, name):
    old, new = MUTANTS[name]
    with open(SRC) as f:
        src = f.read()
    assert old in src, "mutation site moved: update the mutant table"
    lib = _compile(src.replace(old, new), str(tmp_path / (name + ".so")))
    assert not _pins_pass(lib), "planted mistake %r went unnoticed" % name
