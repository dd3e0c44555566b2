"""Pins for the CPU oracle (paper, Section 2.6: LSD order, stable counting
sort per digit).  Each test ties the oracle to something other than itself:
brute force against a definitional insertion sort and a library stable sort,
a hand-worked example, closed forms of the distributions, r-invariance, and
the exact O(n) certificate.  ``test_oracle_mutants.py`` shows that planted
mistakes in the oracle fail these pins."""
import itertools
import os

import numpy as np
import pytest

import datagen
from tests.certify import certify_stable_sort, certify_sorted_keys

HERE = os.path.dirname(os.path.abspath(__file__))


def insertion_sort_stable(pairs):
    """Definitional O(n^2) stable sort: an element moves left only past
    strictly greater keys."""
    out = []
    for kv in pairs:
        j = len(out)
        while j > 0 and out[j - 1][0] > kv[0]:
            j -= 1
        out.insert(j, kv)
    return out


MULTISETS_32 = [
    [0, 0, 2**31, 2**32 - 1, 5, 5, 5, 1],
    [7, 7, 7, 7, 7, 7, 7, 7],
    [2**31 - 1, 2**31, 0, 2**32 - 1, 255, 256, 65535, 65536],
    [3, 1, 2],
    [1],
]
MULTISETS_64 = [
    [1 << 32, 0, 1 << 32, 1, 2**63, 2**64 - 1, 255 << 56, 0],
    [2**63, 2**63 - 1, 1 << 56, 1 << 55, 0xFFFFFFFF, 0x100000000, 5, 5],
]


@pytest.mark.parametrize("bits,ms", [(32, m) for m in MULTISETS_32] + [(64, m) for m in MULTISETS_64])
def test_bruteforce_all_permutations(oracle_lib, bits, ms):
    dt = np.uint32 if bits == 32 else np.uint64
    n = len(ms)
    perms = list(itertools.permutations(range(n)))
    if n == 8:
        perms = perms[::3]  # 13,440 of the 40,320 orders keeps the CPU suite quick
    for perm in perms:
        keys = np.array([ms[i] for i in perm], dtype=dt)
        vals = np.arange(n, dtype=dt)
        ok, ov = oracle_lib.sort(keys, vals)
        want = insertion_sort_stable([(int(k), i) for i, k in enumerate(keys)])
        assert [int(x) for x in ok] == [k for k, _ in want]
        assert [int(x) for x in ov] == [i for _, i in want]
        # library stable sort (Python's sorted is stable by contract)
        lib = sorted(range(n), key=lambda i: int(keys[i]))
        assert [int(x) for x in ov] == lib


def test_full_8_permutations_u32(oracle_lib):
    """Every one of the 8! orders of a multiset with duplicates and the
    32-bit extremes, checked by the exact certificate."""
    ms = np.array(MULTISETS_32[0], dtype=np.uint32)
    for perm in itertools.permutations(range(8)):
        keys = ms[list(perm)]
        ok, ov = oracle_lib.sort(keys, np.arange(8, dtype=np.uint32))
        assert certify_stable_sort(keys, ok, ov) is None


def _load_golden():
    rec = {}
    with open(os.path.join(HERE, "golden", "worked_example_r4.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, *items = line.split()
            rec[name] = items
    return rec


def test_hand_worked_example(oracle_lib):
    g = _load_golden()
    keys = np.array([int(x, 16) for x in g["keys"]], dtype=np.uint32)
    vals = np.array([int(x) for x in g["vals"]], dtype=np.uint32)
    for p, tag in ((1, "pass0"), (2, "pass1")):
        k, v = oracle_lib.sort(keys, vals, r=4, passes=p)
        assert [int(x) for x in k] == [int(x, 16) for x in g[tag + "_keys"]]
        assert [int(x) for x in v] == [int(x) for x in g[tag + "_vals"]]
    k, v = oracle_lib.sort(keys, vals, r=4)
    assert [int(x) for x in k] == [int(x, 16) for x in g["sorted_keys"]]
    assert [int(x) for x in v] == [int(x) for x in g["sorted_vals"]]
    h = oracle_lib.digit_histograms(keys, r=4)
    for p, tag in ((0, "hist0"), (1, "hist1")):
        want = np.zeros(16, dtype=np.uint64)
        for item in g[tag]:
            b, c = item.split("=")
            want[int(b)] = int(c)
        assert np.array_equal(h[p], want)
    assert h[2:].sum(axis=1).tolist() == [6] * 6 and (h[2:, 0] == 6).all()


@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("dist", datagen.DISTRIBUTIONS)
def test_numpy_stable_argsort_agrees(oracle_lib, bits, dist):
    n = (1 << 15) + (1 << 14)  # a 2^n + 2^(n-1) length, as the paper tests
    keys = datagen.keys(dist, n, bits, seed=1)
    vals = datagen.values(n, bits)
    ok, ov = oracle_lib.sort(keys, vals)
    assert np.array_equal(ok, np.sort(keys, kind="stable"))
    assert np.array_equal(ov.astype(np.int64), np.argsort(keys, kind="stable"))
    assert certify_stable_sort(keys, ok, ov) is None


@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("r", [1, 2, 4, 8, 11, 16])
def test_result_independent_of_digit_width(oracle_lib, bits, r):
    n = 5000
    keys = datagen.keys("bucket", n, bits, seed=3)
    keys[::7] = datagen.keys("uniform", keys[::7].size, bits, seed=4)
    vals = datagen.values(n, bits)
    k8, v8 = oracle_lib.sort(keys, vals, r=8)
    kr, vr = oracle_lib.sort(keys, vals, r=r)
    assert np.array_equal(k8, kr) and np.array_equal(v8, vr)


@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("r", [3, 8, 11])
def test_state_after_each_pass(oracle_lib, bits, r):
    """After pass p the order is the stable sort by the low (p+1)*r bits."""
    n = 3000
    keys = datagen.keys("uniform", n, bits, seed=5)
    vals = datagen.values(n, bits)
    d = (bits + r - 1) // r
    for p in range(d):
        k, v = oracle_lib.sort(keys, vals, r=r, passes=p + 1)
        nbits = min((p + 1) * r, bits)
        mask = (1 << nbits) - 1
        low = np.array([int(x) & mask for x in keys], dtype=np.uint64)
        assert np.array_equal(v.astype(np.int64), np.argsort(low, kind="stable"))
        assert np.array_equal(k, keys[v.astype(np.int64)])


@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("r", [4, 8, 11])
def test_histograms(oracle_lib, bits, r):
    n = 4097
    keys = datagen.keys("gaussian", n, bits, seed=2)
    h = oracle_lib.digit_histograms(keys, r=r)
    d = (bits + r - 1) // r
    assert h.shape == (d, 1 << r)
    assert (h.sum(axis=1) == n).all()
    for p in range(d):
        dig = [(int(x) >> (p * r)) & ((1 << r) - 1) for x in keys]
        assert np.array_equal(h[p], np.bincount(dig, minlength=1 << r).astype(np.uint64))


@pytest.mark.parametrize("bits", [32, 64])
def test_closed_forms(oracle_lib, bits):
    n = 10000
    vals = datagen.values(n, bits)
    # zero: every key equal -> the values stay the identity
    z = datagen.keys("zero", n, bits)
    k, v = oracle_lib.sort(z, vals)
    assert np.array_equal(v, vals) and not k.any()
    # sorted: already in order -> the identity
    s = datagen.keys("sorted", n, bits)
    k, v = oracle_lib.sort(s, vals)
    assert np.array_equal(k, s) and np.array_equal(v, vals)
    # reverse: runs of equal keys keep ascending index, runs come reversed
    rv = datagen.keys("reverse", n, bits)
    k, v = oracle_lib.sort(rv, vals)
    assert np.array_equal(k, rv[::-1])
    if np.unique(rv).size == n:
        assert np.array_equal(v, vals[::-1])
    else:
        assert certify_stable_sort(rv, k, v) is None
    # bucket: 64 distinct values; the output histogram equals the input's
    b = datagen.keys("bucket", n, bits)
    k, v = oracle_lib.sort(b, vals)
    ui, ci = np.unique(b, return_counts=True)
    uo, co = np.unique(k, return_counts=True)
    assert ui.size == 64 and np.array_equal(ui, uo) and np.array_equal(ci, co)
    # idempotent
    k2, v2 = oracle_lib.sort(k, v)
    assert np.array_equal(k2, k) and np.array_equal(v2, v)


@pytest.mark.parametrize("n", [0, 1, 2, 3, 63, 64, 65])
def test_tiny_lengths(oracle_lib, n):
    for bits in (32, 64):
        keys = datagen.keys("uniform", n, bits, seed=9)
        ok, ov = oracle_lib.sort(keys, datagen.values(n, bits))
        assert certify_stable_sort(keys, ok, ov) is None
        ko, _ = oracle_lib.sort(keys)
        assert certify_sorted_keys(keys, ko) is None


def test_segmented_equals_per_segment(oracle_lib):
    sizes = [0, 1, 17, 0, 300, 2, 1000, 0]
    off = np.zeros(len(sizes) + 1, dtype=np.uint64)
    off[1:] = np.cumsum(sizes)
    tot = int(off[-1])
    keys = datagen.keys("bucket", tot, 32, seed=11)
    vals = datagen.values(tot)
    k, v = oracle_lib.segmented_sort(keys, vals, off)
    for s in range(len(sizes)):
        a, b = int(off[s]), int(off[s + 1])
        ks, vs = oracle_lib.sort(keys[a:b], vals[a:b])
        assert np.array_equal(k[a:b], ks) and np.array_equal(v[a:b], vs)


def test_certificate_has_teeth(oracle_lib):
    """The certificate rejects each kind of wrong answer."""
    n = 2000
    keys = datagen.keys("bucket", n, 32, seed=6)
    ok, ov = oracle_lib.sort(keys, datagen.values(n))
    assert certify_stable_sort(keys, ok, ov) is None
    # swap two equal keys (with their values): unstable
    i = int(np.nonzero(ok[1:] == ok[:-1])[0][0])
    k2, v2 = ok.copy(), ov.copy()
    v2[[i, i + 1]] = v2[[i + 1, i]]
    assert "unstable" in certify_stable_sort(keys, k2, v2)
    # swap two unequal keys with their values: not sorted
    j = int(np.nonzero(ok[1:] != ok[:-1])[0][0])
    k3, v3 = ok.copy(), ov.copy()
    k3[[j, j + 1]] = k3[[j + 1, j]]
    v3[[j, j + 1]] = v3[[j + 1, j]]
    assert "decrease" in certify_stable_sort(keys, k3, v3)
    # duplicate a value: not a permutation
    v4 = ov.copy()
    v4[0] = v4[1]
    assert "permutation" in certify_stable_sort(keys, ok, v4)
    # a key that does not belong to its value
    k5 = ok.copy()
    k5[-1] = k5[-1] ^ np.uint32(1)
    assert certify_stable_sort(keys, k5, ov) is not None


def test_mt19937_standard_check_values():
    """The C++ standard fixes the 10000th output of a default-seeded
    mt19937 (seed 5489) at 4123659995."""
    g = datagen.MT19937(5489)
    assert int(g.u32(10000)[-1]) == 4123659995
    # 64-bit keys are two consecutive outputs, high word first
    a = datagen.MT19937(5489).u32(4)
    b = datagen.MT19937(5489).u64(2)
    assert int(b[0]) == (int(a[0]) << 32) | int(a[1])
    assert int(b[1]) == (int(a[2]) << 32) | int(a[3])


def test_distribution_recipes():
    n = 1 << 16
    u = datagen.keys("uniform", n, 32)
    assert np.array_equal(u, datagen.MT19937(1).u32(n))
    g = datagen.keys("gaussian", n, 32)
    w = datagen.MT19937(1).u32(4 * n).astype(np.uint64).reshape(n, 4)
    assert np.array_equal(g, (w.sum(axis=1) // 4).astype(np.uint32))
    assert abs(float(g.mean()) / 2**31 - 1.0) < 0.01
    g64 = datagen.keys("gaussian", 1000, 64)
    w64 = datagen.MT19937(1).u64(4000).reshape(1000, 4)
    exact = [sum(int(x) for x in row) // 4 for row in w64]
    assert [int(x) for x in g64] == exact
    s = datagen.keys("sorted", n, 64)
    assert (s[1:] >= s[:-1]).all()
    rv = datagen.keys("reverse", n, 64)
    assert np.array_equal(rv, s[::-1])
    b = datagen.keys("bucket", n, 64)
    assert np.unique(b).size == 64
    assert (b >> np.uint64(32)).any()  # the high word is random too
    assert not datagen.keys("zero", n, 32).any()


def test_segmented_certificate_has_teeth(oracle_lib):
    from tests.certify import certify_segmented
    sizes = [5, 0, 300, 2, 1000]
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    total = int(off[-1])
    keys = datagen.keys("bucket", total, 32, seed=8)
    vals = (np.arange(total) - np.repeat(off[:-1], sizes)).astype(np.uint32)
    k, v = oracle_lib.segmented_sort(keys, vals, off)
    assert certify_segmented(keys, k, v, off) is None
    # a sort across a segment boundary is caught
    kk, vv = oracle_lib.sort(keys, np.arange(total, dtype=np.uint32))
    assert certify_segmented(keys, kk, vv, off) is not None
    # an unstable swap inside a segment is caught
    a, b = int(off[4]), int(off[5])
    i = a + int(np.nonzero(k[a + 1:b] == k[a:b - 1])[0][0])
    k2, v2 = k.copy(), v.copy()
    v2[[i, i + 1]] = v2[[i + 1, i]]
    assert "unstable" in certify_segmented(keys, k2, v2, off)


def _mix64(x):
    """splitmix64's finalizer (a published 64-bit mixing function), on uint64 arrays."""
    x = x.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        x ^= x >> np.uint64(30)
        x *= np.uint64(0xBF58476D1CE4E5B9)
        x ^= x >> np.uint64(27)
        x *= np.uint64(0x94D049BB133111EB)
        x ^= x >> np.uint64(31)
    return x


def multiset_hash(keys, vals=None):
    """Order-independent hash of the multiset of (key, value) pairs: the sum
    mod 2^64 of a mixed 64-bit word per pair."""
    k = np.asarray(keys).astype(np.uint64)
    h = _mix64(k)
    if vals is not None:
        with np.errstate(over="ignore"):
            h = _mix64(h ^ (np.asarray(vals).astype(np.uint64) * np.uint64(0x9E3779B97F4A7C15)))
    with np.errstate(over="ignore"):
        return int(h.sum(dtype=np.uint64))


@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("dist", datagen.DISTRIBUTIONS)
def test_multiset_hash_preserved(oracle_lib, bits, dist):
    """The output is a rearrangement of the input: the multiset hash of the
    (key, value) pairs is the same before and after every oracle sort."""
    n = (1 << 14) + 77
    keys = datagen.keys(dist, n, bits, seed=5)
    vals = datagen.values(n, bits)
    want = multiset_hash(keys, vals)
    for k, v in (oracle_lib.sort(keys, vals), oracle_lib.merge_sort(keys, vals),
                 oracle_lib.bitonic_sort(keys[:4096], vals[:4096])):
        ref = want if k.size == n else multiset_hash(keys[:4096], vals[:4096])
        assert multiset_hash(k, v) == ref


def test_multiset_hash_has_teeth(oracle_lib):
    """A changed key, a duplicated pair or a pair split apart changes the hash."""
    keys = datagen.keys("bucket", 5000, 32, seed=6)
    vals = datagen.values(5000, 32)
    k, v = oracle_lib.sort(keys, vals)
    h = multiset_hash(k, v)
    k2 = k.copy(); k2[17] ^= np.uint32(1)
    assert multiset_hash(k2, v) != h
    k3, v3 = k.copy(), v.copy(); k3[5], v3[5] = k3[6], v3[6]
    assert multiset_hash(k3, v3) != h
    v4 = v.copy(); v4[[3, 4000]] = v4[[4000, 3]]
    assert multiset_hash(k, v4) != h or k[3] == k[4000]
