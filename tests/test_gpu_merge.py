"""GPU parity of the merge sort (paper, Section 2.4) through the C-ABI: bit
for bit equal to the oracle's merge sort (itself pinned to the stable sort)
on every kind and distribution, at sizes that cover one tile, tile
boundaries, odd numbers of runs at a level and ragged tails; in place; in
every key order; and at the benchmark size through the exact certificate."""
import numpy as np
import pytest
import torch

import datagen
from tests.certify import certify_stable_sort

pytestmark = pytest.mark.gpu

TILE = 8192       # elements per tile sort
PASS_TILE = 2048  # outputs per merge-pass workgroup
SIZES = [1, 2, 3, 100, TILE - 1, TILE, TILE + 1, 2 * TILE + 5, 3 * PASS_TILE + 17,
         5 * TILE + 3, 100003, (1 << 18) + (1 << 17) + 7]
KINDS = [(32, False), (32, True), (64, False), (64, True)]


@pytest.fixture(scope="module")
def rs():
    import paper_1511_03404_amd as rs
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    rs.lib()
    return rs


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


def gpu_merge(rs, keys, vals, in_place=False, order="unsigned", desc=False):
    kd = dev(keys)
    vd = dev(vals) if vals is not None else None
    out = rs.merge_sort(kd, vd, kd if in_place else None, vd if in_place else None,
                        order=order, descending=desc)
    torch.cuda.synchronize()
    if vals is None:
        return host(out), None
    return host(out[0]), host(out[1])


@pytest.mark.parametrize("bits,pairs", KINDS)
def test_merge_matches_oracle(rs, oracle_lib, bits, pairs):
    for n in SIZES:
        for dist in datagen.DISTRIBUTIONS:
            print(f"case merge bits={bits} pairs={pairs} n={n} {dist}", flush=True)
            keys = datagen.keys(dist, n, bits, seed=n + 3)
            vals = datagen.values(n, bits) if pairs else None
            ok, ov = oracle_lib.merge_sort(keys, vals)
            gk, gv = gpu_merge(rs, keys, vals)
            assert np.array_equal(gk, ok), f"keys differ n={n} {dist}"
            if pairs:
                assert np.array_equal(gv, ov), f"values differ n={n} {dist}"


@pytest.mark.parametrize("bits,pairs", KINDS)
def test_merge_in_place_and_extreme_keys(rs, oracle_lib, bits, pairs):
    """In place (an even and an odd number of merge levels), with keys equal
    to the tile sort's padding value (all ones) mixed in."""
    u = np.uint32 if bits == 32 else np.uint64
    for n in (TILE + 7, 2 * TILE + 1, 3 * TILE, 9 * TILE + 11):
        print(f"case merge in-place bits={bits} pairs={pairs} n={n}", flush=True)
        keys = datagen.keys("bucket", n, bits, seed=5)
        keys[::3] = ~u(0)
        keys[1::7] = 0
        vals = datagen.values(n, bits) if pairs else None
        ok, ov = oracle_lib.merge_sort(keys, vals)
        gk, gv = gpu_merge(rs, keys, vals, in_place=True)
        assert np.array_equal(gk, ok)
        if pairs:
            assert np.array_equal(gv, ov)


@pytest.mark.parametrize("order,desc", [("signed", False), ("float", False), ("unsigned", True),
                                        ("float", True)])
@pytest.mark.parametrize("bits", [32, 64])
def test_merge_orders(rs, oracle_lib, bits, order, desc):
    for n in (500, TILE, 3 * TILE + 17):
        print(f"case merge order={order} desc={desc} bits={bits} n={n}", flush=True)
        keys = datagen.keys("uniform", n, bits, seed=9)
        keys[1::4] = keys[::4][: keys[1::4].size]  # duplicates
        vals = datagen.values(n, bits)
        ok, ov = oracle_lib.merge_sort_ordered(keys, vals, order, desc)
        gk, gv = gpu_merge(rs, keys, vals, order=order, desc=desc)
        assert np.array_equal(gk, ok) and np.array_equal(gv, ov)


def test_merge_equals_radix_sort(rs):
    """Both sorts compute the unique stable sort: equal outputs on the device."""
    for bits in (32, 64):
        n = (1 << 20) + 333
        print(f"case merge vs radix bits={bits}", flush=True)
        keys = dev(datagen.keys("gaussian", n, bits, seed=1))
        vals = dev(datagen.values(n, bits))
        mk, mv = rs.merge_sort(keys, vals)
        rk, rv = rs.sort_pairs(keys, vals)
        torch.cuda.synchronize()
        assert torch.equal(mk, rk) and torch.equal(mv, rv)


@pytest.mark.parametrize("bits", [32, 64])
def test_merge_benchmark_size_certificate(rs, bits):
    """At the benchmark sizes (2^26 u32 pairs, 2^25 u64 pairs) the output is
    certified as the stable sort with the exact O(n) certificate."""
    n = (1 << 26) if bits == 32 else (1 << 25)
    print(f"case merge certificate bits={bits} n={n}", flush=True)
    keys = datagen.keys("uniform", n, bits, seed=1)
    vals = datagen.values(n, bits)
    kd, vd = dev(keys), dev(vals)
    ko, vo = rs.merge_sort(kd, vd)
    torch.cuda.synchronize()
    assert certify_stable_sort(keys, host(ko), host(vo)) is None
