"""GPU parity of the tiny-segment class of the segmented sort: segments of
2 .. 1024 elements are sorted by one wave each with a bitonic network on
(key, position) pairs (paper, Section 2.1), which must give bit for bit the
stable sort -- the oracle's radix sort and its bitonic network both -- on
every kind, register count (64 to 1024 slots), key order and in place, and
the same output as the one-workgroup radix sort (cap 0)."""
import numpy as np
import pytest
import torch

import datagen

pytestmark = pytest.mark.gpu

KINDS = [(32, False), (32, True), (64, False), (64, True)]
# every register count, both sides of each power of two, and the edges
TINY_SIZES = [1, 2, 3, 31, 32, 33, 63, 64, 65, 100, 127, 128, 129, 255, 256, 257, 511, 512, 513,
              777, 1023, 1024, 1025, 4096, 0, 2]


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


def batch(sizes, bits, pairs, dist, seed):
    off = np.zeros(len(sizes) + 1, dtype=np.uint64)
    off[1:] = np.cumsum(sizes)
    total = int(off[-1])
    keys = datagen.keys(dist, total, bits, seed=seed)
    vals = datagen.values(total, bits) if pairs else None
    return keys, vals, off


def run(rs, ctx, keys, vals, off, in_place=False, order="unsigned", desc=False):
    kd = dev(keys)
    vd = dev(vals) if vals is not None else None
    ko, vo = rs.segmented_sort(kd, vd, dev(off.view(np.int64)), kd if in_place else None,
                               vd if in_place else None, ctx=ctx, order=order, descending=desc)
    torch.cuda.synchronize()
    return host(ko), (host(vo) if vo is not None else None)


@pytest.mark.parametrize("bits,pairs", KINDS)
def test_tiny_segments_match_oracles(rs, oracle_lib, bits, pairs):
    ctx = rs.Context(0)
    assert ctx.tiny_cap() == 1024
    for dist in datagen.DISTRIBUTIONS:
        print(f"case tiny bits={bits} pairs={pairs} {dist}", flush=True)
        keys, vals, off = batch(TINY_SIZES * 3, bits, pairs, dist, seed=bits)
        ok, ov = oracle_lib.segmented_sort(keys, vals, off)
        bk, bv = oracle_lib.segmented_bitonic_sort(keys, vals, off)
        assert np.array_equal(ok, bk) and (not pairs or np.array_equal(ov, bv))
        gk, gv = run(rs, ctx, keys, vals, off)
        assert np.array_equal(gk, ok), dist
        if pairs:
            assert np.array_equal(gv, ov), dist
    ctx.close()


@pytest.mark.parametrize("bits,pairs", KINDS)
def test_tiny_in_place_and_against_radix_class(rs, oracle_lib, bits, pairs):
    rng = np.random.RandomState(bits + pairs)
    sizes = list(rng.randint(2, 1025, size=3000)) + [1024] * 10 + [2] * 10
    keys, vals, off = batch(sizes, bits, pairs, "bucket", seed=4)
    ok, ov = oracle_lib.segmented_sort(keys, vals, off)
    bit_ctx = rs.Context(0)
    rad_ctx = rs.Context(0)
    assert rad_ctx.tiny_cap(0) == 0
    for in_place in (False, True):
        print(f"case tiny in_place={in_place} bits={bits} pairs={pairs}", flush=True)
        gk, gv = run(rs, bit_ctx, keys, vals, off, in_place)
        rk, rv = run(rs, rad_ctx, keys, vals, off, in_place)
        assert np.array_equal(gk, ok) and np.array_equal(rk, ok)
        if pairs:
            assert np.array_equal(gv, ov) and np.array_equal(rv, ov)
    bit_ctx.close()
    rad_ctx.close()


@pytest.mark.parametrize("order,desc", [("signed", False), ("float", True), ("unsigned", True)])
@pytest.mark.parametrize("bits", [32, 64])
def test_tiny_orders(rs, oracle_lib, bits, order, desc):
    ctx = rs.Context(0)
    keys, vals, off = batch(TINY_SIZES, bits, True, "uniform", seed=8)
    keys[::5] = keys[1::5][: keys[::5].size] if keys.size > 1 else keys[::5]
    print(f"case tiny order={order} desc={desc} bits={bits}", flush=True)
    ok, ov = oracle_lib.segmented_sort_ordered(keys, vals, off, order, desc)
    gk, gv = run(rs, ctx, keys, vals, off, order=order, desc=desc)
    assert np.array_equal(gk, ok) and np.array_equal(gv, ov)
    ctx.close()


@pytest.mark.parametrize("cap", [2, 64, 100, 1000])
def test_tiny_cap_values(rs, oracle_lib, cap):
    """Any cap splits the segments between the network and the radix sort;
    the output does not change."""
    ctx = rs.Context(0)
    assert ctx.tiny_cap(cap) == cap
    keys, vals, off = batch(TINY_SIZES, 32, True, "gaussian", seed=cap)
    print(f"case tiny cap={cap}", flush=True)
    ok, ov = oracle_lib.segmented_sort(keys, vals, off)
    gk, gv = run(rs, ctx, keys, vals, off)
    assert np.array_equal(gk, ok) and np.array_equal(gv, ov)
    ctx.close()
