"""Pins of the oracle's key orders (signed, float, descending) against things
other than itself: numpy's stable sorts of typed arrays, the IEEE 754
totalOrder written out by hand for the special values, and a definitional
stable descending sort on small inputs."""
import itertools

import numpy as np
import pytest

import oracle

INT = {32: np.int32, 64: np.int64}
UINT = {32: np.uint32, 64: np.uint64}
FLT = {32: np.float32, 64: np.float64}


def ints(bits, n, seed):
    rng = np.random.RandomState(seed)
    t = INT[bits]
    info = np.iinfo(t)
    x = rng.randint(-1000, 1000, size=n).astype(t)
    x[::7] = rng.randint(info.min, info.max, size=x[::7].size, dtype=np.int64).astype(t) \
        if bits == 32 else (rng.randint(0, 2**62, size=x[::7].size).astype(t) *
                            rng.choice([-2, 1], size=x[::7].size).astype(t))
    x[:4] = [info.min, -1, 0, info.max]
    return x


@pytest.mark.parametrize("bits", [32, 64])
def test_signed_equals_numpy_stable(bits):
    x = ints(bits, 5000, bits)
    vals = np.arange(x.size, dtype=UINT[bits])
    k, v = oracle.sort_ordered(x.view(UINT[bits]), vals, "signed")
    order = np.argsort(x, kind="stable")
    assert np.array_equal(k.view(INT[bits]), x[order])
    assert np.array_equal(v, order.astype(UINT[bits]))


@pytest.mark.parametrize("bits", [32, 64])
def test_float_equals_numpy_stable_without_nan_and_signed_zero(bits):
    rng = np.random.RandomState(bits)
    x = (rng.standard_normal(6000) * 10.0 ** rng.randint(-30, 30, size=6000)).astype(FLT[bits])
    x[::11] = x[rng.randint(0, x.size, size=x[::11].size)]   # duplicates
    x[:3] = [np.inf, -np.inf, np.finfo(FLT[bits]).tiny]
    x[x == 0] = 1.0                                 # no zeros: numpy takes -0 == +0
    vals = np.arange(x.size, dtype=UINT[bits])
    k, v = oracle.sort_ordered(x.view(UINT[bits]), vals, "float")
    order = np.argsort(x, kind="stable")
    assert np.array_equal(k.view(FLT[bits]), x[order])
    assert np.array_equal(v, order.astype(UINT[bits]))


@pytest.mark.parametrize("bits", [32, 64])
def test_float_total_order_of_special_values(bits):
    """IEEE 754 totalOrder: -NaN < -inf < negatives < -0 < +0 < positives <
    +inf < +NaN (the list below, written out by hand)."""
    t, u = FLT[bits], UINT[bits]
    want = np.array([-np.inf, -1.5, -np.finfo(t).tiny, -0.0, 0.0, np.finfo(t).tiny, 2.0,
                     np.inf], dtype=t)
    neg_nan = np.array([np.nan], dtype=t)
    neg_nan.view(u)[0] |= u(1) << u(bits - 1)
    pos_nan = np.array([np.nan], dtype=t)
    pos_nan.view(u)[0] &= ~(u(1) << u(bits - 1))
    want = np.concatenate([neg_nan, want, pos_nan])
    for seed in range(5):
        perm = np.random.RandomState(seed).permutation(want.size)
        k, _ = oracle.sort_ordered(want[perm].view(u), None, "float")
        assert np.array_equal(k, want.view(u))
        kd, _ = oracle.sort_ordered(want[perm].view(u), None, "float", descending=True)
        assert np.array_equal(kd, want.view(u)[::-1])


@pytest.mark.parametrize("order", ["unsigned", "signed"])
def test_descending_is_the_stable_descending_sort(order):
    """Brute force: every arrangement of a small multiset; the definitional
    stable descending sort orders by (-value, input index)."""
    base = [0, 1, 1, 2**31, 2**32 - 1, 5, 2**31 - 1]
    for perm in itertools.permutations(range(len(base))):
        x = np.array([base[i] for i in perm], dtype=np.uint32)
        vals = np.arange(x.size, dtype=np.uint32)
        k, v = oracle.sort_ordered(x, vals, order, descending=True)
        value = [int(e) if order == "unsigned" else int(np.uint32(e).view(np.int32)) for e in x]
        want = sorted(range(x.size), key=lambda i: (-value[i], i))
        assert v.tolist() == want
        assert k.tolist() == [int(x[i]) for i in want]


@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("order", oracle.ORDERS)
@pytest.mark.parametrize("descending", [False, True])
def test_maps_are_bijections(bits, order, descending):
    rng = np.random.RandomState(1)
    u = UINT[bits]
    x = rng.randint(0, 2**32, size=4000).astype(u)
    if bits == 64:
        x = (x << u(32)) | rng.randint(0, 2**32, size=4000).astype(u)
    x[:4] = [0, u(1) << u(bits - 1), ~u(0), (u(1) << u(bits - 1)) - u(1)]
    m = oracle.order_key(x, order, descending)
    assert np.array_equal(oracle.order_unkey(m, order, descending), x)
    assert np.unique(m).size == np.unique(x).size


def test_pins_have_teeth():
    """A plausible mistake in the float map (negatives not complemented, only
    the sign bit flipped) fails the numpy comparison above."""
    x = np.array([-3.0, -1.0, 2.0, -2.0], dtype=np.float32)
    sign = np.uint32(1 << 31)
    wrong = x.view(np.uint32) ^ sign
    k, _ = oracle.sort(wrong)
    got = (k ^ sign).view(np.float32)
    assert not np.array_equal(got, np.sort(x))


def test_segmented_orders_equal_per_segment_sorts():
    x = ints(32, 3000, 7)
    off = np.array([0, 10, 10, 900, 2999, 3000], dtype=np.uint64)
    vals = np.arange(3000, dtype=np.uint32)
    k, v = oracle.segmented_sort_ordered(x.view(np.uint32), vals, off, "signed", True)
    for a, b in zip(off[:-1], off[1:]):
        a, b = int(a), int(b)
        ks, vs = oracle.sort_ordered(x.view(np.uint32)[a:b], vals[a:b], "signed", True)
        assert np.array_equal(k[a:b], ks) and np.array_equal(v[a:b], vs)
