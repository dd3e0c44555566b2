"""GPU parity of the key orders (signed, float total order, descending): the
maps are fused into the first and last moving pass, the one-workgroup sorts,
the odd-pass copy and the segmented sort, so every path is run in every order
and compared bit for bit with the oracle's sort of the mapped keys."""
import numpy as np
import pytest
import torch

import datagen

pytestmark = pytest.mark.gpu

TILE = 16384
SIZES = [1, 2, 100, 4096, 5000, 16384, 16385, 3 * TILE + 17, 100003]
ORDERS = [("signed", False), ("float", False), ("unsigned", True), ("signed", True),
          ("float", True)]
KINDS = [(32, False), (32, True), (64, False), (64, True)]
UINT = {32: np.uint32, 64: np.uint64}
FLT = {32: np.float32, 64: np.float64}


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


def float_specials(bits):
    """Bit patterns of -NaN, -inf, -max, -1, -denormal, -0, +0, +denormal, 1,
    max, inf, NaN (both NaN signs, two payloads each)."""
    t, u = FLT[bits], UINT[bits]
    fi = np.finfo(t)
    x = np.array([-np.inf, -fi.max, -1.0, -fi.tiny / 4, -0.0, 0.0, fi.tiny / 4, 1.0, fi.max,
                  np.inf, np.nan], dtype=t).view(u)
    sign = u(1) << u(bits - 1)
    nan = x[-1]
    return np.concatenate([x, [nan | sign, nan | u(1), (nan | u(1)) | sign]]).astype(u)


def order_keys(dist, n, bits, seed, order):
    k = datagen.keys(dist, n, bits, seed=seed)
    if order == "float" and dist == "gaussian":
        # finite floats of both signs and many magnitudes, with duplicates
        rng = np.random.RandomState(seed)
        f = rng.standard_normal(n) * 10.0 ** rng.randint(-8, 8, size=n)
        f[rng.randint(0, n, size=n // 8)] = f[rng.randint(0, n, size=n // 8)]
        k = f.astype(FLT[bits]).view(UINT[bits])
    if n >= 64:
        sp = float_specials(bits)
        k[: sp.size] = sp
        k[n // 2: n // 2 + sp.size] = sp[::-1]
    return np.ascontiguousarray(k)


def run_sort(rs, keys, vals, order, desc, in_place=False):
    kd = dev(keys)
    if vals is None:
        out = rs.sort_keys(kd, kd if in_place else None, order=order, descending=desc)
        torch.cuda.synchronize()
        return host(out), None
    vd = dev(vals)
    ko, vo = rs.sort_pairs(kd, vd, kd if in_place else None, vd if in_place else None,
                           order=order, descending=desc)
    torch.cuda.synchronize()
    return host(ko), host(vo)


@pytest.mark.parametrize("order,desc", ORDERS)
@pytest.mark.parametrize("bits,pairs", KINDS)
def test_orders_match_oracle(rs, oracle_lib, bits, pairs, order, desc):
    for n in SIZES:
        for dist in ("uniform", "gaussian", "bucket"):
            print(f"case bits={bits} pairs={pairs} order={order} desc={desc} n={n} {dist}",
                  flush=True)
            keys = order_keys(dist, n, bits, n + bits, order)
            vals = datagen.values(n, bits) if pairs else None
            ok, ov = oracle_lib.sort_ordered(keys, vals, order, desc)
            gk, gv = run_sort(rs, keys, vals, order, desc)
            assert np.array_equal(gk, ok), f"keys differ n={n} {dist}"
            if pairs:
                assert np.array_equal(gv, ov), f"values differ n={n} {dist}"


@pytest.mark.parametrize("order,desc", [("signed", True), ("float", False)])
@pytest.mark.parametrize("bits,pairs,tile", [(32, True, TILE), (64, False, TILE),
                                             (64, True, TILE // 2)])
def test_orders_with_grouped_claims(rs, oracle_lib, bits, pairs, tile, order, desc):
    """Sorts of 1025 tiles claim them in XCD groups (smaller ones in arrival
    order): the maps of the first and last pass on that path too."""
    n = 1024 * tile + 1
    print(f"case bits={bits} pairs={pairs} order={order} desc={desc} n={n}", flush=True)
    keys = order_keys("gaussian", n, bits, 11, order)
    vals = datagen.values(n, bits) if pairs else None
    ok, ov = oracle_lib.sort_ordered(keys, vals, order, desc)
    gk, gv = run_sort(rs, keys, vals, order, desc)
    assert np.array_equal(gk, ok)
    if pairs:
        assert np.array_equal(gv, ov)


@pytest.mark.parametrize("order,desc", ORDERS)
@pytest.mark.parametrize("bits,pairs", KINDS)
def test_orders_in_place_and_skipped_passes(rs, oracle_lib, bits, pairs, order, desc):
    """In place and out of place, with low digits all equal (skipped passes,
    odd pass counts ending in the scratch copy), with a single moving pass,
    and with every key equal (no pass moves data)."""
    n = 2 * TILE + 5
    base = datagen.keys("uniform", n, bits, seed=11)
    u = UINT[bits]
    cases = {
        "low zero": (base >> u(9)) << u(9),
        "one digit": base & u(0xFF),
        "top digit": (base >> u(bits - 8)) << u(bits - 8),
        "all equal": np.full(n, base[0], dtype=u),
    }
    for name, keys in cases.items():
        for in_place in (False, True):
            print(f"case bits={bits} pairs={pairs} order={order} desc={desc} {name} "
                  f"in_place={in_place}", flush=True)
            vals = datagen.values(n, bits) if pairs else None
            ok, ov = oracle_lib.sort_ordered(keys, vals, order, desc)
            gk, gv = run_sort(rs, keys, vals, order, desc, in_place)
            assert np.array_equal(gk, ok), name
            if pairs:
                assert np.array_equal(gv, ov), name


@pytest.mark.parametrize("order,desc", ORDERS)
@pytest.mark.parametrize("bits,pairs", [(32, True), (64, False), (64, True)])
def test_orders_segmented(rs, oracle_lib, bits, pairs, order, desc):
    sizes = [17, 5000, 0, 16385, 1, 3 * TILE + 5, 70001, 2, 12000, 64]
    off = np.zeros(len(sizes) + 1, dtype=np.uint64)
    off[1:] = np.cumsum(sizes)
    total = int(off[-1])
    keys = order_keys("uniform", total, bits, 5, order)
    vals = datagen.values(total, bits) if pairs else None
    ok, ov = oracle_lib.segmented_sort_ordered(keys, vals, off, order, desc)
    offd = dev(off.view(np.int64))
    for in_place in (False, True):
        print(f"case segmented bits={bits} pairs={pairs} order={order} desc={desc} "
              f"in_place={in_place}", flush=True)
        kd = dev(keys)
        vd = dev(vals) if pairs else None
        ko, vo = rs.segmented_sort(kd, vd, offd, kd if in_place else None,
                                   vd if in_place else None, order=order, descending=desc)
        torch.cuda.synchronize()
        assert np.array_equal(host(ko), ok)
        if pairs:
            assert np.array_equal(host(vo), ov)


@pytest.mark.parametrize("dtype", [torch.int32, torch.int64])
@pytest.mark.parametrize("desc", [False, True])
def test_signed_tensors_match_torch_stable_sort(rs, dtype, desc):
    """An independent check on the device: torch's stable sort of signed
    integer tensors gives the same keys and the same permutation."""
    n = 3 * TILE + 17
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    lim = 1 << 31 if dtype == torch.int32 else 1 << 62
    k = torch.randint(-lim, lim, (n,), dtype=torch.int64, device="cuda", generator=g).to(dtype)
    k[::5] = k[::5] % 100  # duplicates
    v = torch.arange(n, dtype=dtype, device="cuda")
    ko, vo = rs.sort_pairs(k, v, order="signed", descending=desc)
    ref_k, ref_i = torch.sort(k, stable=True, descending=desc)
    torch.cuda.synchronize()
    assert torch.equal(ko, ref_k)
    assert torch.equal(vo, ref_i.to(dtype))


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_float_tensors_default_to_total_order(rs, oracle_lib, dtype):
    """A float tensor sorts in IEEE total order without an explicit order;
    on finite values without signed zeros that equals torch's stable sort."""
    n = 100003
    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    k = torch.randn(n, dtype=dtype, device="cuda", generator=g) * 1e3
    k[k == 0] = 1.0
    out = rs.sort_keys(k)
    ref, _ = torch.sort(k, stable=True)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    bits = 32 if dtype == torch.float32 else 64
    raw = host(k).view(UINT[bits])
    ok, _ = oracle_lib.sort_ordered(raw, None, "float")
    assert np.array_equal(host(out).view(UINT[bits]), ok)
