"""GPU parity: the HIP radix sort (through the C-ABI) against the CPU oracle,
bit-exact, on seeded inputs of the six distributions; plus the exact O(n)
stable-sort certificate at the full benchmark sizes, and the edge cases
(ragged tails, tile boundaries, in-place, unaligned starts, skipped passes)."""
import os

import numpy as np
import pytest
import torch

import datagen
from tests.certify import certify_stable_sort, certify_sorted_keys

pytestmark = pytest.mark.gpu

TILE = 16384  # elements per tile of the digit-pass kernel (8192 for 64-bit pairs)
# every path: one-workgroup LDS sorts (caps 4096 and 16384/8192), one tile,
# several tiles with a ragged tail, the paper's 2^n + 2^(n-1) lengths
SIZES = [1, 2, 3, 63, 64, 65, 255, 256, 4095, 4096, 4097, 8191, 8192, 8193, TILE - 1, TILE,
         TILE + 1, 3 * TILE + 17, (1 << 15) + (1 << 14), 100003]


@pytest.fixture(scope="module")
def rs():
    import paper_1511_03404_amd as rs
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    rs.lib()  # raises if librs.so is missing: there is no fallback
    return rs


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


def gpu_sort(rs, keys, vals=None, in_place=False):
    kd = dev(keys)
    if vals is None:
        out = rs.sort_keys(kd, out=kd if in_place else None)
        torch.cuda.synchronize()
        return host(out), None
    vd = dev(vals)
    if in_place:
        ko, vo = rs.sort_pairs(kd, vd, kd, vd)
    else:
        ko, vo = rs.sort_pairs(kd, vd)
    torch.cuda.synchronize()
    return host(ko), host(vo)


def test_native_library_is_loaded(rs):
    import paper_1511_03404_amd as pkg
    assert os.path.dirname(pkg.LIB_PATH) == os.path.dirname(os.path.abspath(pkg.__file__))
    maps = open("/proc/self/maps").read()
    assert pkg.LIB_PATH in maps


@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("pairs", [False, True])
@pytest.mark.parametrize("dist", datagen.DISTRIBUTIONS)
def test_parity_ragged_sizes(rs, oracle_lib, bits, pairs, dist):
    for n in SIZES:
        print(f"case bits={bits} pairs={pairs} dist={dist} n={n}", flush=True)
        keys = datagen.keys(dist, n, bits, seed=n)
        vals = datagen.values(n, bits) if pairs else None
        ok, ov = oracle_lib.sort(keys, vals)
        gk, gv = gpu_sort(rs, keys, vals)
        assert np.array_equal(gk, ok), f"keys differ at n={n}"
        if pairs:
            assert np.array_equal(gv, ov), f"values differ at n={n}"


def test_empty(rs):
    for dt in (torch.uint32, torch.uint64):
        k = torch.empty(0, dtype=dt, device="cuda")
        assert rs.sort_keys(k).numel() == 0
        a, b = rs.sort_pairs(k, torch.empty(0, dtype=dt, device="cuda"))
        assert a.numel() == 0 and b.numel() == 0


def test_small_config_uniform_2p20(rs, oracle_lib):
    """2^20 uniform 32-bit keys from MT19937 seed 1."""
    keys = datagen.keys("uniform", 1 << 20, 32, seed=1)
    ok, _ = oracle_lib.sort(keys)
    gk, _ = gpu_sort(rs, keys)
    assert np.array_equal(gk, ok)


@pytest.mark.parametrize("dist", datagen.DISTRIBUTIONS)
def test_full_size_u32_pairs(rs, oracle_lib, dist):
    """2^26 32-bit pairs, value = input index: exact certificate and the oracle."""
    n = 1 << 26
    print(f"case u32 pairs n=2^26 dist={dist}", flush=True)
    keys = datagen.keys(dist, n, 32, seed=1)
    vals = datagen.values(n, 32)
    gk, gv = gpu_sort(rs, keys, vals)
    assert certify_stable_sort(keys, gk, gv) is None
    ok, ov = oracle_lib.sort(keys, vals)
    assert np.array_equal(gk, ok) and np.array_equal(gv, ov)


@pytest.mark.parametrize("dist,n", [("uniform", 1 << 26), ("bucket", 1 << 26),
                                    ("gaussian", (1 << 26) + 12345), ("zero", 1 << 26)])
def test_full_size_u32_keys(rs, oracle_lib, dist, n):
    """32-bit keys alone from 2^26 on: tiles of 1024 x 24 claimed in arrival
    order (the built-in choice there), against the oracle."""
    print(f"case u32 keys n={n} dist={dist}", flush=True)
    keys = datagen.keys(dist, n, 32, seed=2)
    gk, _ = gpu_sort(rs, keys)
    assert certify_sorted_keys(keys, gk) is None
    ok, _ = oracle_lib.sort(keys)
    assert np.array_equal(gk, ok)


@pytest.mark.parametrize("pairs", [False, True])
@pytest.mark.parametrize("dist", datagen.DISTRIBUTIONS)
def test_full_size_u64(rs, oracle_lib, pairs, dist):
    """2^25 64-bit keys (random high words), alone and with 64-bit values."""
    n = 1 << 25
    print(f"case u64 pairs={pairs} n=2^25 dist={dist}", flush=True)
    keys = datagen.keys(dist, n, 64, seed=1)
    vals = datagen.values(n, 64) if pairs else None
    gk, gv = gpu_sort(rs, keys, vals)
    if pairs:
        assert certify_stable_sort(keys, gk, gv) is None
    else:
        assert certify_sorted_keys(keys, gk) is None
    ok, ov = oracle_lib.sort(keys, vals)
    assert np.array_equal(gk, ok)
    if pairs:
        assert np.array_equal(gv, ov)


@pytest.mark.parametrize("n", [3000, 3 * TILE + 5])
@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("mask_bits", [0, 8, 24, None])
@pytest.mark.parametrize("pairs", [False, True])
def test_in_place_and_skipped_passes(rs, oracle_lib, n, bits, mask_bits, pairs):
    """In-place sorts with 0, 1, 3 and all moving passes (skipped passes
    change which buffer the result lands in), on the one-workgroup path and
    the multi-tile path."""
    keys = datagen.keys("uniform", n, bits, seed=7)
    if mask_bits is not None:
        keys = keys & keys.dtype.type((1 << mask_bits) - 1)
    vals = datagen.values(n, bits) if pairs else None
    ok, ov = oracle_lib.sort(keys, vals)
    for in_place in (False, True):
        gk, gv = gpu_sort(rs, keys, vals, in_place=in_place)
        assert np.array_equal(gk, ok)
        if pairs:
            assert np.array_equal(gv, ov)


@pytest.mark.parametrize("bits", [32, 64])
def test_unaligned_start_and_arbitrary_values(rs, oracle_lib, bits):
    """Arrays that start one element past a 16-byte boundary; values that are
    not the index."""
    n = 2 * TILE + 77
    keys = datagen.keys("bucket", n, bits, seed=3)
    vals = datagen.keys("uniform", n, bits, seed=4)
    kbuf = dev(np.concatenate([keys[:1], keys]))
    vbuf = dev(np.concatenate([vals[:1], vals]))
    ko = torch.empty(n + 1, dtype=kbuf.dtype, device="cuda")
    vo = torch.empty(n + 1, dtype=vbuf.dtype, device="cuda")
    rs.sort_pairs(kbuf[1:], vbuf[1:], ko[1:], vo[1:])
    torch.cuda.synchronize()
    ok, ov = oracle_lib.sort(keys, vals)
    assert np.array_equal(host(ko[1:]), ok) and np.array_equal(host(vo[1:]), ov)


def test_signed_tensors_sort_as_unsigned(rs, oracle_lib):
    keys = datagen.keys("uniform", 5000, 32, seed=2)
    t = dev(keys).view(torch.int32)
    out = rs.sort_keys(t)
    torch.cuda.synchronize()
    ok, _ = oracle_lib.sort(keys)
    assert np.array_equal(host(out.view(torch.uint32)), ok)


def test_repeatable(rs):
    keys = datagen.keys("gaussian", 1 << 20, 32, seed=5)
    vals = datagen.values(1 << 20)
    a = gpu_sort(rs, keys, vals)
    b = gpu_sort(rs, keys, vals)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_caller_workspace_and_streams(rs, oracle_lib):
    """A caller-provided workspace, reused across calls on a side stream."""
    n = 50000
    ctx = rs.context(0)
    ws = torch.empty(ctx.workspace_bytes(64, True, n), dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for seed in (1, 2, 3):
            keys = datagen.keys("uniform", n, 64, seed=seed)
            vals = datagen.values(n, 64)
            ko, vo = rs.sort_pairs(dev(keys), dev(vals), workspace=ws)
            s.synchronize()
            ok, ov = oracle_lib.sort(keys, vals)
            assert np.array_equal(host(ko), ok) and np.array_equal(host(vo), ov)


@pytest.mark.parametrize("n", [1024 * TILE, 1024 * TILE + 1])
def test_claim_modes_at_the_limit(rs, oracle_lib, n):
    """32-bit pairs in 1024 tiles (claimed in arrival order) and in 1025
    (claimed in XCD groups): both equal the oracle."""
    print(f"case u32 pairs n={n}", flush=True)
    keys = datagen.keys("uniform", n, 32, seed=7)
    vals = datagen.values(n, 32)
    gk, gv = gpu_sort(rs, keys, vals)
    ok, ov = oracle_lib.sort(keys, vals)
    assert np.array_equal(gk, ok) and np.array_equal(gv, ov)


def test_concurrent_sorts_on_streams(rs, oracle_lib):
    """Sorts of several kinds and sizes enqueued on four streams with no
    synchronisation between them run on the device at the same time: passes
    that claim tiles in arrival order (up to 1024 tiles, and 32-bit keys
    alone at any size) beside passes that claim them in XCD groups (1025
    tiles), each with its own workspace.  Every result equals the oracle's
    and every workspace reports no device error."""
    cases = [(32, False, 1 << 17), (32, True, 1 << 20), (64, False, 1 << 19),
             (32, True, 1024 * TILE + 5), (32, False, 1 << 25), (64, True, 1 << 18),
             (32, True, 3 * TILE + 1), (64, False, (1 << 21) + 77)]
    ctx = rs.context(0)
    streams = [torch.cuda.Stream() for _ in range(4)]
    jobs = []
    for i, (bits, pairs, n) in enumerate(cases):
        keys = datagen.keys("uniform", n, bits, seed=100 + i)
        vals = datagen.values(n, bits) if pairs else None
        kd = dev(keys)
        vd = dev(vals) if pairs else None
        ws = torch.empty(ctx.workspace_bytes(bits, pairs, n), dtype=torch.uint8, device="cuda")
        jobs.append((bits, pairs, n, keys, vals, kd, vd, ws))
    torch.cuda.synchronize()
    outs = []
    for i, (bits, pairs, n, keys, vals, kd, vd, ws) in enumerate(jobs):
        print(f"case stream={i % 4} bits={bits} pairs={pairs} n={n}", flush=True)
        with torch.cuda.stream(streams[i % 4]):
            if pairs:
                outs.append(rs.sort_pairs(kd, vd, workspace=ws))
            else:
                outs.append((rs.sort_keys(kd, workspace=ws), None))
    torch.cuda.synchronize()
    for (bits, pairs, n, keys, vals, kd, vd, ws), (ko, vo) in zip(jobs, outs):
        assert ctx.status(ws) == rs.RS_OK, (bits, pairs, n)
        ok, ov = oracle_lib.sort(keys, vals)
        assert np.array_equal(host(ko), ok), (bits, pairs, n)
        if pairs:
            assert np.array_equal(host(vo), ov), (bits, pairs, n)


@pytest.mark.parametrize("n", [3000, 3 * TILE + 5])
@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("mask_bits", [0, 8, 16, 24, None])
@pytest.mark.parametrize("aliased", ["keys", "values"])
def test_mixed_in_place_pairs(rs, oracle_lib, n, bits, mask_bits, aliased):
    """Only one of the two arrays sorted in place: keys_out is keys_in with a
    separate values_out, or the reverse.  With every pass skipped (mask 0)
    the array that is not in place must still receive the input; with odd
    and even numbers of moving passes the result lands in the same place."""
    print(f"case mixed in-place n={n} bits={bits} mask={mask_bits} aliased={aliased}",
          flush=True)
    keys = datagen.keys("uniform", n, bits, seed=9)
    if mask_bits is not None:
        keys = keys & keys.dtype.type((1 << mask_bits) - 1)
    vals = datagen.values(n, bits)
    ok, ov = oracle_lib.sort(keys, vals)
    kd, vd = dev(keys), dev(vals)
    if aliased == "keys":
        vo = torch.full_like(vd, 7)
        ko, vo = rs.sort_pairs(kd, vd, kd, vo)
    else:
        ko = torch.full_like(kd, 7)
        ko, vo = rs.sort_pairs(kd, vd, ko, vd)
    torch.cuda.synchronize()
    assert np.array_equal(host(ko), ok) and np.array_equal(host(vo), ov)


@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("pairs", [False, True])
def test_device_status_is_ok_after_a_sort(rs, bits, pairs):
    """The status query reads RS_OK after working sorts, small and large, with
    a caller workspace and with the context's own scratch."""
    ctx = rs.context(0)
    for n in (1000, 3 * TILE + 5):
        keys = dev(datagen.keys("uniform", n, bits, seed=n))
        vals = dev(datagen.values(n, bits)) if pairs else None
        ws = torch.empty(ctx.workspace_bytes(bits, pairs, n), dtype=torch.uint8, device="cuda")
        if pairs:
            rs.sort_pairs(keys, vals, workspace=ws)
        else:
            rs.sort_keys(keys, workspace=ws)
        assert ctx.status(ws) == rs.RS_OK
        f = rs.lib().rs_sort_pairs_u32 if bits == 32 else rs.lib().rs_sort_pairs_u64
        if pairs:
            ko, vo = torch.empty_like(keys), torch.empty_like(vals)
            rs._check(f(ctx.handle, rs._ptr(keys), rs._ptr(vals), rs._ptr(ko), rs._ptr(vo), n,
                        None, 0, rs._stream(0)))
            assert ctx.status(None) == rs.RS_OK


def test_device_copy_is_exact(rs):
    """The copy that measures the bench's copy ceiling copies exactly,
    including sizes that leave the last workgroup partly idle."""
    for nbytes in (16, 4096 * 16 + 48, (1 << 26) + 16 * 7):
        src = torch.randint(-(1 << 31), 1 << 31, (nbytes // 4,), dtype=torch.int64,
                            device="cuda").to(torch.int32)
        dst = torch.zeros_like(src)
        rs.device_copy(src, dst)
        torch.cuda.synchronize()
        assert torch.equal(src, dst), nbytes
